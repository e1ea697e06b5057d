"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU,
in a temporary directory), builds it, points the oracle module at the copy and
runs the pin checks of test_oracle_pins.py; at least one must fail.  The
planted mistakes never index outside the arrays the checks pass.

The error metrics (the parity gate, written in Python in the oracle package)
are mutated the same way: one mistake in a copy of the package's source,
executed as a separate module whose metric functions replace the oracle's,
and the pins of test_oracle_metrics.py must catch it.
"""
import os
import subprocess
import types

import pytest

import oracle
import test_oracle_metrics as metric_pins
import test_oracle_pins as pins
import test_oracle_sell_runs as sell_pins

# (name, text in dose_oracle.c, replacement)
MUTANTS = [
    ("dropped last term of a row",
     "for (int64_t k = 0; k < n; ++k) acc += (double)dec[k] * (double)x[col[k]];",
     "for (int64_t k = 0; k + 1 < n; ++k) acc += (double)dec[k] * (double)x[col[k]];"),
    ("x indexed by entry instead of column",
     "acc += (double)dec[k] * (double)x[col[k]];",
     "acc += (double)dec[k] * (double)x[col[k] > 0 ? col[k] - 1 : 0];"),
    ("subtracted term",
     "acc += (double)dec[k] * (double)x[col[k]];",
     "acc -= (double)dec[k] * (double)x[col[k]];"),
    ("product rounded to FP32",
     "acc += (double)dec[k] * (double)x[col[k]];",
     "acc += (double)(dec[k] * x[col[k]]);"),
    ("adjoint weight of the wrong row",
     "g[col[k]] += (double)dec[k] * (double)v[i];",
     "g[col[k]] += (double)dec[k] * (double)v[i > 0 ? i - 1 : 0];"),
    ("binary16 truncation instead of nearest-even",
     "double q = nearbyint(ldexp(a, 10 - E)); /* 1024 <= q <= 2048 */",
     "double q = floor(ldexp(a, 10 - E)); /* 1024 <= q <= 2048 */"),
    ("binary16 exponent bias 14",
     "return (uint16_t)(sign | (uint16_t)((E + 15) << 10) | (uint16_t)(q - 1024.0));",
     "return (uint16_t)(sign | (uint16_t)((E + 14) << 10) | (uint16_t)(q - 1024.0));"),
    ("binary16 subnormals flushed",
     "double q = nearbyint(ldexp(a, 24));\n    return (uint16_t)(sign | (uint16_t)q);",
     "return sign;"),
    ("bfloat16 ties away from zero",
     "double q = nearbyint(ldexp(a, 7 - E)); /* 128 <= q <= 256 */",
     "double q = round(ldexp(a, 7 - E)); /* 128 <= q <= 256 */"),
    ("E4M3 without saturation of the NaN code",
     "if (code > 0x7Eu) code = 0x7Eu;",
     "if (code > 0x7Fu) code = 0x7Fu;"),
    ("E4M3 exponent bias 8",
     "mag = ldexp((double)(8 + m), E - 10);",
     "mag = ldexp((double)(8 + m), E - 11);"),
    ("row scale against 480",
     "float s = amax / 448.0f;",
     "float s = amax / 480.0f;"),
    ("objective residual with the wrong sign",
     "double r = d[v] - (double)p[v];",
     "double r = d[v] + (double)p[v];"),
    ("seed without the factor 2",
     "out[v] = 2.0 * (double)w[v] * (d[v] - (double)p[v]);",
     "out[v] = (double)w[v] * (d[v] - (double)p[v]);"),
    ("transpose lists rows in descending order",
     "  for (int64_t i = 0; i < n_rows; ++i)\n    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {\n      int64_t j = col[k];",
     "  for (int64_t i = n_rows - 1; i >= 0; --i)\n    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {\n      int64_t j = col[k];"),
    ("beam sum skips the last beam",
     "for (int32_t b = 0; b < n_beams; ++b) s += part[(int64_t)b * n + v];",
     "for (int32_t b = 0; b + 1 < n_beams; ++b) s += part[(int64_t)b * n + v];"),
    ("beam sum with (voxel, beam) order transposed",
     "for (int32_t b = 0; b < n_beams; ++b) s += part[(int64_t)b * n + v];",
     "for (int32_t b = 0; b < n_beams; ++b) s += part[v * n_beams + b];"),
    ("worst case takes the last of tied scenarios",
     "    if (f[s] > w) {",
     "    if (f[s] >= w) {"),
    ("expectation ignores the probabilities",
     "for (int32_t s = 0; s < n_scen; ++s) e += prob[s] * f[s];",
     "for (int32_t s = 0; s < n_scen; ++s) e += f[s] / n_scen;"),
    ("worst-case weight on the last of tied scenarios",
     "      if (f[s] > f[a]) a = s;",
     "      if (f[s] >= f[a]) a = s;"),
    ("expectation weights ignore the probabilities",
     "c[s] = prob ? prob[s] : 1.0 / (double)n_scen;",
     "c[s] = 1.0 / (double)n_scen;"),
    ("worst-case weight on the least scenario",
     "      if (f[s] > f[a]) a = s;",
     "      if (f[s] < f[a]) a = s;"),
    ("SELL sort ascending",
     "while (q > w0 && row_ptr[perm[q - 1] + 1] - row_ptr[perm[q - 1]] < len) {",
     "while (q > w0 && row_ptr[perm[q - 1] + 1] - row_ptr[perm[q - 1]] > len) {"),
    ("SELL sort not stable",
     "while (q > w0 && row_ptr[perm[q - 1] + 1] - row_ptr[perm[q - 1]] < len) {",
     "while (q > w0 && row_ptr[perm[q - 1] + 1] - row_ptr[perm[q - 1]] <= len) {"),
    ("SELL sort across windows",
     "      while (q > w0 && row_ptr",
     "      while (q > 0 && row_ptr"),
    ("SELL width misses the chunk's last row",
     "for (int64_t i = c * C; i < (c + 1) * C && i < n_rows; ++i) {",
     "for (int64_t i = c * C; i + 1 < (c + 1) * C && i < n_rows; ++i) {"),
    ("SELL pack row-major inside a chunk",
     "int64_t slot = off + j * C + i, pos = c * C + i;",
     "int64_t slot = off + i * width[c] + j, pos = c * C + i;"),
    ("SELL product stored at the sorted position",
     "      y[perm[c * C + i]] = acc;",
     "      y[c * C + i] = acc;"),
    ("runs: a break not detected",
     "if (k > row_ptr[i] && col[k] == col[k - 1] + 1) {",
     "if (k > row_ptr[i] && col[k] >= col[k - 1] + 1) {"),
    ("runs continue across rows",
     "if (k > row_ptr[i] && col[k] == col[k - 1] + 1) {",
     "if (k > 0 && col[k] == col[k - 1] + 1) {"),
    ("runs decode off by one",
     "for (int32_t t = 0; t < len[r]; ++t) col[k++] = start[r] + t;",
     "for (int32_t t = 0; t < len[r]; ++t) col[k++] = start[r] + t + (t > 0);"),
]

CHECKS = [
    pins.test_fp16_encode_matches_numpy_on_ties_and_subnormals,
    pins.test_fp16_decode_exhaustive,
    pins.test_bf16_encode_matches_torch,
    pins.test_e4m3_decode_exhaustive_matches_torch,
    pins.test_e4m3_saturates_at_448,
    pins.test_e4m3_row_scale_closed_forms,
    pins.test_decode_matrix_fp8_error_bound,
    lambda: pins.test_spmv_bit_exact_vs_dense_brute_force(0),
    pins.test_spmv_hand_worked_example,
    pins.test_spmv_T_matches_dense_transpose_and_adjointness,
    pins.test_transpose_structure,
    pins.test_objective_closed_form_and_seed,
    pins.test_gradient_matches_central_finite_differences,
    pins.test_beam_sum_equals_product_with_side_by_side_beams,
    pins.test_beam_sum_is_the_correctly_rounded_sum_of_few_terms,
    pins.test_robust_closed_forms,
    pins.test_robust_expectation_vs_exact_fractions,
    pins.test_robust_weights_are_the_derivatives_of_the_robust_forms,
    sell_pins.test_sell_layout_hand_worked_example,
    sell_pins.test_sell_layout_ties_keep_row_order,
    sell_pins.test_sell_layout_is_windowed_stable_argsort,
    sell_pins.test_sell_pack_holds_every_entry_once_and_product_equals_csr_bitwise,
    sell_pins.test_runs_hand_worked_example,
    sell_pins.test_runs_count_maximality_and_decode_on_dose_rows,
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, old, new, tmp_path, monkeypatch):
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, f"mutation site not found: {name}"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
                           "-std=c11", "-o", str(so), str(path), "-lm"])
    monkeypatch.setattr(oracle, "_lib", oracle.load_library(str(so)))
    caught = []
    for check in CHECKS:
        try:
            check()
        except AssertionError:
            caught.append(getattr(check, "__name__", "lambda"))
    assert caught, f"no pin caught: {name}"


def test_unmutated_copy_passes_every_check(tmp_path, monkeypatch):
    so = tmp_path / "libcopy.so"
    subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
                           "-std=c11", "-o", str(so), oracle._SRC, "-lm"])
    monkeypatch.setattr(oracle, "_lib", oracle.load_library(str(so)))
    for check in CHECKS:
        check()
    assert os.path.exists(so)


# (name, function, text in that function of oracle/__init__.py, replacement)
METRIC_MUTANTS = [
    ("relative error divided by the result",
     "max_rel_err", "/ np.abs(y_ref[keep])", "/ np.abs(y[keep])"),
    ("relative error: mean instead of maximum",
     "max_rel_err", "return float(np.max(rel))", "return float(np.mean(rel))"),
    ("relative error: zero-reference rule inverted",
     "max_rel_err", "if np.any(y[ref_zero] != 0.0):", "if np.any(y[ref_zero] == 0.0):"),
    ("relative error: zero-reference rule dropped",
     "max_rel_err", "if np.any(y[ref_zero] != 0.0):", "if False:"),
    ("relative error: signed difference",
     "max_rel_err", "np.abs(y[keep] - y_ref[keep])", "(y[keep] - y_ref[keep])"),
    ("relative error: non-finite results pass",
     "max_rel_err", "if not np.all(np.isfinite(y)):", "if False:"),
    ("scaled error divided by the reference",
     "max_scaled_err", "/ scale[held]", "/ np.abs(y_ref[held])"),
    ("scaled error: mean instead of maximum",
     "max_scaled_err", "return float(np.max(scaled))", "return float(np.mean(scaled))"),
    ("scaled error: zero-scale rule inverted",
     "max_scaled_err", "if np.any(y[scale_zero] != 0.0):", "if np.any(y[scale_zero] == 0.0):"),
    ("scaled error: signed difference",
     "max_scaled_err", "np.abs(y[held] - y_ref[held])", "(y[held] - y_ref[held])"),
    ("scaled error: non-finite results pass",
     "max_scaled_err", "if not np.all(np.isfinite(y)):", "if False:"),
]


def _function_span(src, name):
    start = src.index(f"def {name}(")
    end = src.find("\ndef ", start + 1)
    return start, (len(src) if end < 0 else end)


def _mutated_module(src):
    mod = types.ModuleType("oracle_mutant")
    mod.__file__ = oracle.__file__
    exec(compile(src, "oracle_mutant", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name,func,old,new", METRIC_MUTANTS, ids=[m[0] for m in METRIC_MUTANTS])
def test_metric_pins_catch_planted_mistake(name, func, old, new, monkeypatch):
    src = open(oracle.__file__).read()
    a, b = _function_span(src, func)
    body = src[a:b]
    assert body.count(old) == 1, f"mutation site not found: {name}"
    mod = _mutated_module(src[:a] + body.replace(old, new) + src[b:])
    monkeypatch.setattr(oracle, func, getattr(mod, func))
    caught = []
    for check in metric_pins.CHECKS:
        try:
            check()
        except AssertionError:
            caught.append(check.__name__)
    assert caught, f"no pin caught: {name}"


def test_unmutated_metrics_pass_every_check(monkeypatch):
    mod = _mutated_module(open(oracle.__file__).read())
    monkeypatch.setattr(oracle, "max_rel_err", mod.max_rel_err)
    monkeypatch.setattr(oracle, "max_scaled_err", mod.max_scaled_err)
    for check in metric_pins.CHECKS:
        check()
