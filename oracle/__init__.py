"""CPU oracle for the dose product d = A x (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library: the arithmetic lives in ``dose_oracle.c`` (plain C, FP64), written
from the definitions cited there; this module only marshals numpy arrays.

Value formats are named by strings here ("fp16", "bf16", "fp8e4m3_rowscale",
"fp32")
so that no enumeration is shared with the library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dose_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

FORMATS = {"fp16": 1, "bf16": 2, "fp8e4m3_rowscale": 3, "fp32": 4}


def build() -> str:
    """Compile liboracle.so with gcc, keeping every rounding as written."""
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
                           "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = load_library(_LIB_PATH)
    return _lib


def load_library(path: str):
    """A compiled copy of dose_oracle.c with its ctypes signatures declared."""
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    sigs = {
        "or_f16_encode": ([ctypes.c_float], ctypes.c_uint16),
        "or_f16_decode": ([ctypes.c_uint16], ctypes.c_double),
        "or_bf16_encode": ([ctypes.c_float], ctypes.c_uint16),
        "or_bf16_decode": ([ctypes.c_uint16], ctypes.c_double),
        "or_e4m3_encode_sat": ([ctypes.c_float], ctypes.c_uint8),
        "or_e4m3_decode": ([ctypes.c_uint8], ctypes.c_double),
        "or_e4m3_row_scale": ([vp, i64], ctypes.c_float),
        "or_f16_encode_n": ([vp, i64, vp], None),
        "or_f16_decode_n": ([vp, i64, vp], None),
        "or_bf16_encode_n": ([vp, i64, vp], None),
        "or_bf16_decode_n": ([vp, i64, vp], None),
        "or_e4m3_encode_n": ([vp, i64, vp], None),
        "or_e4m3_decode_n": ([vp, i64, vp], None),
        "or_decode_matrix": ([ctypes.c_int, i64, vp, vp, vp, vp], ctypes.c_int),
        "or_row_dot": ([i64, vp, vp, vp], ctypes.c_double),
        "or_spmv": ([i64, vp, vp, vp, vp, vp], None),
        "or_spmv_rows_parallel": ([i64, vp, vp, vp, vp, vp], None),
        "or_num_threads": ([], ctypes.c_int),
        "or_spmv_multi": ([i64, i32, vp, vp, vp, vp, vp], None),
        "or_spmv_T": ([i64, i64, vp, vp, vp, vp, vp], None),
        "or_transpose": ([i64, i64, vp, vp, vp, vp, vp, vp], None),
        "or_objective": ([i64, vp, vp, vp], ctypes.c_double),
        "or_objective_seed": ([i64, vp, vp, vp, vp], None),
        "or_norm2": ([i64, vp], ctypes.c_double),
        "or_beam_sum": ([i32, i64, vp, vp], None),
        "or_robust": ([i32, vp, vp, vp, vp, vp], None),
        "or_robust_weights": ([i32, vp, vp, i32, vp], None),
        "or_sell_layout": ([i64, vp, i64, i64, vp, vp], None),
        "or_sell_pack": ([i64, vp, vp, vp, i64, vp, vp, vp, vp], None),
        "or_sell_spmv": ([i64, i64, vp, vp, vp, vp, vp, vp], None),
        "or_runs_encode": ([i64, vp, vp, vp, vp, vp], i64),
        "or_runs_decode": ([i64, vp, vp, vp, vp], None),
    }
    for name, (args, res) in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


# ----------------------------------------------------------------- formats
def encode(fmt: str, v) -> np.ndarray:
    """Codes of FP32 values: uint16 for fp16/bf16, uint8 for E4M3 (no scaling)."""
    v, pv = _c(v, np.float32)
    lib = _load()
    if fmt == "fp16":
        out = np.empty(v.size, np.uint16)
        lib.or_f16_encode_n(pv, v.size, out.ctypes.data)
    elif fmt == "bf16":
        out = np.empty(v.size, np.uint16)
        lib.or_bf16_encode_n(pv, v.size, out.ctypes.data)
    elif fmt in ("e4m3", "fp8e4m3_rowscale"):
        out = np.empty(v.size, np.uint8)
        lib.or_e4m3_encode_n(pv, v.size, out.ctypes.data)
    else:
        raise ValueError(fmt)
    return out


def decode(fmt: str, codes) -> np.ndarray:
    """FP64 values of codes."""
    lib = _load()
    if fmt in ("fp16", "bf16"):
        c, pc = _c(codes, np.uint16)
        out = np.empty(c.size, np.float64)
        (lib.or_f16_decode_n if fmt == "fp16" else lib.or_bf16_decode_n)(pc, c.size,
                                                                        out.ctypes.data)
    elif fmt in ("e4m3", "fp8e4m3_rowscale"):
        c, pc = _c(codes, np.uint8)
        out = np.empty(c.size, np.float64)
        lib.or_e4m3_decode_n(pc, c.size, out.ctypes.data)
    else:
        raise ValueError(fmt)
    return out


def row_scale(vals) -> np.float32:
    v, pv = _c(vals, np.float32)
    return np.float32(_load().or_e4m3_row_scale(pv, v.size))


def decode_matrix(fmt: str, row_ptr, vals):
    """Decoded entries (FP32, exact) of a CSR matrix stored in format ``fmt``.

    Returns (dec, scales); scales is None except for the E4M3 row-scale format.
    """
    rp, prp = _c(row_ptr, np.int64)
    v, pv = _c(vals, np.float32)
    n_rows = rp.size - 1
    dec = np.empty(max(v.size, 1), np.float32)
    scales = np.empty(max(n_rows, 1), np.float32) if fmt == "fp8e4m3_rowscale" else None
    rc = _load().or_decode_matrix(FORMATS[fmt], n_rows, prp, pv, dec.ctypes.data,
                                  scales.ctypes.data if scales is not None else None)
    if rc != 0:
        raise ValueError(fmt)
    return dec[:v.size], (scales[:n_rows] if scales is not None else None)


# ----------------------------------------------------------------- products
def row_dot(cols, dec, x) -> float:
    c, pc = _c(cols, np.int32)
    d, pd = _c(dec, np.float32)
    xx, px = _c(x, np.float32)
    return float(_load().or_row_dot(c.size, pc, pd, px))


def spmv(row_ptr, cols, dec, x) -> np.ndarray:
    rp, prp = _c(row_ptr, np.int64)
    c, pc = _c(cols, np.int32)
    d, pd = _c(dec, np.float32)
    xx, px = _c(x, np.float32)
    y = np.empty(max(rp.size - 1, 1), np.float64)
    _load().or_spmv(rp.size - 1, prp, pc, pd, px, y.ctypes.data)
    return y[:rp.size - 1]


def spmv_parallel(row_ptr, cols, dec, x) -> np.ndarray:
    """spmv with the rows shared among the host's threads (same sums)."""
    rp, prp = _c(row_ptr, np.int64)
    c, pc = _c(cols, np.int32)
    d, pd = _c(dec, np.float32)
    xx, px = _c(x, np.float32)
    y = np.empty(max(rp.size - 1, 1), np.float64)
    _load().or_spmv_rows_parallel(rp.size - 1, prp, pc, pd, px, y.ctypes.data)
    return y[:rp.size - 1]


def num_threads() -> int:
    """Threads spmv_parallel uses."""
    return int(_load().or_num_threads())


def spmv_multi(row_ptr, cols, dec, x2d) -> np.ndarray:
    """x2d is [n_cols][n_rhs]; returns [n_rows][n_rhs] in FP64."""
    rp, prp = _c(row_ptr, np.int64)
    c, pc = _c(cols, np.int32)
    d, pd = _c(dec, np.float32)
    xx, px = _c(x2d, np.float32)
    n_rhs = xx.shape[1]
    y = np.empty((max(rp.size - 1, 1), n_rhs), np.float64)
    _load().or_spmv_multi(rp.size - 1, n_rhs, prp, pc, pd, px, y.ctypes.data)
    return y[:rp.size - 1]


# ------------------------------------------------------ SELL-C-sigma, runs
def sell_layout(row_ptr, C: int, sigma: int):
    """SELL-C-sigma layout (Kreutzer et al. 2014): (perm, width).  perm[k] is
    the row at sorted position k (descending length inside windows of sigma
    rows, ties in ascending row order); width[c] the longest row of chunk c
    (positions [c C, c C + C))."""
    rp, prp = _c(row_ptr, np.int64)
    n = rp.size - 1
    perm = np.empty(max(n, 1), np.int64)
    width = np.empty(max((n + C - 1) // C, 1), np.int64)
    _load().or_sell_layout(n, prp, C, sigma, perm.ctypes.data, width.ctypes.data)
    return perm[:n], width[:(n + C - 1) // C]


def sell_pack(row_ptr, cols, dec, C: int, perm, width):
    """Column-major padded chunk arrays (values, columns; padding 0 and -1)."""
    rp, prp = _c(row_ptr, np.int64)
    c, pc = _c(cols, np.int32)
    d, pd = _c(dec, np.float32)
    pm, ppm = _c(perm, np.int64)
    wd, pwd = _c(width, np.int64)
    total = int(C * wd.sum())
    sval = np.empty(max(total, 1), np.float32)
    scol = np.empty(max(total, 1), np.int32)
    _load().or_sell_pack(rp.size - 1, prp, pc, pd, C, ppm, pwd, sval.ctypes.data, scol.ctypes.data)
    return sval[:total], scol[:total]


def sell_spmv(n_rows: int, C: int, perm, width, sval, scol, x) -> np.ndarray:
    """y = A x in FP64 over the packed SELL-C-sigma arrays."""
    pm, ppm = _c(perm, np.int64)
    wd, pwd = _c(width, np.int64)
    sv, psv = _c(sval, np.float32)
    sc, psc = _c(scol, np.int32)
    xx, px = _c(x, np.float32)
    y = np.empty(max(n_rows, 1), np.float64)
    _load().or_sell_spmv(n_rows, C, ppm, pwd, psv, psc, px, y.ctypes.data)
    return y[:n_rows]


def runs_encode(row_ptr, cols):
    """Maximal runs of consecutive columns of every row: (run_ptr, start, len)."""
    rp, prp = _c(row_ptr, np.int64)
    c, pc = _c(cols, np.int32)
    n = rp.size - 1
    run_ptr = np.empty(n + 1, np.int64)
    start = np.empty(max(c.size, 1), np.int32)
    length = np.empty(max(c.size, 1), np.int32)
    nr = int(_load().or_runs_encode(n, prp, pc, run_ptr.ctypes.data, start.ctypes.data, length.ctypes.data))
    return run_ptr, start[:nr], length[:nr]


def runs_decode(run_ptr, start, length) -> np.ndarray:
    """The columns the runs describe, row after row."""
    rp, prp = _c(run_ptr, np.int64)
    st, pst = _c(start, np.int32)
    ln, pln = _c(length, np.int32)
    cols = np.empty(max(int(ln.sum()), 1), np.int32)
    _load().or_runs_decode(rp.size - 1, prp, pst, pln, cols.ctypes.data)
    return cols[:int(ln.sum())]


def spmv_T(row_ptr, cols, dec, v, n_cols: int) -> np.ndarray:
    rp, prp = _c(row_ptr, np.int64)
    c, pc = _c(cols, np.int32)
    d, pd = _c(dec, np.float32)
    vv, pv = _c(v, np.float32)
    g = np.empty(max(n_cols, 1), np.float64)
    _load().or_spmv_T(rp.size - 1, n_cols, prp, pc, pd, pv, g.ctypes.data)
    return g[:n_cols]


def transpose(row_ptr, cols, dec, n_cols: int):
    rp, prp = _c(row_ptr, np.int64)
    c, pc = _c(cols, np.int32)
    d, pd = _c(dec, np.float32)
    t_rp = np.empty(n_cols + 1, np.int64)
    t_c = np.empty(max(c.size, 1), np.int32)
    t_d = np.empty(max(c.size, 1), np.float32)
    _load().or_transpose(rp.size - 1, n_cols, prp, pc, pd, t_rp.ctypes.data, t_c.ctypes.data,
                         t_d.ctypes.data)
    return t_rp, t_c[:c.size], t_d[:c.size]


def objective(d, p, w) -> float:
    dd, pdd = _c(d, np.float64)
    pp, ppp = _c(p, np.float32)
    ww, pww = _c(w, np.float32)
    return float(_load().or_objective(dd.size, pdd, ppp, pww))


def objective_seed(d, p, w) -> np.ndarray:
    dd, pdd = _c(d, np.float64)
    pp, ppp = _c(p, np.float32)
    ww, pww = _c(w, np.float32)
    out = np.empty(max(dd.size, 1), np.float64)
    _load().or_objective_seed(dd.size, pdd, ppp, pww, out.ctypes.data)
    return out[:dd.size]


def beam_sum(part) -> np.ndarray:
    """Scenario dose from its beams' doses: part is (n_beams, n); returns the
    FP64 sum over beams for every voxel."""
    pa = np.ascontiguousarray(np.asarray(part, np.float64))
    if pa.ndim != 2:
        raise ValueError("part must be (n_beams, n)")
    out = np.empty(max(pa.shape[1], 1), np.float64)
    _load().or_beam_sum(pa.shape[0], pa.shape[1], pa.ctypes.data, out.ctypes.data)
    return out[:pa.shape[1]]


def robust(f, prob=None) -> tuple[float, int, float]:
    """(worst case, first scenario attaining it, expectation) of the scenario
    objectives f; uniform expectation (sum f / S) when prob is None."""
    ff = np.ascontiguousarray(np.asarray(f, np.float64))
    if ff.size < 1:
        raise ValueError("at least one scenario")
    pp = None if prob is None else np.ascontiguousarray(np.asarray(prob, np.float64))
    if pp is not None and pp.size != ff.size:
        raise ValueError("one probability per scenario")
    worst, expected = ctypes.c_double(), ctypes.c_double()
    arg = ctypes.c_int64()
    _load().or_robust(ff.size, ff.ctypes.data, None if pp is None else pp.ctypes.data,
                      ctypes.byref(worst), ctypes.byref(arg), ctypes.byref(expected))
    return worst.value, arg.value, expected.value


def robust_weights(f, prob=None, mode: str = "expected") -> np.ndarray:
    """Weights c_s of the robust forms: the derivative of the expectation
    (mode "expected") or of the worst case (mode "worst") with respect to
    each scenario's objective f_s."""
    ff = np.ascontiguousarray(np.asarray(f, np.float64))
    if ff.size < 1:
        raise ValueError("at least one scenario")
    if mode not in ("expected", "worst"):
        raise ValueError(mode)
    pp = None if prob is None else np.ascontiguousarray(np.asarray(prob, np.float64))
    if pp is not None and pp.size != ff.size:
        raise ValueError("one probability per scenario")
    c = np.empty(ff.size, np.float64)
    _load().or_robust_weights(ff.size, ff.ctypes.data, None if pp is None else pp.ctypes.data,
                              1 if mode == "worst" else 0, c.ctypes.data)
    return c


def norm2(g) -> float:
    gg, pg = _c(g, np.float64)
    return float(_load().or_norm2(gg.size, pg))


# ----------------------------------------------------------------- error metrics
# The parity bar of the dose product (Listing 1's per-voxel sum, FP32 against
# the FP64 definition): a per-voxel relative error, or, for signed inputs, the
# error scaled componentwise by |A| |x|.  Both are maxima over all entries; an
# entry whose reference (or scale) is exactly zero must itself be zero (either
# sign; where the sign is fixed, as for empty rows, tests check the bits), and
# a non-finite result is never within any bound.
def max_rel_err(y, y_ref) -> float:
    """max_i |y_i - y*_i| / |y*_i| over entries with y*_i != 0; returns inf if
    an entry with y*_i == 0 is not 0 in y, or if any y_i is not finite."""
    y = np.asarray(y, np.float64).reshape(-1)
    y_ref = np.asarray(y_ref, np.float64).reshape(-1)
    if y.shape != y_ref.shape:
        raise ValueError("y and y_ref differ in size")
    if not np.all(np.isfinite(y)):
        return float("inf")
    ref_zero = y_ref == 0.0
    if np.any(y[ref_zero] != 0.0):
        return float("inf")
    keep = ~ref_zero
    if not np.any(keep):
        return 0.0
    rel = np.abs(y[keep] - y_ref[keep]) / np.abs(y_ref[keep])
    return float(np.max(rel))


def max_scaled_err(y, y_ref, scale) -> float:
    """max_j |y_j - y*_j| / scale_j with scale = |A| |x| (componentwise);
    returns inf if an entry with scale_j == 0 is not 0 in y, or if any y_j is
    not finite."""
    y = np.asarray(y, np.float64).reshape(-1)
    y_ref = np.asarray(y_ref, np.float64).reshape(-1)
    scale = np.asarray(scale, np.float64).reshape(-1)
    if y.shape != y_ref.shape or y.shape != scale.shape:
        raise ValueError("y, y_ref and scale differ in size")
    if not np.all(np.isfinite(y)):
        return float("inf")
    scale_zero = scale == 0.0
    if np.any(y[scale_zero] != 0.0):
        return float("inf")
    held = ~scale_zero
    if not np.any(held):
        return 0.0
    scaled = np.abs(y[held] - y_ref[held]) / scale[held]
    return float(np.max(scaled))
