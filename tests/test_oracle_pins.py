"""Pins of the CPU oracle against things other than itself.

Each test compares the oracle with an independent implementation (numpy's and
torch's own float conversions), a pure-Python brute force over the dense
matrix, a correctly rounded sum (math.fsum), a closed form, or a finite
difference.  Together they are meant to fail on any plausible slip in the
oracle: a dropped term, a wrong sign or index, a transposed operand, a
rounding-mode or exponent-bias mistake in an encoder.
"""
import math

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# --------------------------------------------------------------------------
# value formats
# --------------------------------------------------------------------------
def _f16_grid_and_midpoints():
    """Every finite binary16 value, the midpoints between neighbours (ties) and
    one FP32 ulp either side of each midpoint."""
    codes = np.arange(0, 0x7C00, dtype=np.uint16)
    vals = codes.view(np.float16).astype(np.float64)
    mids = (vals[:-1] + vals[1:]) / 2.0  # exact in FP32: at most 12 significant bits
    mids32 = mids.astype(np.float32)
    assert np.all(mids32.astype(np.float64) == mids)
    up = np.nextafter(mids32, np.float32(np.inf))
    dn = np.nextafter(mids32, np.float32(0))
    allv = np.concatenate([vals.astype(np.float32), mids32, up, dn])
    return np.concatenate([allv, -allv])


def test_fp16_encode_matches_numpy_on_ties_and_subnormals():
    v = _f16_grid_and_midpoints()
    ours = oracle.encode("fp16", v)
    ref = v.astype(np.float16).view(np.uint16)
    np.testing.assert_array_equal(ours, ref)


def test_fp16_encode_matches_numpy_on_random_fp32_bits():
    rng = np.random.default_rng(11)
    bits = rng.integers(0, 2**32, size=400_000, dtype=np.uint64).astype(np.uint32)
    v = bits.view(np.float32)
    v = v[np.isfinite(v)]
    ours = oracle.encode("fp16", v)
    ref = v.astype(np.float16).view(np.uint16)  # numpy rounds to nearest even, overflows to inf
    np.testing.assert_array_equal(ours, ref)


def test_fp16_decode_exhaustive():
    codes = np.arange(0, 65536, dtype=np.uint32).astype(np.uint16)
    ours = oracle.decode("fp16", codes)
    ref = codes.view(np.float16).astype(np.float64)
    np.testing.assert_array_equal(np.isnan(ours), np.isnan(ref))
    ok = ~np.isnan(ref)
    np.testing.assert_array_equal(ours[ok], ref[ok])
    # signed zero kept
    assert math.copysign(1.0, ours[0x8000]) == -1.0


def test_bf16_encode_matches_torch():
    rng = np.random.default_rng(12)
    bits = rng.integers(0, 2**32, size=400_000, dtype=np.uint64).astype(np.uint32)
    # add bfloat16 midpoints (ties) explicitly: low 16 bits == 0x8000
    ties = (bits & np.uint32(0xFFFF0000)) | np.uint32(0x8000)
    v = np.concatenate([bits, ties]).view(np.float32)
    v = v[np.isfinite(v)]
    ours = oracle.encode("bf16", v)
    ref = torch.from_numpy(v).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(ours, ref)


def test_bf16_decode_exhaustive():
    codes = np.arange(0, 65536, dtype=np.uint32).astype(np.uint16)
    ours = oracle.decode("bf16", codes)
    ref = torch.from_numpy(codes.view(np.int16)).view(torch.bfloat16).double().numpy()
    np.testing.assert_array_equal(np.isnan(ours), np.isnan(ref))
    ok = ~np.isnan(ref)
    np.testing.assert_array_equal(ours[ok], ref[ok])


def test_e4m3_decode_exhaustive_matches_torch():
    codes = np.arange(256, dtype=np.uint8)
    ours = oracle.decode("e4m3", codes)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).double().numpy()
    np.testing.assert_array_equal(np.isnan(ours), np.isnan(ref))
    ok = ~np.isnan(ref)
    np.testing.assert_array_equal(ours[ok], ref[ok])
    assert ours[0x7E] == 448.0 and ours[0x01] == 2.0 ** -9 and ours[0x08] == 2.0 ** -6


def test_e4m3_encode_matches_torch_below_saturation():
    finite = oracle.decode("e4m3", np.arange(0, 0x7F, dtype=np.uint8))  # 0 .. 448
    mids = (finite[:-1] + finite[1:]) / 2.0
    m32 = mids.astype(np.float32)
    grid = np.concatenate([finite.astype(np.float32), m32, np.nextafter(m32, np.float32(np.inf)),
                           np.nextafter(m32, np.float32(0))])
    rng = np.random.default_rng(13)
    rand = rng.uniform(0.0, 463.9, size=200_000).astype(np.float32)
    tiny = rng.uniform(0.0, 2.0 ** -5, size=50_000).astype(np.float32)
    v = np.concatenate([grid, rand, tiny])
    v = np.concatenate([v, -v])
    ours = oracle.encode("e4m3", v)
    ref = torch.from_numpy(v).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(ours, ref)


def test_e4m3_saturates_at_448():
    v = np.array([464.0, 470.0, 480.0, 1e6, 3e38, -500.0], dtype=np.float32)
    ours = oracle.encode("e4m3", v)
    np.testing.assert_array_equal(ours, [0x7E, 0x7E, 0x7E, 0x7E, 0x7E, 0xFE])


def test_e4m3_row_scale_closed_forms():
    assert oracle.row_scale(np.array([448.0, 1.0], np.float32)) == 1.0
    assert oracle.row_scale(np.array([0.0, -896.0], np.float32)) == 2.0
    assert oracle.row_scale(np.array([0.0, 0.0], np.float32)) == 1.0
    assert oracle.row_scale(np.array([], np.float32)) == 1.0
    # quotient underflows FP32: the scale falls back to 1
    assert oracle.row_scale(np.array([1e-44], np.float32)) == 1.0
    # one correctly rounded FP32 division
    a = np.float32(0.7)
    assert oracle.row_scale(np.array([a], np.float32)) == np.float32(a) / np.float32(448.0)


def test_decode_matrix_fp8_error_bound():
    rng = np.random.default_rng(14)
    n_rows = 200
    lens = rng.integers(0, 40, size=n_rows)
    rp = np.zeros(n_rows + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    vals = np.exp(rng.normal(-3, 1, size=rp[-1])).astype(np.float32)
    vals[::7] *= -1
    dec, scales = oracle.decode_matrix("fp8e4m3_rowscale", rp, vals)
    for i in range(n_rows):
        seg = slice(rp[i], rp[i + 1])
        a = vals[seg].astype(np.float64)
        if a.size == 0:
            assert scales[i] == 1.0
            continue
        s = np.float64(scales[i])
        assert s == np.float32(np.max(np.abs(vals[seg]))) / np.float32(448.0)
        # half an E4M3 ulp relative (2^-4) on normals, half the subnormal quantum
        # (2^-10 * s) absolute, plus the FP32 roundings of a/s and q*s
        bound = (2.0 ** -4 + 3 * 2.0 ** -24) * np.abs(a) + 2.0 ** -10 * s
        assert np.all(np.abs(dec[seg].astype(np.float64) - a) <= bound)
        # the largest magnitude maps to 448 * s up to the two FP32 roundings
        k = np.argmax(np.abs(a))
        assert abs(abs(dec[seg][k]) - 448.0 * s) <= 2.0 ** -22 * 448.0 * s


def test_decode_matrix_fp16_bf16_are_elementwise():
    rng = np.random.default_rng(15)
    rp = np.array([0, 3, 3, 7], np.int64)
    vals = rng.uniform(-2, 2, size=7).astype(np.float32)
    d16, _ = oracle.decode_matrix("fp16", rp, vals)
    np.testing.assert_array_equal(d16, vals.astype(np.float16).astype(np.float32))
    db, _ = oracle.decode_matrix("bf16", rp, vals)
    ref = torch.from_numpy(vals).to(torch.bfloat16).float().numpy()
    np.testing.assert_array_equal(db, ref)


# --------------------------------------------------------------------------
# the product, against a pure-Python dense brute force
# --------------------------------------------------------------------------
def _random_csr(rng, n_rows, n_cols, density, signed=True, empty_rows=True):
    dense = np.zeros((n_rows, n_cols), np.float32)
    mask = rng.random((n_rows, n_cols)) < density
    if empty_rows:
        mask[rng.random(n_rows) < 0.3] = False
    vals = rng.uniform(-1 if signed else 0, 1, size=mask.sum()).astype(np.float32)
    dense[mask] = vals
    rp = np.zeros(n_rows + 1, np.int64)
    np.cumsum(mask.sum(1), out=rp[1:])
    cols = np.nonzero(mask)[1].astype(np.int32)
    return dense, rp, cols, dense[mask]


def _dense_python(dense64, x):
    """y_i = sum_j a_ij x_j over ALL columns, ascending j, Python floats."""
    y = []
    for i in range(dense64.shape[0]):
        acc = 0.0
        for j in range(dense64.shape[1]):
            acc += dense64[i, j] * float(x[j])
        y.append(acc)
    return np.array(y)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_spmv_bit_exact_vs_dense_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    dense, rp, cols, vals = _random_csr(rng, 37, 23, 0.35)
    x = rng.uniform(-1, 1, size=23).astype(np.float32)
    # decoded entries in the paper's format; the dense copy uses the same values
    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    d64 = np.zeros(dense.shape)
    d64[dense != 0] = dec
    y = oracle.spmv(rp, cols, dec, x)
    y_ref = _dense_python(d64, x)
    # adding exact zeros (0*x) never changes a running sum except -0 -> +0,
    # so the dense loop performs the same sequence of non-zero additions
    np.testing.assert_array_equal(y, y_ref)


def test_spmv_within_fsum_bound_on_long_rows():
    rng = np.random.default_rng(200)
    n_rows, n_cols = 8, 5000
    rp = np.arange(0, (n_rows + 1) * n_cols, n_cols, dtype=np.int64)
    cols = np.tile(np.arange(n_cols, dtype=np.int32), n_rows)
    vals = np.exp(rng.normal(-3, 1, size=rp[-1])).astype(np.float32)
    x = rng.uniform(0, 1, size=n_cols).astype(np.float32)
    dec, _ = oracle.decode_matrix("bf16", rp, vals)
    y = oracle.spmv(rp, cols, dec, x)
    for i in range(n_rows):
        terms = [float(dec[k]) * float(x[cols[k]]) for k in range(rp[i], rp[i + 1])]
        exact = math.fsum(terms)
        n = len(terms)
        assert abs(y[i] - exact) <= (n - 1) * 2.0 ** -53 * math.fsum(abs(t) for t in terms)


def test_spmv_hand_worked_example():
    # A = [[0.5, 0, 0.25, 0], [0, 0, 0, 0], [1, 2, 0, 0.125]], x = [1, 2, 3, 4]
    rp = np.array([0, 2, 2, 5], np.int64)
    cols = np.array([0, 2, 0, 1, 3], np.int32)
    vals = np.array([0.5, 0.25, 1.0, 2.0, 0.125], np.float32)
    x = np.array([1, 2, 3, 4], np.float32)
    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    y = oracle.spmv(rp, cols, dec, x)
    np.testing.assert_array_equal(y, [1.25, 0.0, 5.5])
    assert math.copysign(1.0, y[1]) == 1.0  # empty row: +0
    g = oracle.spmv_T(rp, cols, dec, np.array([1, 7, 2], np.float32), 4)
    np.testing.assert_array_equal(g, [2.5, 4.0, 0.25, 0.25])


def test_spmv_unit_vectors_give_columns():
    rng = np.random.default_rng(300)
    dense, rp, cols, vals = _random_csr(rng, 40, 17, 0.4)
    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    d32 = np.zeros(dense.shape, np.float32)
    d32[dense != 0] = dec
    for j in range(17):
        e = np.zeros(17, np.float32)
        e[j] = 1.0
        y = oracle.spmv(rp, cols, dec, e)
        np.testing.assert_array_equal(y, d32[:, j].astype(np.float64))


def test_spmv_identity():
    n = 50
    rp = np.arange(n + 1, dtype=np.int64)
    cols = np.arange(n, dtype=np.int32)
    dec = np.ones(n, np.float32)
    x = np.random.default_rng(1).uniform(-3, 3, n).astype(np.float32)
    np.testing.assert_array_equal(oracle.spmv(rp, cols, dec, x), x.astype(np.float64))


def test_spmv_linearity_and_nonnegativity():
    rng = np.random.default_rng(400)
    dense, rp, cols, vals = _random_csr(rng, 60, 30, 0.3, signed=False)
    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    x = rng.uniform(0, 1, 30).astype(np.float32)
    z = rng.uniform(0, 1, 30).astype(np.float32)
    yx, yz = oracle.spmv(rp, cols, dec, x), oracle.spmv(rp, cols, dec, z)
    assert np.all(yx >= 0) and np.all(yz >= 0)
    xz = (x.astype(np.float64) + z.astype(np.float64)).astype(np.float32)
    # x + z is rounded to FP32, so linearity holds up to that rounding
    yxz = oracle.spmv(rp, cols, dec, xz)
    absA = oracle.spmv(rp, cols, np.abs(dec), np.abs(xz))
    assert np.all(np.abs(yxz - (yx + yz)) <= 1e-6 * absA + 1e-300)


def test_spmv_T_matches_dense_transpose_and_adjointness():
    rng = np.random.default_rng(500)
    dense, rp, cols, vals = _random_csr(rng, 45, 28, 0.3)
    dec, _ = oracle.decode_matrix("bf16", rp, vals)
    d64 = np.zeros(dense.shape)
    d64[dense != 0] = dec
    v = rng.uniform(-1, 1, 45).astype(np.float32)
    g = oracle.spmv_T(rp, cols, dec, v, 28)
    # dense brute force over A^T: ascending i for each j
    g_ref = _dense_python(np.ascontiguousarray(d64.T), v)
    np.testing.assert_array_equal(g, g_ref)
    x = rng.uniform(-1, 1, 28).astype(np.float32)
    y = oracle.spmv(rp, cols, dec, x)
    lhs = math.fsum(float(a) * float(b) for a, b in zip(v, y))
    rhs = math.fsum(float(a) * float(b) for a, b in zip(g, x))
    scale = math.fsum(abs(float(d64[i, j]) * v[i] * x[j]) for i in range(45) for j in range(28))
    assert abs(lhs - rhs) <= 1e-13 * scale


def test_transpose_structure():
    rng = np.random.default_rng(600)
    dense, rp, cols, vals = _random_csr(rng, 33, 19, 0.3)
    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    t_rp, t_c, t_d = oracle.transpose(rp, cols, dec, 19)
    dT = np.zeros((19, 33), np.float32)
    for j in range(19):
        seg = slice(t_rp[j], t_rp[j + 1])
        assert np.all(np.diff(t_c[seg]) > 0)
        dT[j, t_c[seg]] = t_d[seg]
    d32 = np.zeros(dense.shape, np.float32)
    d32[dense != 0] = dec
    np.testing.assert_array_equal(dT, d32.T)


def test_spmv_parallel_equals_sequential_bitwise():
    """The all-core timing variant sums every row exactly as the sequential
    oracle (rows are independent): equal bits, on a matrix with empty rows
    and rows long enough to be split among threads' chunks."""
    rng = np.random.default_rng(12)
    lens = rng.integers(0, 60, 20000)
    lens[::7] = 0
    rp = np.zeros(lens.size + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    cols = np.concatenate([np.sort(rng.choice(900, L, replace=False)) for L in lens]).astype(np.int32)
    dec = rng.random(rp[-1]).astype(np.float32)
    x = rng.random(900).astype(np.float32)
    a = oracle.spmv(rp, cols, dec, x)
    b = oracle.spmv_parallel(rp, cols, dec, x)
    np.testing.assert_array_equal(a.view(np.uint64), b.view(np.uint64))
    assert oracle.num_threads() >= 1


def test_spmv_multi_matches_columns_of_single():
    rng = np.random.default_rng(700)
    dense, rp, cols, vals = _random_csr(rng, 30, 12, 0.4)
    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    X = rng.uniform(0, 1, (12, 4)).astype(np.float32)
    Y = oracle.spmv_multi(rp, cols, dec, X)
    for r in range(4):
        np.testing.assert_array_equal(Y[:, r], oracle.spmv(rp, cols, dec, X[:, r].copy()))


# --------------------------------------------------------------------------
# objective and gradient
# --------------------------------------------------------------------------
def test_objective_closed_form_and_seed():
    d = np.array([1.0, 61.0, 20.5, -2.0])
    p = np.array([0.0, 60.0, 20.0, 0.0], np.float32)
    w = np.array([1.0, 10.0, 10.0, 1.0], np.float32)
    assert oracle.objective(d, p, w) == 1.0 + 10.0 + 2.5 + 4.0
    np.testing.assert_array_equal(oracle.objective_seed(d, p, w), [2.0, 20.0, 10.0, -4.0])
    assert oracle.norm2(np.array([3.0, 4.0])) == 5.0


def test_gradient_matches_central_finite_differences():
    rng = np.random.default_rng(800)
    dense, rp, cols, vals = _random_csr(rng, 80, 20, 0.3, signed=False)
    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    p = rng.choice([0.0, 20.0, 60.0], size=80).astype(np.float32)
    w = rng.choice([1.0, 10.0], size=80).astype(np.float32)
    x = rng.uniform(0, 1, 20).astype(np.float32)

    def f(xx):
        return oracle.objective(oracle.spmv(rp, cols, dec, xx), p, w)

    d = oracle.spmv(rp, cols, dec, x)
    seed = oracle.objective_seed(d, p, w).astype(np.float32)
    # the adjoint of the exact seed, in FP64 through a dense product
    d64 = np.zeros(dense.shape)
    d64[dense != 0] = dec
    grad = d64.T @ oracle.objective_seed(d, p, w)
    g_oracle = oracle.spmv_T(rp, cols, dec, seed, 20)  # FP32 seed: within FP32 rounding
    h = 0.5
    for j in range(20):
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (f(xp) - f(xm)) / (float(xp[j]) - float(xm[j]))
        # f is quadratic: central differences are exact up to FP64 rounding of f
        assert abs(fd - grad[j]) <= 1e-9 * max(1.0, abs(f(x)))
        bound_j = 2.0 ** -23 * float(np.abs(d64[:, j]) @ np.abs(seed))
        assert abs(g_oracle[j] - grad[j]) <= bound_j + 1e-12


def test_fp32_format_is_the_values_themselves():
    """The Single control stores the FP32 source values: its decoded matrix is
    the input, bit for bit (signed zeros, subnormals and large values
    included)."""
    rp = np.array([0, 3, 3, 7], np.int64)
    vals = np.array([1.5, -0.0, 3.4028235e38, 1e-45, -2.5e-40, 7.0, 0.1], np.float32)
    dec, scales = oracle.decode_matrix("fp32", rp, vals)
    assert scales is None
    np.testing.assert_array_equal(dec.view(np.uint32), vals.view(np.uint32))


# --------------------------------------------------------------------------
# scenario dose and robust objective
# --------------------------------------------------------------------------
def _csr_of_dense(dense):
    mask = dense != 0
    rp = np.zeros(dense.shape[0] + 1, np.int64)
    np.cumsum(mask.sum(1), out=rp[1:])
    return rp, np.nonzero(mask)[1].astype(np.int32), dense[mask].astype(np.float32)


def test_beam_sum_equals_product_with_side_by_side_beams():
    """Placing a scenario's beam matrices side by side (one column block per
    beam) and their spot weights end to end gives one matrix whose product is
    the scenario dose.  Small integers keep every sum exact, so a dropped beam,
    a beam read twice or a transposed (beam, voxel) index fails."""
    rng = np.random.default_rng(900)
    n_rows, widths = 60, [7, 11, 5, 9]
    doses, blocks, xs = [], [], []
    for nc in widths:
        dense = np.where(rng.random((n_rows, nc)) < 0.4, rng.integers(1, 9, (n_rows, nc)), 0)
        dense = dense.astype(np.float32)
        dense[rng.random(n_rows) < 0.2] = 0.0
        x = rng.integers(0, 5, nc).astype(np.float32)
        rp, cols, vals = _csr_of_dense(dense)
        dec, _ = oracle.decode_matrix("fp16", rp, vals)
        doses.append(oracle.spmv(rp, cols, dec, x))
        blocks.append(dense)
        xs.append(x)
    big, xb = np.hstack(blocks), np.concatenate(xs)
    rp, cols, vals = _csr_of_dense(big)
    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    d = oracle.beam_sum(np.stack(doses))
    np.testing.assert_array_equal(d, oracle.spmv(rp, cols, dec, xb))
    np.testing.assert_array_equal(d, _dense_python(big.astype(np.float64), xb))
    np.testing.assert_array_equal(oracle.beam_sum(np.stack(doses[:1])), doses[0])


def test_beam_sum_is_the_correctly_rounded_sum_of_few_terms():
    rng = np.random.default_rng(901)
    part = rng.uniform(2.0 ** -10, 1, (4, 1000)).astype(np.float32).astype(np.float64)
    d = oracle.beam_sum(part)
    ref = np.array([math.fsum(part[:, v]) for v in range(part.shape[1])])
    # four FP32 terms in [2^-10, 1): every bit of the exact sum lies between
    # 2^1 and 2^-33, so the FP64 sum is exact and equals the rounded one
    np.testing.assert_array_equal(d, ref)


def test_robust_closed_forms():
    assert oracle.robust([3.0, 7.0, 5.0], [0.5, 0.25, 0.25]) == (7.0, 1, 4.5)
    assert oracle.robust([4.0]) == (4.0, 0, 4.0)
    worst, arg, expected = oracle.robust([2.0, 9.0, 9.0])
    assert (worst, arg) == (9.0, 1)  # ties go to the first scenario
    assert expected == 20.0 / 3.0
    f = [1.5, 8.25, 3.0, 8.0]
    for k in range(4):
        onehot = np.zeros(4)
        onehot[k] = 1.0
        assert oracle.robust(f, onehot) == (8.25, 1, f[k])


def test_robust_expectation_vs_exact_fractions():
    from fractions import Fraction
    rng = np.random.default_rng(902)
    for _ in range(20):
        n = int(rng.integers(1, 12))
        fi, pi = rng.integers(0, 4000, n), rng.integers(0, 65, n)
        f, prob = fi / 4.0, pi / 64.0
        worst, arg, expected = oracle.robust(f, prob)
        # every product and partial sum is a multiple of 1/256 below 2^24: exact in FP64
        assert expected == float(sum(Fraction(int(a), 4) * Fraction(int(b), 64) for a, b in zip(fi, pi)))
        assert worst == f.max() and arg == int(np.argmax(f))
        _, _, mean = oracle.robust(f)
        assert mean == float(Fraction(int(fi.sum()), 4)) / n


def test_robust_weights_are_the_derivatives_of_the_robust_forms():
    """c_s = d(robust form)/d f_s, checked by one-sided differences of the
    oracle's robust forms with a dyadic step (exact: every value is a
    multiple of 1/64 well below 2^40) away from ties, and the first-scenario
    convention on ties."""
    rng = np.random.default_rng(77)
    h = 1.0 / 64.0
    for _ in range(20):
        n = int(rng.integers(1, 10))
        f = rng.permutation(n).astype(np.float64) * 4.0 + 1.0  # distinct: no ties
        prob = rng.integers(0, 65, n) / 64.0
        for mode in ("expected", "worst"):
            for pr in ((prob, None) if mode == "expected" else (None,)):
                c = oracle.robust_weights(f, pr, mode)
                for s in range(n):
                    fp = f.copy()
                    fp[s] += h
                    w0, _, e0 = oracle.robust(f, pr)
                    w1, _, e1 = oracle.robust(fp, pr)
                    slope = ((e1 - e0) if mode == "expected" else (w1 - w0)) / h
                    if mode == "expected" and pr is None:
                        # the mean: (sum f) / n rounds; the slope is 1/n up to that rounding
                        assert abs(slope - c[s]) <= 1e-9 and c[s] == 1.0 / n
                    else:
                        assert slope == c[s], (mode, n, s, slope, c[s])
    # ties: the first worst scenario takes the whole weight
    np.testing.assert_array_equal(oracle.robust_weights([2.0, 9.0, 9.0, 1.0], mode="worst"), [0, 1, 0, 0])
    np.testing.assert_array_equal(oracle.robust_weights([5.0], mode="worst"), [1.0])
    np.testing.assert_array_equal(oracle.robust_weights([5.0, 6.0], [0.75, 0.25]), [0.75, 0.25])


# --------------------------------------------------------------------------
# format error: the oracle on decoded values against the oracle on the FP32
# source values (reported, and held to each format's rounding bound)
# --------------------------------------------------------------------------
def test_format_error_within_each_formats_rounding_bound(capsys):
    """Per row, |y(decoded) - y(source)| <= sum_k e_k x_k with the per-entry
    rounding bound e_k of the format: FP16 max(2^-11 |a|, 2^-25) (normal and
    subnormal half-ulp), BF16 2^-8 |a|, E4M3 with row scale s
    (2^-4 + 2^-22) |a| + 2^-10 s (1 + 2^-22) (half-ulp of normal and
    subnormal codes of a/s, plus the FP32 roundings of a/s and q s).  The
    largest relative format error over non-empty rows is printed."""
    import dosegen
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    x = dosegen.spot_weights(spec.seed, 0, spec.n_cols)
    src, _ = oracle.decode_matrix("fp32", rp, vals)
    y_src = oracle.spmv(rp, cols, src, x)
    a = np.abs(vals.astype(np.float64))
    lens = np.diff(rp)
    row_of = np.repeat(np.arange(lens.size), lens)
    report = {}
    for fmt in ("fp16", "bf16", "fp8e4m3_rowscale"):
        dec, scale = oracle.decode_matrix(fmt, rp, vals)
        y = oracle.spmv(rp, cols, dec, x)
        if fmt == "fp16":
            e = np.maximum(2.0 ** -11 * a, 2.0 ** -25)
        elif fmt == "bf16":
            e = 2.0 ** -8 * a
        else:
            s = np.asarray(scale, np.float64)[row_of]
            e = (2.0 ** -4 + 2.0 ** -22) * a + 2.0 ** -10 * s * (1 + 2.0 ** -22)
        bound = np.bincount(row_of, weights=e * x[cols].astype(np.float64), minlength=lens.size)
        assert np.all(np.abs(y - y_src) <= bound * (1 + 1e-9) + 1e-300), fmt
        nz = y_src != 0
        report[fmt] = float(np.max(np.abs(y[nz] - y_src[nz]) / y_src[nz]))
    with capsys.disabled():
        print(f"\nformat error (max relative, {spec.name}): " +
              ", ".join(f"{k} {v:.3e}" for k, v in report.items()))
    # the formats' unit roundoffs order the errors
    assert report["fp16"] < report["bf16"] < report["fp8e4m3_rowscale"]
