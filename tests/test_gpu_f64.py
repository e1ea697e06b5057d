"""FP64 products (the paper's half/double configuration, Sec. II-D): FP64
spot weights and dose, FP64 products and sums over the stored FP16 / BF16 /
E4M3 matrix.

Reference: the oracle's FP64 sums.  Each FP64 input is built as hi + lo with
both parts exact in FP32 and lo below hi's last bit, and the reference is
oracle(hi) + oracle(lo): a kernel that rounded x to FP32 would lose the lo
part (about 2^-26 of x).

Tolerances: the FP64 kernel rounds each product once and sums in a tree of
depth below 50, so its error is below 50 * 2^-53 (about 6e-15) of sum |a||x|;
1e-12 is written.  The forward E4M3 product factors the FP32 row scale out of
the row sum (s * sum q x) where the oracle sums fl32(q s) x, so each term
may differ by 2^-24 relative: 2^-22 there.
"""
import numpy as np
import pytest
import torch

import dosegen
import oracle
import paper_2103_09683_amd as dm

pytestmark = pytest.mark.gpu

FORMATS = ["fp16", "bf16", "fp8e4m3_rowscale"]
TOL64 = 1e-12


def _say(*a):
    print(*a, flush=True)


def _with_low_bits(hi32, rng):
    """FP64 values hi + lo, both parts exact in FP32, lo below hi's last bit
    (hi = m 2^e with m in [0.5, 1) holds bits 2^(e-1) .. 2^(e-24); lo = u
    2^(e-26) with |u| in [0.5, 1) holds bits 2^(e-27) .. 2^(e-50)): the sum
    spans at most 50 bits, so it is exact in FP64, and rounding it to FP32
    loses lo."""
    hi = np.asarray(hi32, np.float32)
    e = np.frexp(hi.astype(np.float64))[1]
    u = (rng.choice([-1.0, 1.0], hi.size) * rng.uniform(0.5, 1.0, hi.size)).astype(np.float32)  # |u| in [0.5, 1)
    lo = np.ldexp(u.astype(np.float64), e - 26).astype(np.float32)
    x = hi.astype(np.float64) + lo.astype(np.float64)
    assert np.array_equal(x - hi.astype(np.float64), lo.astype(np.float64))
    return x, hi, lo


def _long_row_csr(seed, n_rows=3000, n_cols=6000):
    """Short rows, empty rows and a few rows of 2,100 to 5,900 entries (split
    groups under small partitions)."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 40, n_rows)
    lens[rng.random(n_rows) < 0.3] = 0
    lens[[7, 1500, 2999]] = [5900, 2100, 4097]
    rp = np.zeros(n_rows + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    cols = np.concatenate([np.sort(rng.choice(n_cols, l, replace=False)) for l in lens]).astype(np.int32)
    vals = rng.lognormal(-3, 1, rp[-1]).astype(np.float32)
    return rp, cols, vals, n_cols


def _cases():
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    yield "small_plain", rp, cols, vals, spec.n_cols
    yield "long_rows", *_long_row_csr(7)


@pytest.mark.parametrize("fmt", FORMATS)
def test_forward_and_adjoint_f64_vs_oracle(fmt, dev):
    rng = np.random.default_rng(64)
    for name, rp, cols, vals, n_cols in _cases():
        _say("f64", fmt, name)
        A = dm.DoseMatrix(rp, cols, vals, n_cols, fmt, transpose=True)
        dec, _ = oracle.decode_matrix(fmt, rp, vals)
        x, hi, lo = _with_low_bits(rng.random(n_cols).astype(np.float32), rng)
        y = A.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
        assert y.dtype == np.float64
        y_ref = oracle.spmv(rp, cols, dec, hi) + oracle.spmv(rp, cols, dec, lo)
        tol = 2.0 ** -22 if fmt == "fp8e4m3_rowscale" else TOL64
        assert oracle.max_rel_err(y, y_ref) <= tol, (fmt, name)
        lens = np.diff(rp)
        assert np.all(y[lens == 0].view(np.uint64) == 0)
        # adjoint with a signed FP64 seed
        v, vh, vl = _with_low_bits(rng.standard_normal(rp.size - 1).astype(np.float32), rng)
        g = A.adjoint(torch.from_numpy(v).cuda()).cpu().numpy()
        g_ref = oracle.spmv_T(rp, cols, dec, vh, n_cols) + oracle.spmv_T(rp, cols, dec, vl, n_cols)
        scale = oracle.spmv_T(rp, cols, np.abs(dec), np.abs(vh), n_cols)
        assert oracle.max_scaled_err(g, g_ref, scale) <= TOL64, (fmt, name)
        A.close()


@pytest.mark.parametrize("fmt", FORMATS)
def test_f64_bitwise_under_any_partition(fmt, dev):
    rp, cols, vals, n_cols = _long_row_csr(11)
    A = dm.DoseMatrix(rp, cols, vals, n_cols, fmt, transpose=True)
    rng = np.random.default_rng(5)
    x = torch.from_numpy(rng.random(n_cols)).cuda()
    v = torch.from_numpy(rng.standard_normal(rp.size - 1)).cuda()
    outs = []
    for g in [1024, 4096, 16384]:
        _say("f64 partition", fmt, g)
        A.set_partition(g, g)
        outs.append((A.spmv(x).cpu().numpy().view(np.uint64), A.adjoint(v).cpu().numpy().view(np.uint64)))
    for y, g in outs[1:]:
        np.testing.assert_array_equal(y, outs[0][0])
        np.testing.assert_array_equal(g, outs[0][1])
    A.close()


def test_f64_equals_f32_on_exact_inputs(dev):
    """Dyadic values and small integer weights: both precisions are exact, so
    the FP64 dose equals the FP32 dose."""
    rp, cols, _, n_cols = _long_row_csr(3)
    rng = np.random.default_rng(9)
    vals = (rng.integers(1, 64, rp[-1]) / 64.0).astype(np.float32)
    A = dm.DoseMatrix(rp, cols, vals, n_cols, "fp16")
    x = rng.integers(0, 8, n_cols).astype(np.float32)
    y32 = A.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
    y64 = A.spmv(torch.from_numpy(x.astype(np.float64)).cuda()).cpu().numpy()
    np.testing.assert_array_equal(y64, y32.astype(np.float64))
    A.close()


def test_f64_argument_checks(dev):
    rp = np.array([0, 2, 3], np.int64)
    A = dm.DoseMatrix(rp, np.array([0, 3, 1], np.int32), np.ones(3, np.float32), 4, "fp16")
    with pytest.raises(TypeError):
        A.spmv(torch.zeros(4, dtype=torch.float64, device=dev), torch.zeros(2, device=dev))
    from paper_2103_09683_amd import _lib
    buf = torch.zeros(64, dtype=torch.float64, device=dev)
    base = buf.data_ptr()
    lib = _lib.load()
    assert lib.dose_spmv_f64(A.handle, base + 4, base + 256, None) == _lib.ERR_INVALID_ARGUMENT
    assert lib.dose_spmv_adjoint_f64(A.handle, base, base + 256, None) == _lib.ERR_NO_TRANSPOSE
    A.close()
