"""FP64 products over the SELL-C-sigma form (dose_sell_spmv_f64, the paper's
half/double arithmetic, Sec. II-D): FP64 spot weights and dose, FP64 products
and sums in the SELL order.

Reference: the oracle's FP64 sums, with each FP64 input built as hi + lo
(both exact in FP32, lo below hi's last bit; the reference is oracle(hi) +
oracle(lo)), so a kernel that rounded x to FP32 would lose lo.  Tolerance:
the kernel rounds each product once and sums in a fixed order of depth
below (14 + L / 256) for rows of L entries, far below 1e-12 relative; E4M3
factors the FP32 row scale out of the row sum where the oracle sums
fl32(q s) x, so 2^-22 there (as for the CSR FP64 product).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2103_09683_amd as dm

pytestmark = pytest.mark.gpu

FORMATS = ["fp16", "bf16", "fp8e4m3_rowscale", "fp32"]
TOL64 = 1e-12


def _say(*a):
    print(*a, flush=True)


def _with_low_bits(hi32, rng):
    hi = np.asarray(hi32, np.float32)
    e = np.frexp(hi.astype(np.float64))[1]
    u = (rng.choice([-1.0, 1.0], hi.size) * rng.uniform(0.5, 1.0, hi.size)).astype(np.float32)
    lo = np.ldexp(u.astype(np.float64), e - 26).astype(np.float32)
    x = hi.astype(np.float64) + lo.astype(np.float64)
    assert np.array_equal(x - hi.astype(np.float64), lo.astype(np.float64))
    return x, hi, lo


def _ray_matrix(seed, n_rows=2500, n_cols=60000, far=True):
    """Rows of 2-4 runs of consecutive columns near a drifting centre (narrow
    chunk windows), then, with `far`, rows whose runs sit far apart (windows
    beyond the LDS cap) and a few long rows."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n_rows):
        if rng.random() < 0.3:
            rows.append(np.zeros(0, np.int64))
            continue
        c = (i * 3) % 5000
        row = []
        for _ in range(rng.integers(2, 5)):
            c += int(rng.integers(1, 60))
            L = int(rng.choice([1, 2, 3, 7, 8, 9, 31, 33, 120, 250]))
            row.extend(range(c, c + L))
            c += L
        rows.append(np.array(sorted(set(row)), np.int64))
    if far:
        for i in range(800):
            starts = np.sort(rng.choice(np.arange(0, n_cols - 1000, 500), size=3, replace=False))
            L = int(rng.choice([5, 40, 300]))
            rows.append(np.concatenate([np.arange(s, s + L) for s in starts]))
        rows[5] = np.arange(100, 16100)
    lens = np.array([r.size for r in rows])
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    cols = np.concatenate(rows).astype(np.int32)
    vals = np.exp(rng.normal(-3, 1, cols.size)).astype(np.float32)
    return rp, cols, vals, n_cols


@pytest.mark.parametrize("fmt", FORMATS)
def test_sell_f64_vs_oracle(fmt, dev):
    rp, cols, vals, n_cols = _ray_matrix(70)
    rng = np.random.default_rng(71)
    x, hi, lo = _with_low_bits(rng.random(n_cols).astype(np.float32), rng)
    xd = torch.from_numpy(x).cuda()
    dec, _ = oracle.decode_matrix(fmt, rp, vals)
    y_ref = oracle.spmv(rp, cols, dec, hi) + oracle.spmv(rp, cols, dec, lo)
    tol = 2.0 ** -22 if fmt == "fp8e4m3_rowscale" else TOL64
    lens = np.diff(rp)
    outs = {}
    for idx in ("i32", "u16", "runs"):
        S = dm.SellMatrix(rp, cols, vals, n_cols, fmt, sigma=256, index_format=idx)
        inf = S.info()
        assert 0 < inf["n_groups_windowed"] < inf["n_groups"]
        y = torch.full((S.n_rows,), np.nan, dtype=torch.float64, device=dev)
        S.spmv(xd, y)
        y = y.cpu().numpy()
        err = oracle.max_rel_err(y, y_ref)
        _say(f"sell f64 {fmt} {idx}: max rel err {err:.3e}")
        assert err <= tol, (fmt, idx)
        assert np.all(y[lens == 0].view(np.uint64) == 0)
        outs[idx] = y.view(np.uint64)
        S.close()
    # the three index formats give the same bits
    assert np.array_equal(outs["u16"], outs["i32"]) and np.array_equal(outs["runs"], outs["i32"])


def test_sell_f64_equals_f32_on_exact_inputs(dev):
    """Dyadic values and small integer weights: both precisions are exact, so
    the FP64 dose equals the FP32 dose and the oracle's."""
    rp, cols, _, n_cols = _ray_matrix(72, far=False)
    rng = np.random.default_rng(73)
    vals = (rng.integers(1, 64, rp[-1]) / 64.0).astype(np.float32)
    x = rng.integers(0, 8, n_cols).astype(np.float32)
    S = dm.SellMatrix(rp, cols, vals, n_cols, "fp16", sigma=64, index_format="runs")
    y32 = S.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
    y64 = S.spmv(torch.from_numpy(x.astype(np.float64)).cuda()).cpu().numpy()
    np.testing.assert_array_equal(y64, y32.astype(np.float64))
    np.testing.assert_array_equal(y64, oracle.spmv(rp, cols, vals.astype(np.float64), x))
    S.close()


def test_sell_f64_empty_and_errors(dev):
    for n in (0, 100):
        S = dm.SellMatrix(np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 10, "fp16")
        y = torch.full((n,), np.nan, dtype=torch.float64, device=dev)
        S.spmv(torch.ones(10, dtype=torch.float64, device=dev), y)
        assert np.all(y.cpu().numpy().view(np.uint64) == 0)
        S.close()
    rp = np.array([0, 2, 3], np.int64)
    S = dm.SellMatrix(rp, np.array([0, 3, 1], np.int32), np.ones(3, np.float32), 4, "fp16")
    with pytest.raises(TypeError):
        S.spmv(torch.zeros(4, dtype=torch.float64, device=dev), torch.zeros(2, device=dev))
    lib = dm._lib.load()
    buf = torch.zeros(64, dtype=torch.float64, device=dev)
    base = buf.data_ptr()
    assert lib.dose_sell_spmv_f64(S.handle, base + 4, base + 256, None) == dm._lib.ERR_INVALID_ARGUMENT
    assert lib.dose_sell_spmv_f64(S.handle, base, base + 8, None) == dm._lib.ERR_INVALID_ARGUMENT  # overlap
    assert lib.dose_sell_spmv_f64(S.handle, None, base + 256, None) == dm._lib.ERR_INVALID_ARGUMENT
    S.close()
