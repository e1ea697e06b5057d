"""GPU parity of the SELL-C-sigma storage (C = 64) against the CPU oracle.

* Decode: the device layout read back in Kreutzer's column-major form equals
  the oracle's packing of the oracle's decoded values bit for bit (values,
  columns, padding 0 and -1, row order and chunk widths), in every value and
  index format, for sigma = 1 (no sorting), 64, 256 and 300 (windows that
  straddle chunks), with ragged tails, empty rows and signed values.
* Product: within 1e-5 of the oracle's product over the packed arrays (which
  equals the CSR oracle bit for bit) per voxel, componentwise-scaled for
  signed values; exact +0 on empty rows; bit for bit equal to the CSR
  product and to the oracle on exact-arithmetic inputs; 16-bit indices equal
  32-bit ones bit for bit; LDS-window and global-gather groups agree.
"""
import numpy as np
import pytest
import torch

import dosegen
import oracle
import paper_2103_09683_amd as dm

pytestmark = pytest.mark.gpu

FORMATS = ["fp16", "bf16", "fp8e4m3_rowscale", "fp32"]
TOL = 1e-5


def _say(*a):
    print(*a, flush=True)


def _bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def _csr(rng, lens, n_cols, signed=False, span=None, shift=7):
    """Rows of the given lengths; columns sorted, drawn from a window of
    `span` columns that moves with the row (or from all columns)."""
    rp = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    cols = np.empty(rp[-1], np.int32)
    for i, L in enumerate(lens):
        if L:
            if span is None:
                cols[rp[i]:rp[i + 1]] = np.sort(rng.choice(n_cols, size=L, replace=False))
            else:
                lo = (i * shift) % max(1, n_cols - span)
                cols[rp[i]:rp[i + 1]] = lo + np.sort(rng.choice(span, size=L, replace=False))
    vals = np.exp(rng.normal(-3, 1, size=rp[-1])).astype(np.float32)
    if signed:
        vals[rng.random(vals.size) < 0.4] *= -1
    if vals.size > 64:
        vals[:16] = (np.arange(1, 17) * 2.0 ** -24).astype(np.float32)  # FP16 subnormals
        vals[16:32] = np.float32(1.0 + 2.0 ** -11) * np.arange(1, 17, dtype=np.float32)  # FP16 ties
        vals[32:48] = np.float32(1.0 + 2.0 ** -8)  # BF16 ties
    return rp, cols, vals


def _lens(rng, n, max_len, empty=0.3):
    lens = rng.integers(1, max_len, n)
    lens[rng.random(n) < empty] = 0
    return lens


@pytest.mark.parametrize("fmt", FORMATS)
@pytest.mark.parametrize("sigma", [1, 64, 256, 300])
def test_decode_bit_exact(fmt, sigma, dev):
    rng = np.random.default_rng(sigma)
    rp, cols, vals = _csr(rng, _lens(rng, 700, 120), 3000, signed=True)
    _say("sell decode", fmt, sigma, rp[-1])
    for idx in ("i32", "u16"):
        S = dm.SellMatrix(rp, cols, vals, 3000, fmt, sigma=sigma, index_format=idx)
        perm, width, val, col = S.decode()
        dec, _ = oracle.decode_matrix(fmt, rp, vals)
        perm_o, width_o = oracle.sell_layout(rp, 64, sigma)
        val_o, col_o = oracle.sell_pack(rp, cols, dec, 64, perm_o, width_o)
        assert np.array_equal(perm, perm_o) and np.array_equal(width, width_o)
        assert np.array_equal(col, col_o)
        assert np.array_equal(_bits(val), _bits(val_o))
        inf = S.info()
        assert inf["std_slots"] == 64 * width_o.sum()
        assert inf["stored_slots"] == 512 * int(((width_o + 7) // 8).sum())
        S.close()


@pytest.mark.parametrize("fmt", FORMATS)
@pytest.mark.parametrize("sigma", [1, 64, 256, 300])
def test_product_against_oracle(fmt, sigma, dev):
    rng = np.random.default_rng(100 + sigma)
    n_rows, n_cols = 2000 + sigma, 4000
    rp, cols, vals = _csr(rng, _lens(rng, n_rows, 400), n_cols, span=1500)
    x = dosegen.spot_weights(7, sigma, n_cols)
    S = dm.SellMatrix(rp, cols, vals, n_cols, fmt, sigma=sigma)
    y = S.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
    dec, _ = oracle.decode_matrix(fmt, rp, vals)
    perm, width = oracle.sell_layout(rp, 64, sigma)
    sval, scol = oracle.sell_pack(rp, cols, dec, 64, perm, width)
    y_ref = oracle.sell_spmv(n_rows, 64, perm, width, sval, scol, x)
    assert np.array_equal(y_ref, oracle.spmv(rp, cols, dec, x))
    err = oracle.max_rel_err(y, y_ref)
    _say(f"sell {fmt} sigma {sigma}: max rel err {err:.3e}, windowed {S.info()['n_groups_windowed']}/{S.info()['n_groups']}")
    assert err <= TOL
    assert np.all(_bits(y[np.diff(rp) == 0]) == 0)
    # bitwise repeatable
    y2 = S.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.array_equal(_bits(y), _bits(y2))
    S.close()


def test_signed_values_scaled_error(dev):
    rng = np.random.default_rng(3)
    rp, cols, vals = _csr(rng, _lens(rng, 3000, 300), 5000, signed=True, span=2000)
    x = dosegen.signed_values(9, 0, 5000)
    for fmt in FORMATS:
        S = dm.SellMatrix(rp, cols, vals, 5000, fmt, sigma=128)
        y = S.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
        dec, _ = oracle.decode_matrix(fmt, rp, vals)
        y_ref = oracle.spmv(rp, cols, dec, x)
        scale = oracle.spmv(rp, cols, np.abs(dec), np.abs(x))
        err = oracle.max_scaled_err(y, y_ref, scale)
        assert err <= TOL, (fmt, err)
        S.close()


def test_exact_inputs_equal_csr_and_oracle(dev):
    # dyadic values with 3 significant bits and small integer x: every FP32
    # sum is exact, so any order gives the oracle's value
    rng = np.random.default_rng(11)
    n_rows, n_cols = 1500, 2000
    lens = _lens(rng, n_rows, 600)
    rp = np.zeros(n_rows + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    cols = np.concatenate([np.sort(rng.choice(n_cols, L, replace=False)) for L in lens if L]).astype(np.int32)
    vals = (rng.integers(1, 8, rp[-1]) * 2.0 ** -rng.integers(0, 4, rp[-1])).astype(np.float32)
    x = rng.integers(0, 9, n_cols).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    for fmt in ("fp16", "bf16", "fp32"):
        S = dm.SellMatrix(rp, cols, vals, n_cols, fmt, sigma=256)
        A = dm.DoseMatrix(rp, cols, vals, n_cols, fmt)
        y = S.spmv(xd).cpu().numpy()
        assert np.array_equal(_bits(y), _bits(A.spmv(xd).cpu().numpy()))
        dec, _ = oracle.decode_matrix(fmt, rp, vals)
        assert np.array_equal(y.astype(np.float64), oracle.spmv(rp, cols, dec, x))
        S.close()
        A.close()


def test_u16_equals_i32_and_window_equals_global(dev):
    rng = np.random.default_rng(12)
    n_cols = 60000
    # rows 0..1999 narrow (LDS windows), rows 2000..3999 spread over all
    # columns (windows beyond the LDS cap: global gathers)
    lens = _lens(rng, 4000, 300)
    rp_a, cols_a, vals_a = _csr(rng, lens[:2000], n_cols, span=1000, shift=2)
    rp_b, cols_b, vals_b = _csr(rng, lens[2000:], n_cols)
    rp = np.concatenate([rp_a, rp_a[-1] + rp_b[1:]])
    cols = np.concatenate([cols_a, cols_b])
    vals = np.concatenate([vals_a, vals_b])
    x = dosegen.spot_weights(13, 0, n_cols)
    xd = torch.from_numpy(x).cuda()
    S32 = dm.SellMatrix(rp, cols, vals, n_cols, "fp16", sigma=256)
    S16 = dm.SellMatrix(rp, cols, vals, n_cols, "fp16", sigma=256, index_format="u16")
    inf = S32.info()
    assert 0 < inf["n_groups_windowed"] < inf["n_groups"]
    y32 = S32.spmv(xd).cpu().numpy()
    y16 = S16.spmv(xd).cpu().numpy()
    assert np.array_equal(_bits(y32), _bits(y16))
    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    assert oracle.max_rel_err(y32, oracle.spmv(rp, cols, dec, x)) <= TOL
    S32.close()
    S16.close()


def test_long_rows_error_bound(dev):
    # rows up to 16,000 entries (the paper's longest, Sec. IV) beside short
    # ones: the inner/outer slice sums keep the error far inside 1e-5
    rng = np.random.default_rng(14)
    lens = _lens(rng, 600, 200)
    lens[::50] = 16000
    lens[7] = 15999
    rp, cols, vals = _csr(rng, lens, 25000)
    x = dosegen.spot_weights(15, 0, 25000)
    for fmt in ("fp16", "fp8e4m3_rowscale"):
        S = dm.SellMatrix(rp, cols, vals, 25000, fmt, sigma=64)
        y = S.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
        dec, _ = oracle.decode_matrix(fmt, rp, vals)
        err = oracle.max_rel_err(y, oracle.spmv(rp, cols, dec, x))
        _say(f"sell long rows {fmt}: {err:.3e}")
        assert err <= 3e-6
        S.close()


def test_empty_cases(dev):
    for lens, n_cols in (([], 10), ([0, 0, 0], 10), ([0] * 300, 1)):
        rp = np.zeros(len(lens) + 1, np.int64)
        cols = np.zeros(0, np.int32)
        vals = np.zeros(0, np.float32)
        S = dm.SellMatrix(rp, cols, vals, n_cols, "fp16")
        y = torch.full((len(lens),), np.nan, device=dev)
        S.spmv(torch.ones(n_cols, device=dev), y)
        assert np.all(_bits(y.cpu().numpy()) == 0)
        perm, width, val, col = S.decode()
        assert perm.tolist() == list(range(len(lens))) and val.size == 0
        S.close()


def test_argument_errors(dev):
    rp = np.array([0, 2, 3], np.int64)
    cols = np.array([0, 4, 1], np.int32)
    vals = np.ones(3, np.float32)
    with pytest.raises(dm.DoseError):
        dm.SellMatrix(rp, cols, vals, 5, "fp16", sigma=0)
    with pytest.raises(dm.DoseError):
        dm.SellMatrix(rp, np.array([4, 0, 1], np.int32), vals, 5, "fp16")  # unsorted columns
    S = dm.SellMatrix(rp, cols, vals, 5, "fp16")
    with pytest.raises(ValueError):
        S.spmv(torch.ones(4, device=dev))
    S.close()


def test_clinical_beam_sampled(dev):
    """The clinical-scale beam (2,097,152 x 25,000, 4.2e8 entries) in SELL
    form, every value format with int32 indices, on a 1% row sample
    (stratified to hold the longest and some empty rows) against the oracle."""
    spec = dosegen.clinical_beam()
    rp, cols, vals = dosegen.csr(spec)
    lens = np.diff(rp)
    rng = np.random.default_rng(2105)
    rows = np.unique(np.concatenate([np.argsort(lens, kind="stable")[-200:],
                                     rng.integers(0, lens.size, lens.size // 100),
                                     np.nonzero(lens == 0)[0][:200]]))
    sl = np.repeat(rp[rows], lens[rows]) + (np.arange(lens[rows].sum()) - np.repeat(np.cumsum(lens[rows]) - lens[rows], lens[rows]))
    srp = np.zeros(rows.size + 1, np.int64)
    np.cumsum(lens[rows], out=srp[1:])
    x = dosegen.spot_weights(spec.seed, 0, spec.n_cols)
    for fmt in ("fp16", "fp8e4m3_rowscale"):
        S = dm.SellMatrix(rp, cols, vals, spec.n_cols, fmt, sigma=256)
        y = S.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
        dec, _ = oracle.decode_matrix(fmt, srp, vals[sl])
        err = oracle.max_rel_err(y[rows], oracle.spmv(srp, cols[sl], dec, x))
        inf = S.info()
        _say(f"sell clinical {fmt}: max rel err {err:.3e} on {rows.size} rows; padding "
             f"{inf['stored_slots'] / max(inf['nnz'], 1) - 1:.3%}, windowed {inf['n_groups_windowed']}/{inf['n_groups']}")
        assert err <= TOL
        assert np.all(_bits(y[lens == 0]) == 0)
        S.close()


# ---------------------------------------------------------------- run-length indices
def _ray_matrix(seed, n_rows=3000, n_cols=6000):
    """Rows of 2-4 runs of consecutive columns (short and long runs, runs of
    one entry, rows ending mid-slice), some empty rows, run starts near a
    drifting centre so that groups have narrow windows."""
    rng = np.random.default_rng(seed)
    rp = [0]
    cols = []
    for i in range(n_rows):
        if rng.random() < 0.3:
            rp.append(rp[-1])
            continue
        centre = (i * 3) % (n_cols - 1200)
        row = []
        c = centre
        for _ in range(rng.integers(2, 5)):
            c += int(rng.integers(1, 60))
            L = int(rng.choice([1, 2, 3, 7, 8, 9, 31, 33, 120, 250]))
            row.extend(range(c, c + L))
            c += L
        row = sorted(set(x for x in row if x < n_cols))
        cols.extend(row)
        rp.append(rp[-1] + len(row))
    rp = np.array(rp, np.int64)
    cols = np.array(cols, np.int32)
    vals = np.exp(rng.normal(-3, 1, cols.size)).astype(np.float32)
    return rp, cols, vals, n_cols


@pytest.mark.parametrize("sigma", [1, 64, 256])
def test_runs_read_back_equal_oracle(sigma, dev):
    for rp, cols, vals, n_cols in (_ray_matrix(20 + sigma),
                                   (*dosegen.csr(dosegen.small_plain()), dosegen.small_plain().n_cols)):
        S = dm.SellMatrix(rp, cols, vals, n_cols, "fp16", sigma=sigma, index_format="runs")
        run_ptr, start, length = S.runs()
        run_ptr_o, start_o, length_o = oracle.runs_encode(rp, cols)
        assert np.array_equal(run_ptr, run_ptr_o)
        assert np.array_equal(start, start_o) and np.array_equal(length, length_o)
        assert S.info()["n_runs"] == start_o.size
        # Kreutzer's layout with the columns rebuilt from the device's runs
        perm, width, val, col = S.decode()
        dec, _ = oracle.decode_matrix("fp16", rp, vals)
        perm_o, width_o = oracle.sell_layout(rp, 64, sigma)
        val_o, col_o = oracle.sell_pack(rp, cols, dec, 64, perm_o, width_o)
        assert np.array_equal(col, col_o) and np.array_equal(_bits(val), _bits(val_o))
        S.close()


@pytest.mark.parametrize("fmt", FORMATS)
def test_runs_product_equals_i32_bitwise(fmt, dev):
    rp, cols, vals, n_cols = _ray_matrix(31)
    x = dosegen.spot_weights(32, 0, n_cols)
    xd = torch.from_numpy(x).cuda()
    for sigma in (1, 256):
        S32 = dm.SellMatrix(rp, cols, vals, n_cols, fmt, sigma=sigma)
        SR = dm.SellMatrix(rp, cols, vals, n_cols, fmt, sigma=sigma, index_format="runs")
        y32 = S32.spmv(xd).cpu().numpy()
        yr = SR.spmv(xd).cpu().numpy()
        assert np.array_equal(_bits(yr), _bits(y32)), (fmt, sigma)
        dec, _ = oracle.decode_matrix(fmt, rp, vals)
        assert oracle.max_rel_err(yr, oracle.spmv(rp, cols, dec, x)) <= TOL
        S32.close()
        SR.close()


def test_runs_window_and_global_groups(dev):
    # the ray rows (LDS windows) followed by rows whose runs sit far apart
    # (windows beyond the LDS cap: x gathered from global memory); long rows
    rp_a, cols_a, vals_a, n_cols = _ray_matrix(41, n_rows=2000, n_cols=60000)
    rng = np.random.default_rng(42)
    rows = []
    for i in range(1500):
        starts = np.sort(rng.choice(np.arange(0, 59000, 500), size=3, replace=False))
        L = int(rng.choice([5, 40, 300]))
        rows.append(np.concatenate([np.arange(s, s + L) for s in starts]))
    rows[10] = np.arange(100, 16100)  # one long run of 16,000
    rows[20] = np.concatenate([np.arange(0, 8000), np.arange(20000, 28000)])
    lens_b = np.array([r.size for r in rows])
    rp_b = np.concatenate([[0], np.cumsum(lens_b)])
    cols_b = np.concatenate(rows).astype(np.int32)
    vals_b = np.exp(rng.normal(-3, 1, cols_b.size)).astype(np.float32)
    rp = np.concatenate([rp_a, rp_a[-1] + rp_b[1:]])
    cols = np.concatenate([cols_a, cols_b])
    vals = np.concatenate([vals_a, vals_b])
    x = dosegen.spot_weights(43, 0, n_cols)
    xd = torch.from_numpy(x).cuda()
    S32 = dm.SellMatrix(rp, cols, vals, n_cols, "fp16", sigma=256)
    SR = dm.SellMatrix(rp, cols, vals, n_cols, "fp16", sigma=256, index_format="runs")
    inf = SR.info()
    assert 0 < inf["n_groups_windowed"] < inf["n_groups"]
    yr = SR.spmv(xd).cpu().numpy()
    assert np.array_equal(_bits(yr), _bits(S32.spmv(xd).cpu().numpy()))
    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    assert oracle.max_rel_err(yr, oracle.spmv(rp, cols, dec, x)) <= TOL
    S32.close()
    SR.close()


def test_runs_limits(dev):
    # columns with no runs: 64 rows of 20 scattered entries exceed 1024 runs
    rng = np.random.default_rng(50)
    rp, cols, vals = _csr(rng, np.full(256, 20), 60000)
    with pytest.raises(dm.DoseError) as e:
        dm.SellMatrix(rp, cols, vals, 60000, "fp16", index_format="runs")
    assert e.value.code == dm._lib.ERR_UNSUPPORTED
    with pytest.raises(dm.DoseError) as e:
        dm.DoseMatrix(rp, cols, vals, 60000, "fp16", index_format="runs")
    assert e.value.code == dm._lib.ERR_UNSUPPORTED
    # an empty matrix and rows without entries
    for n in (0, 100):
        S = dm.SellMatrix(np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 10, "fp16",
                          index_format="runs")
        y = torch.full((n,), np.nan, device=dev)
        S.spmv(torch.ones(10, device=dev), y)
        assert np.all(_bits(y.cpu().numpy()) == 0)
        assert S.runs()[0].tolist() == [0] * (n + 1)
        S.close()
