"""GPU parity of the multi-vector and batched SELL-C-sigma products.

* dose_sell_spmv_multi with 2 and 4 vectors: every column of Y is bit for bit
  the single-vector SELL product of the same column of X, in every value and
  index format, for groups through the LDS window, groups gathering x from
  global memory, and groups whose window fits one vector but not four; the
  columns are within 1e-5 of the oracle; empty rows get +0 in every column.
* dose_sell_batch_plan_create: one launch over the chunks of several
  matrices (ragged sizes, a matrix without entries, one without rows) equals
  the per-matrix products bit for bit on every replay of its graph, with
  eager work between the replays; argument errors are reported.
* The clinical beam (2,097,152 x 25,000) with run-length indices and four
  vectors: bitwise equal to four single-vector products, sampled rows within
  1e-5 of the oracle.
"""
import ctypes

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


def _rows(rng, n, n_cols, span, shift, max_len=300, empty=0.3):
    """CSR rows of random lengths, each drawn from a window of `span`
    columns moving by `shift` per row (span None: all columns)."""
    lens = rng.integers(1, max_len, n)
    lens[rng.random(n) < empty] = 0
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    cols = np.empty(rp[-1], np.int32)
    for i, L in enumerate(lens):
        if L:
            if span is None:
                cols[rp[i]:rp[i + 1]] = np.sort(rng.choice(n_cols, size=L, replace=False))
            else:
                lo = (i * shift) % max(1, n_cols - span)
                cols[rp[i]:rp[i + 1]] = lo + np.sort(rng.choice(span, size=L, replace=False))
    return rp, cols


def _concat(parts):
    rp = [np.zeros(1, np.int64)]
    cols = []
    base = 0
    for r, c in parts:
        rp.append(r[1:] + base)
        cols.append(c)
        base += int(r[-1])
    return np.concatenate(rp), np.concatenate(cols).astype(np.int32)


def _mixed_matrix(seed, n_cols=60000):
    """Row blocks whose 64-row chunks have narrow windows (LDS for 1 and 4
    vectors), windows of about 3,500 columns (LDS for one vector, beyond the
    four-vector cap: global gathers), and rows spread over all columns."""
    rng = np.random.default_rng(seed)
    rp, cols = _concat([_rows(rng, 1500, n_cols, 1000, 2),
                        _rows(rng, 700, n_cols, 3500, 0),
                        _rows(rng, 700, n_cols, None, 0)])
    vals = np.exp(rng.normal(-3, 1, cols.size)).astype(np.float32)
    vals[rng.random(vals.size) < 0.2] *= -1
    return rp, cols, vals, n_cols


def _ray_matrix(seed, n_rows=3000, n_cols=8000):
    """Rows of 2-4 runs of consecutive columns near a drifting centre."""
    rng = np.random.default_rng(seed)
    rp = [0]
    cols = []
    for i in range(n_rows):
        if rng.random() < 0.3:
            rp.append(rp[-1])
            continue
        c = (i * 3) % (n_cols - 1500)
        row = []
        for _ in range(rng.integers(2, 5)):
            c += int(rng.integers(1, 60))
            L = int(rng.choice([1, 2, 3, 7, 8, 9, 31, 33, 120, 250]))
            row.extend(range(c, c + L))
            c += L
        row = sorted(set(v for v in row if v < n_cols))
        cols.extend(row)
        rp.append(rp[-1] + len(row))
    rp = np.array(rp, np.int64)
    cols = np.array(cols, np.int32)
    vals = np.exp(rng.normal(-3, 1, cols.size)).astype(np.float32)
    return rp, cols, vals, n_cols


def _xs(seed, n_cols, n_rhs):
    return np.stack([dosegen.spot_weights(seed, r, n_cols) for r in range(n_rhs)], 1)


def _check_columns(S, X, Y):
    """Every column of Y equals the single-vector product of X's column."""
    for r in range(X.shape[1]):
        y1 = S.spmv(X[:, r].contiguous()).cpu().numpy()
        assert np.array_equal(_bits(Y[:, r]), _bits(y1)), r


@pytest.mark.parametrize("fmt", FORMATS)
@pytest.mark.parametrize("idx", ["i32", "u16", "runs"])
def test_multi_equals_single_bitwise(fmt, idx, dev):
    if idx == "runs":
        rp, cols, vals, n_cols = _ray_matrix(60)
    else:
        rp, cols, vals, n_cols = _mixed_matrix(61)  # 60,000 columns: 16-bit indices hold them
    S = dm.SellMatrix(rp, cols, vals, n_cols, fmt, sigma=256, index_format=idx)
    inf = S.info()
    _say(f"sell multi {fmt} {idx}: nnz {inf['nnz']}, windowed {inf['n_groups_windowed']}/{inf['n_groups']}")
    dec, _ = oracle.decode_matrix(fmt, rp, vals)
    empty = np.diff(rp) == 0
    for n_rhs in (2, 4):
        X = torch.from_numpy(_xs(70 + n_rhs, n_cols, n_rhs)).cuda().contiguous()
        Y = torch.full((S.n_rows, n_rhs), np.nan, device=dev)
        S.spmv(X, Y)
        Yh = Y.cpu().numpy()
        _check_columns(S, X, Yh)
        assert np.all(_bits(Yh[empty]) == 0)
        xh = X.cpu().numpy()
        for r in range(n_rhs):
            y_ref = oracle.spmv(rp, cols, dec, xh[:, r])
            scale = oracle.spmv(rp, cols, np.abs(dec), np.abs(xh[:, r]))
            assert oracle.max_scaled_err(Yh[:, r], y_ref, scale) <= TOL
    S.close()


def test_multi_window_switch(dev):
    # chunks of about 3,500 columns: through LDS for one vector, gathered
    # from global memory for four; the bits do not depend on it
    rp, cols, vals, n_cols = _mixed_matrix(62)
    S = dm.SellMatrix(rp, cols, vals, n_cols, "fp16", sigma=1)
    X = torch.from_numpy(_xs(80, n_cols, 4)).cuda().contiguous()
    Y = S.spmv(X).cpu().numpy()
    _check_columns(S, X, Y)
    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    x0 = X[:, 0].cpu().numpy()
    scale = oracle.spmv(rp, cols, np.abs(dec), np.abs(x0))
    assert oracle.max_scaled_err(Y[:, 0], oracle.spmv(rp, cols, dec, x0), scale) <= TOL
    S.close()


def test_multi_exact_inputs_equal_oracle(dev):
    # dyadic values and small integer x: every FP32 sum is exact
    rng = np.random.default_rng(63)
    rp, cols = _rows(rng, 1200, 3000, 800, 2, max_len=700)
    vals = (rng.integers(1, 8, cols.size) * 2.0 ** -rng.integers(0, 4, cols.size)).astype(np.float32)
    X = rng.integers(0, 9, (3000, 4)).astype(np.float32)
    for idx in ("i32", "u16"):
        S = dm.SellMatrix(rp, cols, vals, 3000, "fp16", sigma=64, index_format=idx)
        Y = S.spmv(torch.from_numpy(X).cuda()).cpu().numpy()
        for r in range(4):
            assert np.array_equal(Y[:, r].astype(np.float64), oracle.spmv(rp, cols, vals.astype(np.float64), X[:, r]))
        S.close()


def test_multi_empty_and_errors(dev):
    for n in (0, 100):
        S = dm.SellMatrix(np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 10, "fp16")
        Y = torch.full((n, 4), np.nan, device=dev)
        S.spmv(torch.ones(10, 4, device=dev), Y)
        assert np.all(_bits(Y.cpu().numpy()) == 0)
        S.close()
    rp, cols, vals, n_cols = _ray_matrix(64, n_rows=300, n_cols=3000)
    S = dm.SellMatrix(rp, cols, vals, n_cols, "fp16", index_format="runs")
    lib = dm._lib.load()
    X = torch.ones(n_cols * 4 + 1, device=dev)
    Y = torch.empty(S.n_rows * 4 + 1, device=dev)
    # three vectors: unsupported
    assert lib.dose_sell_spmv_multi(S.handle, 3, X.data_ptr(), Y.data_ptr(), None) == dm._lib.ERR_UNSUPPORTED
    # x not aligned to four floats
    assert lib.dose_sell_spmv_multi(S.handle, 4, X.data_ptr() + 4, Y.data_ptr(), None) == \
        dm._lib.ERR_INVALID_ARGUMENT
    # x and y overlap
    assert lib.dose_sell_spmv_multi(S.handle, 4, X.data_ptr(), X.data_ptr(), None) == dm._lib.ERR_INVALID_ARGUMENT
    assert lib.dose_sell_spmv_multi(S.handle, 4, None, Y.data_ptr(), None) == dm._lib.ERR_INVALID_ARGUMENT
    with pytest.raises(ValueError):
        S.spmv(torch.ones(n_cols, 4, device=dev), torch.empty(S.n_rows, 2, device=dev))
    S.close()


def _batch(dev, idx, n_rhs):
    """Five matrices of different sizes and windows, one without entries and
    one without rows."""
    mats, ents = [], []
    specs = [_ray_matrix(90, 2500, 6000), _ray_matrix(91, 700, 9000), _ray_matrix(92, 4000, 5000)]
    if idx != "runs":
        specs[1] = _mixed_matrix(93)
    specs.append((np.zeros(301, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 50))
    specs.append((np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 20))
    for k, (rp, cols, vals, n_cols) in enumerate(specs):
        S = dm.SellMatrix(rp, cols, vals, n_cols, "fp16", sigma=256, index_format=idx)
        X = torch.from_numpy(_xs(100 + k, n_cols, n_rhs)).cuda().contiguous()
        if n_rhs == 1:
            X = X[:, 0].contiguous()
        Y = torch.full((S.n_rows, n_rhs) if n_rhs > 1 else (S.n_rows,), np.nan, device=dev)
        mats.append(S)
        ents.append((S, X, Y))
    return mats, ents


@pytest.mark.parametrize("idx", ["i32", "runs"])
@pytest.mark.parametrize("n_rhs", [1, 4])
def test_batch_plan_equals_products(idx, n_rhs, dev):
    mats, ents = _batch(dev, idx, n_rhs)
    refs = [S.spmv(X).cpu().numpy() for S, X, _ in ents]
    plan = dm.SellBatchPlan(ents)
    for rep in range(3):
        for _, _, Y in ents:
            Y.fill_(np.nan)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for k, (_, _, Y) in enumerate(ents):
            assert np.array_equal(_bits(Y.cpu().numpy()), _bits(refs[k])), (rep, k)
        # eager work between the replays
        z = torch.randn(1 << 20, device=dev)
        (z * 2).sum().item()
    plan.close()
    for S in mats:
        S.close()


def test_batch_plan_errors(dev):
    mats, ents = _batch(dev, "i32", 4)
    rp, cols, vals, n_cols = _ray_matrix(95, 500, 4000)
    other = dm.SellMatrix(rp, cols, vals, n_cols, "bf16", sigma=256)
    runs = dm.SellMatrix(rp, cols, vals, n_cols, "fp16", sigma=256, index_format="runs")
    X = torch.from_numpy(_xs(96, n_cols, 4)).cuda().contiguous()
    for bad in ((other, X, torch.empty(other.n_rows, 4, device=dev)),
                (runs, X, torch.empty(runs.n_rows, 4, device=dev))):
        with pytest.raises(dm.DoseError) as e:
            dm.SellBatchPlan(ents[:2] + [bad])
        assert e.value.code == dm._lib.ERR_UNSUPPORTED
    S0, X0, Y0 = ents[0]
    S1, X1, _ = ents[1]
    # two items share an output
    Ys = torch.empty(max(S0.n_rows, S1.n_rows) * 4, device=dev)
    with pytest.raises(dm.DoseError) as e:
        dm.SellBatchPlan([(S0, X0, Ys[:S0.n_rows * 4].view(S0.n_rows, 4)),
                          (S1, X1, Ys[:S1.n_rows * 4].view(S1.n_rows, 4))])
    assert e.value.code == dm._lib.ERR_INVALID_ARGUMENT
    # one item's y is another item's x
    Yx = torch.empty(max(S0.n_cols, S1.n_rows) * 4, device=dev)
    with pytest.raises(dm.DoseError) as e:
        dm.SellBatchPlan([(S0, Yx[:S0.n_cols * 4].view(S0.n_cols, 4), Y0),
                          (S1, X1, Yx[:S1.n_rows * 4].view(S1.n_rows, 4))])
    assert e.value.code == dm._lib.ERR_INVALID_ARGUMENT
    # mixed n_rhs
    with pytest.raises(dm.DoseError) as e:
        dm.SellBatchPlan([ents[0], (S1, X1[:, 0].contiguous(), torch.empty(S1.n_rows, device=dev))])
    assert e.value.code == dm._lib.ERR_UNSUPPORTED
    # unknown flags
    lib = dm._lib.load()
    arr = (dm._lib.SellBatchItem * 1)()
    arr[0] = dm._lib.SellBatchItem(S0.handle, 4, 0, X0.data_ptr(), 4, Y0.data_ptr(), 4)
    h = ctypes.c_void_p()
    assert lib.dose_sell_batch_plan_create(arr, 1, 1, None, ctypes.byref(h)) == dm._lib.ERR_INVALID_ARGUMENT
    assert lib.dose_sell_batch_plan_create(arr, 0, 0, None, ctypes.byref(h)) == dm._lib.ERR_INVALID_ARGUMENT
    other.close()
    runs.close()
    for S in mats:
        S.close()


def test_clinical_beam_four_vectors(dev):
    """The clinical beam with run-length indices and four spot-weight
    vectors: bitwise the four single-vector products; a 1% row sample
    (with the longest rows) within 1e-5 of the oracle in every column."""
    spec = dosegen.clinical_beam()
    rp, cols, vals = dosegen.csr(spec)
    S = dm.SellMatrix(rp, cols, vals, spec.n_cols, "fp16", sigma=65536, index_format="runs")
    X = torch.from_numpy(_xs(spec.seed, spec.n_cols, 4)).cuda().contiguous()
    Y = S.spmv(X).cpu().numpy()
    _check_columns(S, X, Y)
    lens = np.diff(rp)
    rng = np.random.default_rng(2106)
    rows = np.unique(np.concatenate([np.argsort(lens, kind="stable")[-200:],
                                     rng.integers(0, lens.size, lens.size // 100),
                                     np.nonzero(lens == 0)[0][:200]]))
    sl = np.repeat(rp[rows], lens[rows]) + (np.arange(lens[rows].sum()) -
                                            np.repeat(np.cumsum(lens[rows]) - lens[rows], lens[rows]))
    srp = np.zeros(rows.size + 1, np.int64)
    np.cumsum(lens[rows], out=srp[1:])
    dec, _ = oracle.decode_matrix("fp16", srp, vals[sl])
    xh = X.cpu().numpy()
    for r in range(4):
        err = oracle.max_rel_err(Y[rows, r], oracle.spmv(srp, cols[sl], dec, xh[:, r]))
        _say(f"sell clinical 4 vectors, column {r}: max rel err {err:.3e} on {rows.size} rows")
        assert err <= TOL
    assert np.all(_bits(Y[lens == 0]) == 0)
    S.close()
