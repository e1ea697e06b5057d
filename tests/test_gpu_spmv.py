"""GPU parity of the forward dose product d = A x against the CPU oracle.

Tolerance: max relative error 1e-5 per voxel (FP32 accumulation against the
FP64 oracle on the same decoded values); rows whose exact dose is 0 must hold
exactly +0.  Decoding is compared bit for bit.
"""
import numpy as np
import pytest
import torch

import dosegen
import oracle
import paper_2103_09683_amd as dm

pytestmark = pytest.mark.gpu

FORMATS = ["fp16", "bf16", "fp8e4m3_rowscale"]
TOL = 1e-5


def _say(*a):
    print(*a, flush=True)


def _bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def _csr_from_lens(rng, lens, n_cols, signed=False, special=False):
    rp = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    cols = np.empty(rp[-1], np.int32)
    for i, L in enumerate(lens):
        if L:
            cols[rp[i]:rp[i + 1]] = np.sort(rng.choice(n_cols, size=L, replace=False))
    vals = np.exp(rng.normal(-3, 1, size=rp[-1])).astype(np.float32)
    if signed:
        vals[rng.random(vals.size) < 0.4] *= -1
    if special and vals.size > 64:
        # FP16 subnormals and values at FP16 / BF16 rounding ties
        vals[:16] = (np.arange(1, 17) * 2.0 ** -24).astype(np.float32)
        vals[16:32] = np.float32(1.0 + 2.0 ** -11) * np.arange(1, 17, dtype=np.float32)
        vals[32:48] = np.float32(1.0 + 2.0 ** -8)
        vals[48:64] = np.float32(6.1e-5)
    return rp, cols, vals


def _check_forward(A, rp, cols, vals, fmt, x, tol=TOL):
    y = A.spmv(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    dec, _ = oracle.decode_matrix(fmt, rp, vals)
    y_ref = oracle.spmv(rp, cols, dec, x)
    y_h = y.cpu().numpy()
    if np.all(vals >= 0) and np.all(x >= 0):
        err = oracle.max_rel_err(y_h, y_ref)
    else:
        scale = oracle.spmv(rp, cols, np.abs(dec), np.abs(x))
        err = oracle.max_scaled_err(y_h, y_ref, scale)
    assert err <= tol, (fmt, err)
    return y_h, y_ref


@pytest.mark.parametrize("fmt", FORMATS)
def test_decode_bit_exact(fmt, dev):
    rng = np.random.default_rng(1)
    lens = rng.integers(0, 300, size=700)
    lens[::9] = 0
    rp, cols, vals = _csr_from_lens(rng, lens, 3000, signed=True, special=True)
    _say("decode", fmt, rp[-1])
    A = dm.DoseMatrix(rp, cols, vals, 3000, fmt)
    rp_d, cols_d, vals_d = A.decode()
    dec, _ = oracle.decode_matrix(fmt, rp, vals)
    np.testing.assert_array_equal(rp_d, rp)
    np.testing.assert_array_equal(cols_d, cols)
    np.testing.assert_array_equal(_bits(vals_d), _bits(dec))
    # a sub-range of rows
    rp_s, cols_s, vals_s = A.decode(100, 250)
    np.testing.assert_array_equal(_bits(vals_s), _bits(dec[rp[100]:rp[250]]))
    np.testing.assert_array_equal(rp_s, rp[100:251] - rp[100])
    A.close()


@pytest.mark.parametrize("fmt", FORMATS)
def test_small_plain_parity(fmt, dev):
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    x = dosegen.spot_weights(spec.seed, 0, spec.n_cols)
    _say("small_plain", fmt)
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, fmt)
    _check_forward(A, rp, cols, vals, fmt, x)
    A.close()


@pytest.mark.parametrize("fmt", FORMATS)
def test_partitions_long_rows_and_ragged_tail(fmt, dev):
    """Rows from 1 to 20,000 entries (many 512-entry steps), empty runs, a
    ragged last row; the product is checked under several partitions and must
    be bitwise the same under all of them (each row's summation order is its
    own)."""
    rng = np.random.default_rng(11)
    lens = rng.integers(0, 700, size=3001)
    lens[rng.random(lens.size) < 0.5] = 0
    lens[[5, 1000, 3000]] = [20000, 4089, 9999]  # long rows
    lens[1001:1010] = 1                           # short rows
    lens[2000:2300] = 0                           # a run of empty rows
    rp, cols, vals = _csr_from_lens(rng, lens, 20000, signed=True)
    x = rng.uniform(-1, 1, 20000).astype(np.float32)
    A = dm.DoseMatrix(rp, cols, vals, 20000, fmt)
    ys, splits = [], []
    for group_nnz in (1024, 4096, 32768, 1 << 20):
        _say("partition", fmt, group_nnz, rp[-1])
        A.set_partition(group_nnz)
        assert A.info()["group_nnz"] == group_nnz
        splits.append(A.info()["n_groups_split"])
        ys.append(_check_forward(A, rp, cols, vals, fmt, x)[0])
    # the long rows are split groups (shared by four waves) or one wave's rows
    assert splits == [3, 3, 2, 0]
    for y in ys[1:]:
        np.testing.assert_array_equal(_bits(y), _bits(ys[0]))
    A.close()


def test_create_autotune(tmp_path, monkeypatch, dev):
    """DOSE_CREATE_AUTOTUNE picks a row-group size from the timed candidates
    for A and A^T; the products are bitwise those of the default partition;
    the choice is written to and read back from DOSE_TUNE_CACHE; unknown
    create flags are refused."""
    monkeypatch.setenv("DOSE_TUNE_CACHE", str(tmp_path / "tune.txt"))
    rng = np.random.default_rng(12)
    lens = rng.integers(0, 700, size=40000)
    lens[rng.random(lens.size) < 0.5] = 0
    rp, cols, vals = _csr_from_lens(rng, lens, 6000)
    x = torch.from_numpy(rng.uniform(0, 1, 6000).astype(np.float32)).cuda()
    v = torch.from_numpy(rng.uniform(-1, 1, lens.size).astype(np.float32)).cuda()
    A0 = dm.DoseMatrix(rp, cols, vals, 6000, "fp16", transpose=True)
    for rep in range(2):
        _say("autotuned create", rep)
        A1 = dm.DoseMatrix(rp, cols, vals, 6000, "fp16", transpose=True, autotune=True)
        inf = A1.info()
        assert inf["group_nnz"] in (8192, 16384, 32768, 65536)
        assert inf["group_nnz_t"] in (8192, 16384, 32768, 65536)
        assert np.array_equal(_bits(A1.spmv(x).cpu().numpy()), _bits(A0.spmv(x).cpu().numpy()))
        assert np.array_equal(_bits(A1.adjoint(v).cpu().numpy()), _bits(A0.adjoint(v).cpu().numpy()))
        A1.close()
    assert len((tmp_path / "tune.txt").read_text().split()) == 4  # two keys, each stored once
    c, keep = dm._csr_struct(rp, cols, vals, 6000)
    h = dm.ctypes.c_void_p()
    # 8: the lowest bit no create flag uses
    assert dm._lib.load().dose_matrix_create(dm.ctypes.byref(c), dm._lib.VAL_FP16, dm._lib.IDX_I32, 8, None,
                                             dm.ctypes.byref(h)) == dm._lib.ERR_INVALID_ARGUMENT
    A0.close()


def test_rows_across_many_row_windows(dev):
    """A wave lists its rows 64 at a time; with short rows and large groups
    each wave walks many such windows, and the first non-empty row of every
    window must start from a clean sum (regression: a finished window once
    leaked its last step into the next window's first row)."""
    rng = np.random.default_rng(13)
    lens = rng.integers(1, 40, size=40000)
    lens[rng.random(lens.size) < 0.5] = 0
    lens[64::64] = 7   # a non-empty row at many window starts
    rp, cols, vals = _csr_from_lens(rng, lens, 3000)
    x = rng.uniform(0, 1, 3000).astype(np.float32)
    for fmt in FORMATS:
        A = dm.DoseMatrix(rp, cols, vals, 3000, fmt)
        ys = []
        for group_nnz in (1024, 65536, 1 << 20):
            _say("row windows", fmt, group_nnz)
            A.set_partition(group_nnz)
            ys.append(_check_forward(A, rp, cols, vals, fmt, x)[0])
        for y in ys[1:]:
            np.testing.assert_array_equal(_bits(y), _bits(ys[0]))
        A.close()


def test_many_tiny_rows_per_step(dev):
    """Rows of 1..8 entries packed densely: a 512-entry step then meets up to
    hundreds of rows and crosses several 64-row windows, and rows start at
    every offset of a step's quarters."""
    rng = np.random.default_rng(14)
    lens = rng.integers(1, 9, size=30000)
    lens[rng.random(lens.size) < 0.1] = 0
    rp, cols, vals = _csr_from_lens(rng, lens, 1000, signed=True)
    x = rng.uniform(-1, 1, 1000).astype(np.float32)
    for fmt in FORMATS:
        A = dm.DoseMatrix(rp, cols, vals, 1000, fmt)
        ys = []
        for group_nnz in (1024, 16384, 1 << 20):
            _say("tiny rows", fmt, group_nnz)
            A.set_partition(group_nnz)
            ys.append(_check_forward(A, rp, cols, vals, fmt, x)[0])
        for y in ys[1:]:
            np.testing.assert_array_equal(_bits(y), _bits(ys[0]))
        A.close()


def test_window_and_global_gathers_agree(dev):
    """Groups whose column window fits LDS gather x there, the others from
    global memory; both must give the same bits."""
    rng = np.random.default_rng(12)
    n_cols = 60000
    lens = rng.integers(1, 400, size=4000)
    rp = np.zeros(lens.size + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    cols = np.empty(rp[-1], np.int32)
    for i, L in enumerate(lens):
        # rows 0..1999 use columns below 2000; rows 2000.. spread over all columns
        span = 2000 if i < 2000 else n_cols
        cols[rp[i]:rp[i + 1]] = np.sort(rng.choice(span, size=L, replace=False))
    vals = np.exp(rng.normal(-3, 1, size=rp[-1])).astype(np.float32)
    x = rng.uniform(0, 1, n_cols).astype(np.float32)
    A = dm.DoseMatrix(rp, cols, vals, n_cols, "fp16")
    A.set_partition(8192)
    info = A.info()
    assert 0 < info["n_groups_windowed"] < info["n_groups"]
    y, _ = _check_forward(A, rp, cols, vals, "fp16", x)
    A.set_partition(1 << 20)  # one group per 2^20 entries: no window fits
    assert A.info()["n_groups_windowed"] == 0
    y2, _ = _check_forward(A, rp, cols, vals, "fp16", x)
    np.testing.assert_array_equal(_bits(y), _bits(y2))
    A.close()


def test_empty_and_degenerate_matrices(dev):
    _say("degenerate")
    # no rows
    A = dm.DoseMatrix(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 5)
    A.spmv(torch.ones(5, device=dev), torch.empty(0, device=dev))
    A.close()
    # rows but no entries: every y must be +0
    A = dm.DoseMatrix(np.zeros(3001, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 7)
    y = torch.full((3000,), 7.0, device=dev)
    A.spmv(torch.ones(7, device=dev), y)
    torch.cuda.synchronize()
    assert np.all(_bits(y.cpu().numpy()) == 0)
    A.close()
    # one row holding every column (longer than any block)
    n = 60000
    rp = np.array([0, n], np.int64)
    cols = np.arange(n, dtype=np.int32)
    vals = np.full(n, 0.5, np.float32)
    x = np.ones(n, np.float32)
    A = dm.DoseMatrix(rp, cols, vals, n)
    y = A.spmv(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    assert y.item() == 30000.0  # exact: every partial sum is a multiple of 0.5 below 2^24
    A.close()
    # a single entry
    A = dm.DoseMatrix(np.array([0, 0, 1, 1], np.int64), np.array([2], np.int32), np.array([0.75], np.float32), 3)
    y = A.spmv(torch.tensor([1.0, 2.0, 4.0], device=dev))
    torch.cuda.synchronize()
    assert y.cpu().tolist() == [0.0, 3.0, 0.0]
    A.close()


def test_exact_arithmetic_is_bit_exact(dev):
    """Values k/16 (exact in every format) and small integer x: every partial
    sum is an exact dyadic, so any summation order gives the oracle's bits."""
    rng = np.random.default_rng(5)
    lens = rng.integers(0, 600, size=2000)
    rp, cols, _ = _csr_from_lens(rng, lens, 5000)
    vals = (rng.integers(1, 16, size=rp[-1]) / 16.0).astype(np.float32)
    x = rng.integers(0, 8, size=5000).astype(np.float32)
    for fmt in ("fp16", "bf16"):
        _say("exact", fmt)
        A = dm.DoseMatrix(rp, cols, vals, 5000, fmt)
        y = A.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
        y_ref = oracle.spmv(rp, cols, oracle.decode_matrix(fmt, rp, vals)[0], x)
        np.testing.assert_array_equal(_bits(y), _bits(y_ref.astype(np.float32)))
        A.close()


@pytest.mark.parametrize("fmt", FORMATS)
def test_unit_vectors_give_decoded_columns(fmt, dev):
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, fmt)
    dec, _ = oracle.decode_matrix(fmt, rp, vals)
    dense = np.zeros((spec.n_rows, spec.n_cols), np.float32)
    dense[np.repeat(np.arange(spec.n_rows), np.diff(rp)), cols] = dec
    _say("unit vectors", fmt)
    for j in [0, 1, 137, 250, 499]:
        e = torch.zeros(spec.n_cols, device=dev)
        e[j] = 1.0
        y = A.spmv(e).cpu().numpy()
        np.testing.assert_array_equal(_bits(y), _bits(dense[:, j]))
    A.close()


def test_identity(dev):
    n = 100000
    rp = np.arange(n + 1, dtype=np.int64)
    A = dm.DoseMatrix(rp, np.arange(n, dtype=np.int32), np.ones(n, np.float32), n)
    x = torch.rand(n, device=dev)
    y = A.spmv(x)
    assert torch.equal(y, x)
    A.close()


def test_determinism_repeat_and_rebuild(dev):
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    x = torch.from_numpy(dosegen.spot_weights(spec.seed, 0, spec.n_cols)).cuda()
    _say("determinism")
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols)
    A.set_partition(1024)  # many groups
    y0 = A.spmv(x).clone()
    for _ in range(50):
        assert torch.equal(A.spmv(x), y0)
    B = dm.DoseMatrix(rp, cols, vals, spec.n_cols)
    B.set_partition(65536)
    assert torch.equal(B.spmv(x), y0)
    A.close()
    B.close()


def test_nonnegative_dose_and_positive_zero_rows(dev):
    spec = dosegen.clinical_beam()
    spec = dosegen.Spec("clinical_slab", 128, 128, 6, 100, 250, 200.0, 0.6, seed=spec.seed)
    rp, cols, vals = dosegen.csr(spec)
    x = torch.from_numpy(dosegen.spot_weights(spec.seed, 0, spec.n_cols)).cuda()
    _say("nonneg", rp[-1])
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols)
    y = A.spmv(x).cpu().numpy()
    empty = np.diff(rp) == 0
    assert empty.mean() > 0.5
    assert np.all(_bits(y[empty]) == 0)
    assert np.all(y[~empty] > 0)
    A.close()


def test_linearity(dev):
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols)
    x = torch.from_numpy(dosegen.spot_weights(spec.seed, 0, spec.n_cols)).cuda()
    z = torch.from_numpy(dosegen.spot_weights(spec.seed, 1, spec.n_cols)).cuda()
    y = A.spmv(x + z).double()
    y2 = A.spmv(x).double() + A.spmv(z).double()
    assert torch.max(torch.abs(y - y2) / y2).item() <= 3e-6
    # scaling by a power of two is exact
    assert torch.equal(A.spmv(4.0 * x), 4.0 * A.spmv(x))
    A.close()


def test_error_paths(dev):
    rp, c, v = np.array([0, 2], np.int64), np.array([0, 1], np.int32), np.array([1, 2], np.float32)
    A = dm.DoseMatrix(rp, c, v, 2)
    with pytest.raises(dm.DoseError) as e:
        A.adjoint(torch.ones(1, device=dev))
    assert e.value.code == dm._lib.ERR_NO_TRANSPOSE
    buf = torch.ones(4, device=dev)
    st = dm._lib.load().dose_spmv(A.handle, buf.data_ptr(), buf.data_ptr() + 4, None)
    assert st == dm._lib.ERR_INVALID_ARGUMENT
    with pytest.raises(dm.DoseError) as e:
        dm.DoseMatrix(rp, np.array([1, 0], np.int32), v, 2)
    assert e.value.code == dm._lib.ERR_BAD_CSR
    with pytest.raises(dm.DoseError):
        A.set_partition(1000)
    A.close()


def _sample_rows(lens, rng, n_random):
    order = np.argsort(lens)
    longest = order[-200:]
    empty = np.nonzero(lens == 0)[0]
    pick = [longest, empty[rng.integers(0, empty.size, 200)] if empty.size else np.zeros(0, np.int64),
            rng.integers(0, lens.size, n_random)]
    return np.unique(np.concatenate(pick))


def test_clinical_beam_full_size_sampled(dev):
    """The benchmark's workload at full size, in the launch configuration the
    benchmark times, checked on a seeded sample of rows (longest rows, empty
    rows, random rows) recomputed one by one by the oracle."""
    spec = dosegen.clinical_beam()
    rp, cols, vals = dosegen.csr(spec)
    x = dosegen.spot_weights(spec.seed, 0, spec.n_cols)
    _say("clinical full size", rp[-1])
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16")
    y = A.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
    lens = np.diff(rp)
    rng = np.random.default_rng(7)
    rows = _sample_rows(lens, rng, 5000)
    y_ref = np.empty(rows.size)
    for t, i in enumerate(rows):
        c, v = dosegen.row(spec, int(i))
        d, _ = oracle.decode_matrix("fp16", np.array([0, c.size], np.int64), v)
        y_ref[t] = oracle.row_dot(c, d, x)
    assert oracle.max_rel_err(y[rows], y_ref) <= TOL
    # property at every row: empty rows exactly +0, others positive
    assert np.all(_bits(y[lens == 0]) == 0) and np.all(y[lens > 0] > 0)
    A.close()


@pytest.mark.parametrize("variant", ["beam_along_x", "paper_irregular"])
@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp8e4m3_rowscale"])
def test_bias_control_workloads(variant, fmt, dev):
    """The generator's bias controls at a small size: the beam along x (rows
    of neighbouring voxels no longer share spots) and the paper's irregular
    row lengths (sigma 1.0, rows up to 16,000 entries).  Parity with the
    oracle and bitwise equality under other partitions."""
    base = dosegen.Spec("bias_small", 48, 48, 32, 60, 50, 120.0, 0.6, seed=dosegen.SEED0 + 7)
    spec = getattr(dosegen, variant)(base)
    rp, cols, vals = dosegen.csr(spec)
    _say("bias control", variant, fmt, int(rp[-1]), int(np.diff(rp).max()))
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, fmt)
    x_h = dosegen.spot_weights(spec.seed, 0, spec.n_cols)
    x = torch.from_numpy(x_h).cuda()
    y = A.spmv(x).cpu().numpy()
    dec, _ = oracle.decode_matrix(fmt, rp, vals)
    assert oracle.max_rel_err(y, oracle.spmv(rp, cols, dec, x_h)) <= TOL
    for g in (2048, 65536):
        A.set_partition(g)
        np.testing.assert_array_equal(A.spmv(x).cpu().numpy().view(np.uint32), y.view(np.uint32))
    A.close()
