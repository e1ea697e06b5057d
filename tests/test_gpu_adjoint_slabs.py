"""The adjoint g = A^T v over A^T stored in voxel slabs
(DOSE_CREATE_TRANSPOSE_SLABS): one row per (slab, spot) pair, each spot's
result the sum of its slab rows' partials in ascending slab.

Reference: the oracle's A^T v (Sec. I: the gradient of every iteration).  The
seed is signed, so the error is measured componentwise against |A|^T |v|:
|g_j - g*_j| <= 1e-5 (|A|^T |v|)_j (FP32; the slab split adds one FP32
addition per slab a spot touches to the row sums' rounding), 1e-12 for FP64
vectors (E4M3: 2^-22, the FP32 product fl32(q s) of the code and its row
scale, as for the spot-row adjoint).  Spots with no entries give +0 exactly.
Beyond parity: every row group's seed window fits in LDS (the layout's
purpose), results are bitwise the same under any partition and across A's
index formats (the slab form stores 16-bit slab-local voxel offsets either
way), and the adjoint is the transpose of the forward product.
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
TOL64 = 1e-12


def _say(*a):
    print(*a, flush=True)


def _bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint64 if a.dtype == np.float64 else np.uint32)


def _with_low_bits(hi32, rng):
    """FP64 values hi + lo with both parts exact in FP32 and lo below hi's
    last bit, so a kernel that rounded the seed to FP32 would lose lo."""
    hi = np.asarray(hi32, np.float32)
    e = np.frexp(hi.astype(np.float64))[1]
    u = (rng.choice([-1.0, 1.0], hi.size) * rng.uniform(0.5, 1.0, hi.size)).astype(np.float32)
    lo = np.ldexp(u.astype(np.float64), e - 26).astype(np.float32)
    x = hi.astype(np.float64) + lo.astype(np.float64)
    assert np.array_equal(x - hi.astype(np.float64), lo.astype(np.float64))
    return x, hi, lo


def _dense_block_csr(seed, n_rows=3 * 4096 + 1001, n_cols=40):
    """Spots 0-9 hit about 90% of all voxels (slab rows of ~3,700 entries:
    split groups under small row groups), spots 10-29 a few voxels each,
    spots 30-39 none."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n_rows):
        c = [j for j in range(10) if rng.random() < 0.9]
        c += sorted(rng.choice(np.arange(10, 30), size=int(rng.integers(0, 4)), replace=False).tolist())
        rows.append(np.array(sorted(c), np.int32))
    lens = np.array([r.size for r in rows])
    rp = np.zeros(n_rows + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    cols = np.concatenate(rows).astype(np.int32)
    vals = np.exp(rng.normal(-3, 1, cols.size)).astype(np.float32)
    return rp, cols, vals, n_cols


def _check(g, rp, cols, dec, v, n_cols, tol):
    g_ref = oracle.spmv_T(rp, cols, dec, v, n_cols)
    scale = oracle.spmv_T(rp, cols, np.abs(dec), np.abs(v), n_cols)
    err = oracle.max_scaled_err(g, g_ref, scale)
    return err <= tol, err


@pytest.mark.parametrize("fmt", FORMATS)
def test_slab_adjoint_vs_oracle(fmt, dev):
    """The small workload: 20,000 voxels in slabs of 4,096 (the last one
    ragged) x 500 spots, int32 and 16-bit indices (bitwise the same)."""
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    v = dosegen.signed_values(spec.seed, 3, spec.n_rows)
    dec, _ = oracle.decode_matrix(fmt, rp, vals)
    outs = []
    for idx in ("i32", "u16"):
        _say("slab adjoint", fmt, idx)
        A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, fmt, transpose="slabs", index_format=idx)
        inf = A.info()
        W = inf["slab_voxels"]
        assert W > 0 and W % 8 == 0 and inf["has_transpose"] == 1
        assert inf["n_groups_windowed_t"] == inf["n_groups_t"] > 0
        g = A.adjoint(torch.from_numpy(v).cuda()).cpu().numpy()
        ok, err = _check(g, rp, cols, dec, v, spec.n_cols, TOL)
        _say(f"  slabs of {W}: {inf['n_groups_t']} groups, max scaled err {err:.3e}")
        assert ok, (fmt, idx, err)
        outs.append(_bits(g))
        A.close()
    np.testing.assert_array_equal(outs[0], outs[1])


@pytest.mark.parametrize("fmt", ["fp16", "fp8e4m3_rowscale"])
def test_slab_adjoint_partitions_split_rows_and_empty_spots(fmt, dev):
    """Slab rows of ~3,700 entries: split groups shared by four waves (group
    sizes 1024 and 8192), rows summed by one wave (65536); the same bits
    under every partition and on repeat; spots without entries give +0."""
    rp, cols, vals, n_cols = _dense_block_csr(17)
    rng = np.random.default_rng(18)
    v = rng.uniform(-1, 1, rp.size - 1).astype(np.float32)
    dec, _ = oracle.decode_matrix(fmt, rp, vals)
    A = dm.DoseMatrix(rp, cols, vals, n_cols, fmt, transpose="slabs")
    ref = None
    for gt in (1024, 8192, 65536):
        A.set_partition(8192, gt)
        inf = A.info()
        _say("slab partition", fmt, gt, inf["n_groups_t"], inf["n_groups_split_t"])
        assert (inf["n_groups_split_t"] > 0) == (gt < 65536)
        assert inf["n_groups_windowed_t"] == inf["n_groups_t"]
        g = A.adjoint(torch.from_numpy(v).cuda()).cpu().numpy()
        ok, err = _check(g, rp, cols, dec, v, n_cols, TOL)
        assert ok, (gt, err)
        assert np.all(_bits(g[30:]) == 0)
        g2 = A.adjoint(torch.from_numpy(v).cuda()).cpu().numpy()
        np.testing.assert_array_equal(_bits(g), _bits(g2))
        if ref is None:
            ref = _bits(g)
        np.testing.assert_array_equal(_bits(g), ref)
    A.close()


@pytest.mark.parametrize("fmt", ["fp16", "fp8e4m3_rowscale", "fp32"])
def test_slab_adjoint_f64(fmt, dev):
    """FP64 seeds and results (the paper's half/double arithmetic): the
    reference is oracle(hi) + oracle(lo)."""
    rng = np.random.default_rng(90)
    spec = dosegen.small_plain()
    cases = [("small_plain", *dosegen.csr(spec), spec.n_cols), ("dense_block", *_dense_block_csr(19))]
    for name, rp, cols, vals, n_cols in cases:
        _say("slab adjoint f64", fmt, name)
        dec, _ = oracle.decode_matrix(fmt, rp, vals)
        A = dm.DoseMatrix(rp, cols, vals, n_cols, fmt, transpose="slabs")
        v, vh, vl = _with_low_bits(rng.standard_normal(rp.size - 1).astype(np.float32), rng)
        g = A.adjoint(torch.from_numpy(v).cuda()).cpu().numpy()
        assert g.dtype == np.float64
        g_ref = oracle.spmv_T(rp, cols, dec, vh, n_cols) + oracle.spmv_T(rp, cols, dec, vl, n_cols)
        scale = oracle.spmv_T(rp, cols, np.abs(dec), np.abs(vh), n_cols)
        tol = 2.0 ** -22 if fmt == "fp8e4m3_rowscale" else TOL64
        err = oracle.max_scaled_err(g, g_ref, scale)
        _say(f"  max scaled err {err:.3e}")
        assert err <= tol, (fmt, name, err)
        empty = np.bincount(cols, minlength=n_cols) == 0
        assert np.all(_bits(g[empty]) == 0)
        A.close()


def test_slab_adjoint_edges(dev):
    """No entries, fewer voxels than one slab, one spot, slabs whose entry
    counts need no padding row and slabs that do; errors."""
    # no entries (with and without voxels): g = +0
    for n_rows in (0, 5000):
        A = dm.DoseMatrix(np.zeros(n_rows + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 7,
                          "fp16", transpose="slabs")
        g = torch.full((7,), np.nan, device=dev)
        A.adjoint(torch.ones(n_rows, device=dev), g)
        assert np.all(_bits(g.cpu().numpy()) == 0)
        g64 = torch.full((7,), np.nan, dtype=torch.float64, device=dev)
        A.adjoint(torch.ones(n_rows, dtype=torch.float64, device=dev), g64)
        assert np.all(_bits(g64.cpu().numpy()) == 0)
        A.close()
    rng = np.random.default_rng(21)
    for n_rows, n_cols, density in ((300, 1, 0.7), (4096, 3, 1.0), (4096 * 2 + 3, 5, 0.5), (9000, 64, 0.05)):
        mask = rng.random((n_rows, n_cols)) < density
        rp = np.zeros(n_rows + 1, np.int64)
        np.cumsum(mask.sum(1), out=rp[1:])
        cols = np.nonzero(mask)[1].astype(np.int32)
        vals = rng.uniform(0.01, 1, cols.size).astype(np.float32)
        v = rng.uniform(-1, 1, n_rows).astype(np.float32)
        A = dm.DoseMatrix(rp, cols, vals, n_cols, "bf16", transpose="slabs")
        g = A.adjoint(torch.from_numpy(v).cuda()).cpu().numpy()
        dec, _ = oracle.decode_matrix("bf16", rp, vals)
        ok, err = _check(g, rp, cols, dec, v, n_cols, TOL)
        _say("slab edge", n_rows, n_cols, density, err)
        assert ok, (n_rows, n_cols, err)
        A.close()
    # a dense slab (4096 x 3 entries, a multiple of 4) needs no padding row;
    # the stored transpose is not row-per-spot, so it cannot be decoded
    rp = np.arange(0, 3 * 4097, 3, dtype=np.int64)
    cols = np.tile(np.arange(3, dtype=np.int32), 4096)
    A = dm.DoseMatrix(rp, cols, np.ones(cols.size, np.float32), 3, "fp16", transpose="slabs")
    with pytest.raises(dm._lib.DoseError) as e:
        A.decode(part="AT")
    assert e.value.code == dm._lib.ERR_UNSUPPORTED
    A.decode(part="A")
    B = dm.DoseMatrix(rp, cols, np.ones(cols.size, np.float32), 3, "fp16", transpose=True)
    # byte model: 12,288 entries x (2 B code + 2 B slab-local index), 3 slab
    # rows (offsets, partials written and read back, combine map), the seed,
    # the spot offsets of the combine map and g; over spot rows 4 B indices
    assert A.info()["adjoint_bytes"] == 12288 * 4 + 4 * 4 + 4 * 4096 + 8 * 3 + 4 * 4 + 4 * 3 + 4 * 3
    assert B.info()["adjoint_bytes"] == 12288 * 6 + 4 * 4 + 4 * 4096 + 4 * 3 and B.info()["slab_voxels"] == 0
    np.testing.assert_array_equal(A.adjoint(torch.ones(4096, device=dev)).cpu().numpy(), [4096.0] * 3)
    A.close()
    B.close()
    with pytest.raises(ValueError):
        dm.DoseMatrix(rp, cols, np.ones(cols.size, np.float32), 3, "fp16", transpose="rows")


def test_slab_adjoint_autograd_autotune_and_adjointness(dev):
    """The slab adjoint through autograd (DoseSpMV's backward), with the
    create-time autotune (the same bits as without: speed only), and
    <v, A x> = <A^T v, x> within the FP32 bound."""
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16", transpose="slabs")
    T = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16", transpose="slabs", autotune=True)
    x = torch.from_numpy(dosegen.spot_weights(spec.seed, 0, spec.n_cols)).cuda()
    v = torch.from_numpy(dosegen.signed_values(spec.seed, 4, spec.n_rows)).cuda()
    xt = x.clone().requires_grad_(True)
    (dm.dose(xt, A) * v).sum().backward()
    g = A.adjoint(v)
    np.testing.assert_array_equal(_bits(xt.grad.cpu().numpy()), _bits(g.cpu().numpy()))
    np.testing.assert_array_equal(_bits(T.adjoint(v).cpu().numpy()), _bits(g.cpu().numpy()))
    lhs = torch.dot(v.double(), A.spmv(x).double()).item()
    rhs = torch.dot(g.double(), x.double()).item()
    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    bound = np.dot(np.abs(v.cpu().numpy()), oracle.spmv(rp, cols, np.abs(dec), x.cpu().numpy()))
    assert abs(lhs - rhs) <= 2e-6 * bound
    A.close()
    T.close()


@pytest.mark.parametrize("fmt", ["fp16", "fp8e4m3_rowscale"])
def test_slab_matrix_forward_plans_and_autotune(fmt, dev):
    """A matrix whose transpose is stored in voxel slabs keeps A as it is:
    its forward product, alone and in a batch plan, has the bits of a matrix
    without transpose; the create-time autotune (which times the E4M3
    adjoint without column scales) leaves the slab adjoint's bits unchanged."""
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    x = torch.from_numpy(dosegen.spot_weights(spec.seed, 0, spec.n_cols)).cuda()
    v = torch.from_numpy(dosegen.signed_values(spec.seed, 5, spec.n_rows)).cuda()
    P = dm.DoseMatrix(rp, cols, vals, spec.n_cols, fmt)
    S = dm.DoseMatrix(rp, cols, vals, spec.n_cols, fmt, transpose="slabs")
    T = dm.DoseMatrix(rp, cols, vals, spec.n_cols, fmt, transpose="slabs", autotune=True)
    y_ref = P.spmv(x)
    np.testing.assert_array_equal(_bits(S.spmv(x).cpu().numpy()), _bits(y_ref.cpu().numpy()))
    Y = torch.full((spec.n_rows, 1), np.nan, device=dev)
    plan = dm.BatchPlan([(S, x.view(-1, 1).contiguous(), Y)])
    plan.launch()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_bits(Y[:, 0].cpu().numpy()), _bits(y_ref.cpu().numpy()))
    plan.close()
    np.testing.assert_array_equal(_bits(T.adjoint(v).cpu().numpy()), _bits(S.adjoint(v).cpu().numpy()))
    for M in (P, S, T):
        M.close()
