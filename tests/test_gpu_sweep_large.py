"""The largest workload at full size: 8,388,608 voxels x 60,000 spots (about
1.7e9 stored entries) in the three value formats, forward and adjoint on one
GPU, checked against the CPU oracle on a seeded 1% row sample.

* Forward: y on the sampled rows (the longest rows, empty rows, 1% random
  rows) against the oracle on the sub-matrix of those rows; every row's sign
  property (+0 when empty, > 0 otherwise) at full size.
* Adjoint: g = A^T v with v supported on the sampled rows, so that every one
  of the 60,000 entries of g has an exact oracle value (the sub-matrix's
  transpose product), while the kernel still walks all of A^T.
* Adjointness with a dense v at full size: <v, A x> = <A^T v, x> within the
  FP32 bound.
* The same adjoint checks over A^T in voxel slabs (FP16 and E4M3, FP32 and
  FP64 seeds).
"""
import time

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


def _sub_csr(rp, cols, vals, rows):
    """CSR of the given rows (whole rows, in the given order)."""
    lens = rp[rows + 1] - rp[rows]
    srp = np.zeros(rows.size + 1, np.int64)
    np.cumsum(lens, out=srp[1:])
    idx = np.repeat(rp[rows] - srp[:-1], lens) + np.arange(srp[-1], dtype=np.int64)
    return srp, cols[idx], vals[idx]


@pytest.fixture(scope="module")
def sweep():
    spec = dosegen.sweep_large()
    t0 = time.time()
    rp, cols, vals = dosegen.csr(spec)
    _say(f"generated {spec.name}: {rp[-1]} entries in {time.time() - t0:.1f}s")
    lens = np.diff(rp)
    rng = np.random.default_rng(2103)
    empty = np.nonzero(lens == 0)[0]
    rows = np.unique(np.concatenate([np.argsort(lens)[-200:], empty[rng.integers(0, empty.size, 200)],
                                     rng.integers(0, lens.size, lens.size // 100)]))
    sub = _sub_csr(rp, cols, vals, rows)
    yield spec, rp, cols, vals, rows, sub
    del rp, cols, vals, sub


@pytest.mark.timeout(900)
@pytest.mark.parametrize("fmt", FORMATS)
def test_sweep_large_forward_and_adjoint(sweep, fmt, dev):
    spec, rp, cols, vals, rows, (srp, scols, svals) = sweep
    t0 = time.time()
    _say("sweep_large create", fmt)
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, fmt, transpose=True)
    _say(f"created in {time.time() - t0:.1f}s", A.info())
    x_h = dosegen.spot_weights(spec.seed, 0, spec.n_cols)
    y = A.spmv(torch.from_numpy(x_h).cuda()).cpu().numpy()
    _say("forward done")
    dec, _ = oracle.decode_matrix(fmt, srp, svals)
    y_ref = oracle.spmv(srp, scols, dec, x_h)
    err = oracle.max_rel_err(y[rows], y_ref)
    # reported only: the format's own error (oracle on decoded vs on FP32 source values)
    src, _ = oracle.decode_matrix("fp32", srp, svals)
    fmt_err = oracle.max_rel_err(y_ref, oracle.spmv(srp, scols, src, x_h)) if fmt != "fp32" else 0.0
    _say(f"{fmt}: forward max rel err {err:.3e} on {rows.size} sampled rows; format error {fmt_err:.3e}")
    assert err <= TOL, fmt
    lens = np.diff(rp)
    assert np.all(_bits(y[lens == 0]) == 0) and np.all(y[lens > 0] > 0)

    # adjoint, v on the sampled rows only: every entry of g is checked
    v_s = dosegen.signed_values(spec.seed, 2, rows.size)
    v = np.zeros(spec.n_rows, np.float32)
    v[rows] = v_s
    g = A.adjoint(torch.from_numpy(v).cuda()).cpu().numpy()
    _say("adjoint done")
    g_ref = oracle.spmv_T(srp, scols, dec, v_s, spec.n_cols)
    scale = oracle.spmv_T(srp, scols, np.abs(dec), np.abs(v_s), spec.n_cols)
    err_a = oracle.max_scaled_err(g, g_ref, scale)
    _say(f"{fmt}: adjoint max scaled err {err_a:.3e} over all {spec.n_cols} spots")
    assert err_a <= TOL, fmt

    # adjointness at full size with a dense signed v (A >= 0 and x >= 0, so
    # |A| |x| = A x = y)
    vd = dosegen.signed_values(spec.seed, 3, spec.n_rows)
    gd = A.adjoint(torch.from_numpy(vd).cuda()).cpu().numpy()
    lhs = float(np.dot(vd.astype(np.float64), y.astype(np.float64)))
    rhs = float(np.dot(gd.astype(np.float64), x_h.astype(np.float64)))
    bound = float(np.dot(np.abs(vd).astype(np.float64), y.astype(np.float64)))
    assert abs(lhs - rhs) <= 2 * TOL * bound, (fmt, lhs, rhs, bound)
    A.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("fmt", ["fp16", "fp8e4m3_rowscale"])
def test_sweep_large_adjoint_slabs(sweep, fmt, dev):
    """The adjoint over A^T in voxel slabs at full size: every group's seed
    window in LDS; v on the sampled rows, so that all 60,000 spots are
    checked (FP32 and FP64 seeds); adjointness with a dense v."""
    spec, rp, cols, vals, rows, (srp, scols, svals) = sweep
    t0 = time.time()
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, fmt, transpose="slabs")
    inf = A.info()
    _say(f"sweep_large slabs {fmt}: created in {time.time() - t0:.1f}s", inf)
    assert inf["n_groups_windowed_t"] == inf["n_groups_t"] > 0
    dec, _ = oracle.decode_matrix(fmt, srp, svals)
    v_s = dosegen.signed_values(spec.seed, 2, rows.size)
    v = np.zeros(spec.n_rows, np.float32)
    v[rows] = v_s
    g_ref = oracle.spmv_T(srp, scols, dec, v_s, spec.n_cols)
    scale = oracle.spmv_T(srp, scols, np.abs(dec), np.abs(v_s), spec.n_cols)
    g = A.adjoint(torch.from_numpy(v).cuda()).cpu().numpy()
    err = oracle.max_scaled_err(g, g_ref, scale)
    g64 = A.adjoint(torch.from_numpy(v.astype(np.float64)).cuda()).cpu().numpy()
    err64 = oracle.max_scaled_err(g64, g_ref, scale)
    _say(f"{fmt} slabs: adjoint max scaled err {err:.3e} (FP64 {err64:.3e}) over all {spec.n_cols} spots")
    assert err <= TOL, fmt
    assert err64 <= (2.0 ** -22 if fmt == "fp8e4m3_rowscale" else 1e-12), fmt
    x_h = dosegen.spot_weights(spec.seed, 0, spec.n_cols)
    y = A.spmv(torch.from_numpy(x_h).cuda()).cpu().numpy()
    vd = dosegen.signed_values(spec.seed, 3, spec.n_rows)
    gd = A.adjoint(torch.from_numpy(vd).cuda()).cpu().numpy()
    lhs = float(np.dot(vd.astype(np.float64), y.astype(np.float64)))
    rhs = float(np.dot(gd.astype(np.float64), x_h.astype(np.float64)))
    bound = float(np.dot(np.abs(vd).astype(np.float64), y.astype(np.float64)))
    assert abs(lhs - rhs) <= 2 * TOL * bound, (fmt, lhs, rhs, bound)
    A.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("idx", ["runs", "u16"])
def test_sweep_large_sell(sweep, idx, dev):
    """SELL-C-sigma form (sigma 65,536) of the largest workload: one vector on
    the sampled rows against the oracle, +0 on every empty row; FP64 vectors
    on the sampled rows; four vectors bitwise equal to the single-vector
    products of their columns."""
    spec, rp, cols, vals, rows, (srp, scols, svals) = sweep
    t0 = time.time()
    S = dm.SellMatrix(rp, cols, vals, spec.n_cols, "fp16", sigma=65536, index_format=idx)
    _say(f"sell {idx} created in {time.time() - t0:.1f}s", S.info())
    x_h = dosegen.spot_weights(spec.seed, 0, spec.n_cols)
    y = S.spmv(torch.from_numpy(x_h).cuda()).cpu().numpy()
    dec, _ = oracle.decode_matrix("fp16", srp, svals)
    err = oracle.max_rel_err(y[rows], oracle.spmv(srp, scols, dec, x_h))
    _say(f"sell {idx}: forward max rel err {err:.3e} on {rows.size} sampled rows")
    assert err <= TOL
    lens = np.diff(rp)
    assert np.all(_bits(y[lens == 0]) == 0) and np.all(y[lens > 0] > 0)
    # FP64 weights and dose (half/double): the sampled rows within 1e-12
    y64 = S.spmv(torch.from_numpy(x_h.astype(np.float64)).cuda()).cpu().numpy()
    err64 = oracle.max_rel_err(y64[rows], oracle.spmv(srp, scols, dec, x_h.astype(np.float64)))
    _say(f"sell {idx}: FP64 max rel err {err64:.3e}")
    assert err64 <= 1e-12
    X = torch.from_numpy(np.stack([dosegen.spot_weights(spec.seed, r, spec.n_cols) for r in range(4)], 1)).cuda()
    Y = S.spmv(X.contiguous()).cpu().numpy()
    assert np.array_equal(_bits(Y[:, 0]), _bits(y))
    for r in range(1, 4):
        yr = S.spmv(X[:, r].contiguous()).cpu().numpy()
        assert np.array_equal(_bits(Y[:, r]), _bits(yr)), r
    S.close()
