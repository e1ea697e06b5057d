"""Cleanup after a failed device allocation.  DOSE_FAULT_INJECT=alloc:<n>
makes the n-th device allocation after the variable takes that value fail
with DOSE_ERR_OUT_OF_MEMORY.  For every n up to the first that lets the call
succeed, the create call (a CSR matrix with its transpose in E4M3 with row
scales, over spot rows or in voxel slabs, a SELL-C-sigma matrix with
run-length indices, an autotuned batch plan, an adjoint plan) must fail with
that status and leave the device's free memory where it was: whatever the
call had allocated before the failure is freed."""
import numpy as np
import pytest
import torch

import paper_2103_09683_amd as dm
from paper_2103_09683_amd import _lib

pytestmark = pytest.mark.gpu

SLACK = 1 << 20  # bytes: allocation granularity of the free-memory count


def _matrix(n_rows=200_000, n_cols=6_000, run=20, seed=5):
    """Rows of one run of `run` consecutive columns (4M entries: every
    stream of the matrix is megabytes, so a leaked stream shows in the free
    memory), a tenth of the rows empty."""
    rng = np.random.default_rng(seed)
    lens = np.where(rng.random(n_rows) < 0.1, 0, run)
    rp = np.zeros(n_rows + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    starts = rng.integers(0, n_cols - run, n_rows)
    cols = (np.repeat(starts, lens) + (np.arange(rp[-1]) - np.repeat(rp[:-1], lens))).astype(np.int32)
    vals = np.exp(rng.normal(-3, 1, rp[-1])).astype(np.float32)
    return rp, cols, vals, n_cols


def _free():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def _sweep(make, monkeypatch):
    obj = make()  # warm-up: code objects and library state
    obj.close()
    base = _free()
    for n in range(1, 64):
        monkeypatch.setenv("DOSE_FAULT_INJECT", f"alloc:{n}")
        try:
            obj = make()
        except dm.DoseError as e:
            assert e.code == _lib.ERR_OUT_OF_MEMORY, (n, e)
            assert "injected" in e.message
            assert abs(base - _free()) <= SLACK, (n, base - _free())
            continue
        monkeypatch.delenv("DOSE_FAULT_INJECT")
        obj.close()
        assert abs(base - _free()) <= SLACK
        return n
    pytest.fail("the call never succeeded")


def test_matrix_create_cleans_up(dev, monkeypatch):
    rp, cols, vals, n_cols = _matrix()
    n = _sweep(lambda: dm.DoseMatrix(rp, cols, vals, n_cols, "fp8e4m3_rowscale", transpose=True), monkeypatch)
    print(f"matrix create: {n - 1} allocations failed in turn", flush=True)
    assert n > 8


def test_matrix_create_slabs_cleans_up(dev, monkeypatch):
    # the transpose in voxel slabs: sort, run-length encoding, placement,
    # combine map and partition, each failing in turn
    rp, cols, vals, n_cols = _matrix()
    n = _sweep(lambda: dm.DoseMatrix(rp, cols, vals, n_cols, "fp8e4m3_rowscale", transpose="slabs"),
               monkeypatch)
    print(f"matrix create (voxel slabs): {n - 1} allocations failed in turn", flush=True)
    assert n > 12


def test_sell_create_cleans_up(dev, monkeypatch):
    rp, cols, vals, n_cols = _matrix()
    n = _sweep(lambda: dm.SellMatrix(rp, cols, vals, n_cols, "fp16", sigma=1024, index_format="runs"),
               monkeypatch)
    print(f"sell create: {n - 1} allocations failed in turn", flush=True)
    assert n > 4


def test_batch_plan_create_cleans_up(dev, monkeypatch):
    rp, cols, vals, n_cols = _matrix(n_rows=50_000)
    mats = [dm.DoseMatrix(rp, cols, vals, n_cols, "fp16") for _ in range(3)]
    x = torch.rand(n_cols, 4, device=dev)
    ys = [torch.empty(50_000, 4, device=dev) for _ in mats]
    n = _sweep(lambda: dm.BatchPlan([(A, x, y) for A, y in zip(mats, ys)], autotune=True), monkeypatch)
    print(f"batch plan create: {n - 1} allocations failed in turn", flush=True)
    assert n > 1
    for A in mats:
        A.close()


def test_adjoint_plan_create_cleans_up(dev, monkeypatch):
    # E4M3 over voxel slabs, accumulating: scratch, work list, re-made
    # partitions, the seed-scaling and combine tables, each failing in turn
    rp, cols, vals, n_cols = _matrix(n_rows=50_000)
    mats = [dm.DoseMatrix(rp, cols, vals, n_cols, "fp8e4m3_rowscale", transpose="slabs") for _ in range(3)]
    v = torch.rand(50_000, device=dev)
    g = torch.empty(n_cols, device=dev)
    n = _sweep(lambda: dm.AdjointPlan([(A, v, g) for A in mats], accumulate=True), monkeypatch)
    print(f"adjoint plan create: {n - 1} allocations failed in turn", flush=True)
    assert n > 4
    for A in mats:
        A.close()
