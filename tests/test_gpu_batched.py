"""Batched products: many matrices of uneven sizes and several spot-weight
vectors per matrix in one persistent launch, replayed from a HIP graph.

Under the same partition every vector of a batched product is bitwise what
the plain product gives (the summation order is the partition's), and both
match the oracle within 1e-5.
"""
import numpy as np
import pytest
import torch

import dosegen
import oracle
import paper_2103_09683_amd as dm

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _say(*a):
    print(*a, flush=True)


def _bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def _small_batch(fmt, n=8, scale=0.03):
    specs = dosegen.robust_batch(scale)[:n]
    mats, host = [], []
    for s in specs:
        rp, cols, vals = dosegen.csr(s)
        host.append((s, rp, cols, vals))
        mats.append(dm.DoseMatrix(rp, cols, vals, s.n_cols, fmt))
    return mats, host


@pytest.mark.parametrize("n_rhs", [1, 2, 4])
@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp8e4m3_rowscale"])
def test_batched_matches_plain_bitwise_and_oracle(fmt, n_rhs, dev):
    _say("batched", fmt, n_rhs)
    mats, host = _small_batch(fmt)
    entries, xs = [], []
    for A, (s, rp, cols, vals) in zip(mats, host):
        X = np.stack([dosegen.spot_weights(s.seed, 10 * s.matrix_id + r, s.n_cols) for r in range(n_rhs)], 1)
        xs.append(X)
        Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
        Y = torch.full((s.n_rows, n_rhs), np.nan, device=dev)
        entries.append((A, Xd if n_rhs > 1 else Xd.reshape(-1), Y if n_rhs > 1 else Y.reshape(-1)))
    dm.spmv_batched(entries)
    torch.cuda.synchronize()
    for (A, Xd, Y), X, (s, rp, cols, vals) in zip(entries, xs, host):
        Y2 = Y.reshape(s.n_rows, n_rhs)
        dec, _ = oracle.decode_matrix(fmt, rp, vals)
        Y_ref = oracle.spmv_multi(rp, cols, dec, X)
        for r in range(n_rhs):
            y_plain = A.spmv(torch.from_numpy(np.ascontiguousarray(X[:, r])).cuda()).cpu().numpy()
            np.testing.assert_array_equal(_bits(Y2[:, r].cpu().numpy()), _bits(y_plain))
            assert oracle.max_rel_err(Y2[:, r].cpu().numpy(), Y_ref[:, r]) <= TOL
    for A in mats:
        A.close()


def test_plan_graph_replays_match_eager(dev):
    _say("plan replay")
    mats, host = _small_batch("fp16", n=6)
    entries = []
    for A, (s, rp, cols, vals) in zip(mats, host):
        X = torch.from_numpy(np.stack([dosegen.spot_weights(s.seed, r, s.n_cols) for r in range(4)], 1)).cuda()
        entries.append((A, X.contiguous(), torch.zeros(s.n_rows, 4, device=dev)))
    dm.spmv_batched(entries)
    torch.cuda.synchronize()
    ref = [Y.clone() for _, _, Y in entries]
    plan = dm.BatchPlan(entries)
    for rep in range(4):
        for _, _, Y in entries:
            Y.fill_(-1.0)  # eager work between replays
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for (_, _, Y), R in zip(entries, ref):
            assert torch.equal(Y, R), rep
    # new inputs are picked up by a replay (the graph holds pointers, not values)
    for _, X, _ in entries:
        X.mul_(2.0)
    plan.launch()
    torch.cuda.synchronize()
    for (_, _, Y), R in zip(entries, ref):
        assert torch.equal(Y, 2.0 * R)
    plan.close()
    for A in mats:
        A.close()


def test_autotuned_plan_stays_within_tolerance(dev, tmp_path, monkeypatch):
    monkeypatch.setenv("DOSE_TUNE_CACHE", str(tmp_path / "tune.txt"))
    _say("autotune")
    mats, host = _small_batch("bf16", n=4)
    entries = []
    for A, (s, rp, cols, vals) in zip(mats, host):
        X = torch.from_numpy(np.stack([dosegen.spot_weights(s.seed, r, s.n_cols) for r in range(4)], 1)).cuda()
        entries.append((A, X.contiguous(), torch.zeros(s.n_rows, 4, device=dev)))
    before = [A.info()["group_nnz"] for A in mats]
    plan = dm.BatchPlan(entries, autotune=True)
    plan.launch()
    torch.cuda.synchronize()
    for (A, X, Y), (s, rp, cols, vals), g0 in zip(entries, host, before):
        # the plan runs its own copy of the chosen partition; the matrix keeps its own
        assert A.info()["group_nnz"] == g0
        for r in range(4):
            y_plain = A.spmv(X[:, r].contiguous()).cpu().numpy()
            np.testing.assert_array_equal(_bits(Y[:, r].cpu().numpy()), _bits(y_plain))
        dec, _ = oracle.decode_matrix("bf16", rp, vals)
        Y_ref = oracle.spmv_multi(rp, cols, dec, X.cpu().numpy())
        for r in range(4):
            assert oracle.max_rel_err(Y[:, r].cpu().numpy(), Y_ref[:, r]) <= TOL
    plan.close()
    lines = (tmp_path / "tune.txt").read_text().split("\n")
    assert len([ln for ln in lines if ln]) == 4
    for A in mats:
        A.close()


def test_batched_rejects_mixed_formats(dev):
    mats16, h16 = _small_batch("fp16", n=1)
    mats8, h8 = _small_batch("bf16", n=1)
    s = h16[0][0]
    e = [(mats16[0], torch.zeros(s.n_cols, device=dev), torch.zeros(s.n_rows, device=dev)),
         (mats8[0], torch.zeros(s.n_cols, device=dev), torch.zeros(s.n_rows, device=dev))]
    with pytest.raises(dm.DoseError) as err:
        dm.spmv_batched(e)
    assert err.value.code == dm._lib.ERR_UNSUPPORTED
