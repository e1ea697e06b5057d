"""Adjoint plans (dose_adjoint_plan_create): the adjoints of several
matrices captured into one HIP graph (Sec. I, II-A: every beam's gradient
under every scenario, each iteration).

Each g must carry the bits of the plain adjoint of its item (the same
kernels, the same summation order), on every replay of the graph, with the
program's own eager work between replays, for A^T over spot rows and in
voxel slabs, in FP16, BF16 and E4M3 (whose plan scales the seeds first);
replays read the current seeds.  Parity of the plain adjoint with the oracle
is tested in test_gpu_adjoint.py and test_gpu_adjoint_slabs.py; one item here
is also checked against the oracle.
"""
import numpy as np
import pytest
import torch

import dosegen
import oracle
import paper_2103_09683_amd as dm
from paper_2103_09683_amd import _lib

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _bits(t):
    return t.contiguous().view(torch.int32)


def _matrices(fmt, transpose, n=6):
    # 2 scenarios x 3 beams on one 128 x 128 x 3 grid (beams of 5K-25K spots)
    specs = dosegen.robust_scenarios(0.04, 2, 3)[:n]
    host = [(sp, *dosegen.csr(sp)) for sp in specs]
    mats = [dm.DoseMatrix(rp, cols, vals, sp.n_cols, fmt, transpose=transpose) for sp, rp, cols, vals in host]
    return mats, host


@pytest.mark.parametrize("transpose", [True, "slabs"])
@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp8e4m3_rowscale"])
def test_adjoint_plan_bits_and_replays(fmt, transpose, dev):
    _say("adjoint plan", fmt, transpose)
    mats, host = _matrices(fmt, transpose)
    # items 0-2 share one seed (as the beams of one scenario do)
    n = mats[0].n_rows
    shared = torch.from_numpy(dosegen.signed_values(dosegen.SEED0, 40, n)).cuda()
    vs = [shared if i < 3 else torch.from_numpy(dosegen.signed_values(dosegen.SEED0, 41 + i, A.n_rows)).cuda()
          for i, A in enumerate(mats)]
    gs = [torch.full((A.n_cols,), np.nan, device=dev) for A in mats]
    plan = dm.AdjointPlan(list(zip(mats, vs, gs)))
    ref = [A.adjoint(v) for A, v in zip(mats, vs)]
    for rep in range(3):
        for g in gs:
            g.fill_(np.nan)  # eager work between replays
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for i, (g, r) in enumerate(zip(gs, ref)):
            assert torch.equal(_bits(g), _bits(r)), (rep, i)
    # replays read the current seeds
    for v in vs[3:]:
        v.mul_(-0.5)
    shared.mul_(2.0)
    plan.launch()
    torch.cuda.synchronize()
    for i, (A, v, g) in enumerate(zip(mats, vs, gs)):
        assert torch.equal(_bits(g), _bits(A.adjoint(v))), i
    # one item against the oracle
    sp, rp, cols, vals = host[4]
    dec, _ = oracle.decode_matrix(fmt, rp, vals)
    vh = vs[4].cpu().numpy()
    g_ref = oracle.spmv_T(rp, cols, dec, vh, sp.n_cols)
    scale = oracle.spmv_T(rp, cols, np.abs(dec), np.abs(vh), sp.n_cols)
    assert oracle.max_scaled_err(gs[4].cpu().numpy(), g_ref, scale) <= 1e-5
    plan.close()
    for A in mats:
        A.close()


@pytest.mark.parametrize("fmt,transpose", [("fp16", "slabs"), ("fp8e4m3_rowscale", True)])
def test_adjoint_plan_autotune(fmt, transpose, dev):
    """DOSE_PLAN_AUTOTUNE picks the row-group size by timing the launch; the
    bits stay those of the plain adjoints."""
    mats, _ = _matrices(fmt, transpose)
    vs = [torch.from_numpy(dosegen.signed_values(dosegen.SEED0, 60 + i, A.n_rows)).cuda()
          for i, A in enumerate(mats)]
    gs = [torch.empty(A.n_cols, device=dev) for A in mats]
    plan = dm.AdjointPlan(list(zip(mats, vs, gs)), autotune=True)
    for g in gs:
        g.fill_(np.nan)
    plan.launch()
    torch.cuda.synchronize()
    for i, (A, v, g) in enumerate(zip(mats, vs, gs)):
        assert torch.equal(_bits(g), _bits(A.adjoint(v))), i
    plan.close()
    for A in mats:
        A.close()


def test_adjoint_plan_errors_and_empty(dev):
    mats, _ = _matrices("fp16", "slabs", n=2)
    rows, _ = _matrices("fp16", True, n=1)
    e4, _ = _matrices("fp8e4m3_rowscale", "slabs", n=1)
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    plain = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16")
    v = [torch.zeros(A.n_rows, device=dev) for A in mats]
    g = [torch.zeros(A.n_cols, device=dev) for A in mats]

    def code(entries):
        with pytest.raises(dm.DoseError) as e:
            dm.AdjointPlan(entries)
        return e.value.code

    assert code([(mats[0], v[0], g[0]), (rows[0], torch.zeros(rows[0].n_rows, device=dev),
                                         torch.zeros(rows[0].n_cols, device=dev))]) == _lib.ERR_UNSUPPORTED
    assert code([(mats[0], v[0], g[0]), (e4[0], torch.zeros(e4[0].n_rows, device=dev),
                                         torch.zeros(e4[0].n_cols, device=dev))]) == _lib.ERR_UNSUPPORTED
    assert code([(plain, torch.zeros(plain.n_rows, device=dev),
                  torch.zeros(plain.n_cols, device=dev))]) == _lib.ERR_NO_TRANSPOSE
    # two items writing the same g; an item's g inside another's v
    assert code([(mats[0], v[0], g[0]), (mats[0], v[1], g[0])]) == _lib.ERR_INVALID_ARGUMENT
    big = torch.zeros(mats[0].n_rows + mats[1].n_cols, device=dev)
    assert code([(mats[0], big[:mats[0].n_rows], g[0]),
                 (mats[1], v[1], big[mats[0].n_rows - 8:mats[0].n_rows - 8 + mats[1].n_cols])]) == \
        _lib.ERR_INVALID_ARGUMENT
    arr = (_lib.AdjointItem * 1)()
    arr[0] = _lib.AdjointItem(mats[0].handle, 0, v[0].data_ptr(), g[0].data_ptr())
    h = dm.ctypes.c_void_p()
    # 4: the lowest bit no adjoint-plan flag uses
    assert _lib.load().dose_adjoint_plan_create(arr, 1, 4, None, dm.ctypes.byref(h)) == _lib.ERR_INVALID_ARGUMENT
    arr[0] = _lib.AdjointItem(mats[0].handle, 1, v[0].data_ptr(), g[0].data_ptr())
    assert _lib.load().dose_adjoint_plan_create(arr, 1, 0, None, dm.ctypes.byref(h)) == _lib.ERR_INVALID_ARGUMENT
    assert _lib.load().dose_adjoint_plan_create(arr, 0, 0, None, dm.ctypes.byref(h)) == _lib.ERR_INVALID_ARGUMENT
    # a matrix without entries next to one with entries: its g is +0
    E = dm.DoseMatrix(np.zeros(mats[0].n_rows + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 9,
                      "fp16", transpose="slabs")
    gE = torch.full((9,), np.nan, device=dev)
    plan = dm.AdjointPlan([(E, v[0], gE), (mats[0], v[0], g[0])])
    plan.launch()
    torch.cuda.synchronize()
    assert torch.equal(_bits(gE), torch.zeros(9, dtype=torch.int32, device=dev))
    assert torch.equal(_bits(g[0]), _bits(mats[0].adjoint(v[0])))
    plan.close()
    for A in mats + rows + e4 + [plain, E]:
        A.close()


@pytest.mark.parametrize("fmt", ["fp16", "fp8e4m3_rowscale"])
def test_adjoint_plan_accumulate(fmt, dev):
    """DOSE_ADJOINT_ACCUMULATE: each beam's gradient summed over the
    scenarios by the plan (g_b = sum_s A_sb^T v_s) against the oracle's FP64
    sum; the same bits on every replay; one item per output gives the plain
    adjoint's bits; spot rows and partly overlapping outputs are refused."""
    S, B = 2, 3
    specs = dosegen.robust_scenarios(0.04, S, B)
    host = [dosegen.csr(sp) for sp in specs]
    mats = [dm.DoseMatrix(rp, cols, vals, sp.n_cols, fmt, transpose="slabs")
            for sp, (rp, cols, vals) in zip(specs, host)]
    n = mats[0].n_rows
    vs = [torch.from_numpy(dosegen.signed_values(dosegen.SEED0, 80 + s, n)).cuda() for s in range(S)]
    gs = [torch.full((specs[b].n_cols,), np.nan, device=dev) for b in range(B)]
    plan = dm.AdjointPlan([(mats[s * B + b], vs[s], gs[b]) for s in range(S) for b in range(B)], accumulate=True)
    plan.launch()
    torch.cuda.synchronize()
    first = [g.clone() for g in gs]
    for b in range(B):
        ref = np.zeros(specs[b].n_cols)
        scale = np.zeros(specs[b].n_cols)
        for s in range(S):
            rp, cols, vals = host[s * B + b]
            dec, _ = oracle.decode_matrix(fmt, rp, vals)
            vh = vs[s].cpu().numpy()
            ref += oracle.spmv_T(rp, cols, dec, vh, specs[b].n_cols)
            scale += oracle.spmv_T(rp, cols, np.abs(dec), np.abs(vh), specs[b].n_cols)
        err = oracle.max_scaled_err(gs[b].cpu().numpy(), ref, scale)
        _say(f"accumulated beam {b} ({fmt}): max scaled err {err:.3e}")
        assert err <= 1e-5, (b, err)
    for g in gs:
        g.fill_(np.nan)
    plan.launch()
    torch.cuda.synchronize()
    for g, f in zip(gs, first):
        assert torch.equal(_bits(g), _bits(f))
    plan.close()
    # one item per output: the plain adjoint's bits
    one = [torch.empty(specs[b].n_cols, device=dev) for b in range(B)]
    p1 = dm.AdjointPlan([(mats[b], vs[0], one[b]) for b in range(B)], accumulate=True)
    p1.launch()
    torch.cuda.synchronize()
    for b in range(B):
        assert torch.equal(_bits(one[b]), _bits(mats[b].adjoint(vs[0]))), b
    p1.close()
    # refused: spot rows; outputs that overlap without being the same
    R = dm.DoseMatrix(*host[0], specs[0].n_cols, fmt, transpose=True)
    with pytest.raises(dm.DoseError) as e:
        dm.AdjointPlan([(R, vs[0], one[0])], accumulate=True)
    assert e.value.code == _lib.ERR_UNSUPPORTED
    big = torch.zeros(specs[0].n_cols + 8, device=dev)
    with pytest.raises(dm.DoseError) as e:
        dm.AdjointPlan([(mats[0], vs[0], big[:specs[0].n_cols]), (mats[3], vs[1], big[8:])], accumulate=True)
    assert e.value.code == _lib.ERR_INVALID_ARGUMENT
    # without accumulate a shared output stays refused
    with pytest.raises(dm.DoseError) as e:
        dm.AdjointPlan([(mats[0], vs[0], one[0]), (mats[3], vs[1], one[0])])
    assert e.value.code == _lib.ERR_INVALID_ARGUMENT
    R.close()
    for A in mats:
        A.close()


@pytest.mark.parametrize("mode", ["expected", "worst"])
def test_robust_problem_step(mode, dev):
    """RobustProblem.step: the robust objective's values equal a direct
    scenario_objective on the plan's beam doses (bitwise), and each beam's
    gradient is the oracle's FP64 sum over the scenarios of A_sb^T of the
    step's c_s-weighted seeds; updated spot weights are read at the next step."""
    S, B = 2, 3
    specs = dosegen.robust_scenarios(0.04, S, B)
    host = [dosegen.csr(sp) for sp in specs]
    mats = [[dm.DoseMatrix(*host[s * B + b], specs[s * B + b].n_cols, "fp16", transpose="slabs")
             for b in range(B)] for s in range(S)]
    n = mats[0][0].n_rows
    rng = np.random.default_rng(90)
    xs = [torch.from_numpy(dosegen.spot_weights(dosegen.SEED0, 90 + b, specs[b].n_cols) * np.float32(4)).cuda()
          for b in range(B)]
    p = torch.from_numpy(rng.choice([0.0, 20.0, 60.0], size=n).astype(np.float32)).cuda()
    w = torch.from_numpy(rng.choice([1.0, 10.0], size=n).astype(np.float32)).cuda()
    prob = torch.tensor([0.25, 0.75], dtype=torch.float64, device=dev) if mode == "expected" else None
    R = dm.RobustProblem(mats, xs, p, w, prob=prob, mode=mode)
    for rep in range(2):
        out, grads = R.step()
        torch.cuda.synchronize()
        ref_out = dm.scenario_objective(R.part, p, w, prob=prob)
        assert torch.equal(out.view(torch.int64), ref_out.view(torch.int64)), rep
        ws = R.wseed.cpu().numpy()
        for b in range(B):
            g_ref = np.zeros(specs[b].n_cols)
            scale = np.zeros(specs[b].n_cols)
            for s in range(S):
                rp, cols, vals = host[s * B + b]
                dec, _ = oracle.decode_matrix("fp16", rp, vals)
                g_ref += oracle.spmv_T(rp, cols, dec, ws[s], specs[b].n_cols)
                scale += oracle.spmv_T(rp, cols, np.abs(dec), np.abs(ws[s]), specs[b].n_cols)
            err = oracle.max_scaled_err(grads[b].cpu().numpy(), g_ref, scale)
            _say(f"robust problem ({mode}) step {rep} beam {b}: max scaled err {err:.3e}")
            assert err <= 1e-5, (rep, b, err)
        for x in xs:
            x.mul_(0.5)  # the next step reads the new weights
    R.close()
    for row in mats:
        for A in row:
            A.close()
