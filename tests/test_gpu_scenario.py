"""GPU parity of the robust-optimisation epilogue (scenario dose as the sum of
its beams' doses, per-scenario FP64 objective, worst case and expectation)
against the CPU oracle.

The beam doses come from one batched launch (one item per beam and scenario)
and are themselves checked against the oracle's products (relative 1e-5).  On
the GPU's own beam doses the epilogue must give: the scenario dose bit for bit
as the FP32 sum in ascending beam order, within (n_beams - 1) 2^-24 of the
oracle's FP64 sum (all doses are non-negative); each f_s within 1e-13 of the
oracle's objective of the same FP32 dose (only the FP64 summation order
differs); the seeds bit for bit; the worst case, its scenario and the
expectation exactly as the oracle forms them from the GPU's f_s.
"""
import numpy as np
import pytest
import torch

import dosegen
import oracle
import paper_2103_09683_amd as dm
from paper_2103_09683_amd import _lib

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _say(*a):
    print(*a, flush=True)


def _bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def _scenario_case(n_scen, n_beams, fmt="fp16"):
    """A shared 41 x 40 x 7 grid (11,480 voxels: three reduction chunks, the
    last one ragged) with n_scen x n_beams beam matrices."""
    specs = dosegen.robust_scenarios(7 / 64, n_scen, n_beams, nx=41, ny=40, spots_per_line=20)
    mats, host, xs = [], [], []
    for b in range(n_beams):
        xs.append(dosegen.spot_weights(dosegen.SEED0 + 6, b, specs[b].n_cols))
    for sp in specs:
        rp, cols, vals = dosegen.csr(sp)
        mats.append(dm.DoseMatrix(rp, cols, vals, sp.n_cols, fmt))
        host.append((rp, cols, vals))
    n = specs[0].n_rows
    g = np.random.default_rng(77)
    p = g.choice([0.0, 20.0, 60.0], size=n).astype(np.float32)
    w = g.choice([1.0, 10.0], size=n).astype(np.float32)
    return specs, mats, host, xs, p, w


def _beam_doses(mats, xs, n_scen, n_beams, n):
    part = torch.empty(n_scen, n_beams, n, dtype=torch.float32, device="cuda")
    xd = [torch.from_numpy(x).cuda() for x in xs]
    dm.spmv_batched([(mats[s * n_beams + b], xd[b], part[s, b]) for s in range(n_scen) for b in range(n_beams)])
    return part


@pytest.mark.parametrize("n_scen,n_beams,with_prob", [(3, 2, True), (4, 3, False), (9, 4, True)])
def test_scenario_epilogue_parity(dev, n_scen, n_beams, with_prob):
    _say(f"scenario epilogue: {n_scen} scenarios x {n_beams} beams, prob={with_prob}")
    specs, mats, host, xs, p, w = _scenario_case(n_scen, n_beams)
    n = specs[0].n_rows
    part = _beam_doses(mats, xs, n_scen, n_beams, n)
    pd, wd = torch.from_numpy(p).cuda(), torch.from_numpy(w).cuda()
    prob_h = np.random.default_rng(5).integers(1, 9, n_scen).astype(np.float64)
    prob_h /= prob_h.sum()
    prob = torch.from_numpy(prob_h).cuda() if with_prob else None
    d_out = torch.empty(n_scen, n, dtype=torch.float32, device=dev)
    seed = torch.empty(n_scen, n, dtype=torch.float32, device=dev)
    out = dm.scenario_objective(part, pd, wd, prob=prob, d_out=d_out, seed=seed).cpu().numpy()
    part_h = part.cpu().numpy()
    d_h, seed_h = d_out.cpu().numpy(), seed.cpu().numpy()

    # beam doses against the oracle's products
    d_ref = np.zeros((n_scen, n))
    for s in range(n_scen):
        for b in range(n_beams):
            rp, cols, vals = host[s * n_beams + b]
            dec, _ = oracle.decode_matrix("fp16", rp, vals)
            y_ref = oracle.spmv(rp, cols, dec, xs[b])
            assert oracle.max_rel_err(part_h[s, b], y_ref) <= TOL
            d_ref[s] += y_ref

    f_gpu = out[:n_scen]
    for s in range(n_scen):
        # the FP32 sum in ascending beam order, bit for bit
        acc = part_h[s, 0].copy()
        for b in range(1, n_beams):
            acc = acc + part_h[s, b]
        np.testing.assert_array_equal(_bits(d_h[s]), _bits(acc))
        # within (n_beams - 1) FP32 roundings of the oracle's sum of the same beam doses
        exact = oracle.beam_sum(part_h[s].astype(np.float64))
        assert oracle.max_rel_err(d_h[s], exact) <= max(n_beams - 1, 0) * 2.0 ** -24 * 1.0001
        d64 = d_h[s].astype(np.float64)
        f_ref = oracle.objective(d64, p, w)
        assert abs(f_gpu[s] - f_ref) <= 1e-13 * abs(f_ref)
        np.testing.assert_array_equal(_bits(seed_h[s]), _bits(oracle.objective_seed(d64, p, w).astype(np.float32)))
        # end to end against the oracle's FP64 scenario dose: each voxel's dose
        # is within TOL + n_beams 2^-24 relative (all terms are non-negative)
        delta = (TOL + n_beams * 2.0 ** -24) * d_ref[s]
        bound = np.sum(w * (2 * np.abs(d_ref[s] - p) * delta + delta * delta))
        assert abs(f_gpu[s] - oracle.objective(d_ref[s], p, w)) <= bound + 1e-9

    worst, arg, expected = oracle.robust(f_gpu, prob_h if with_prob else None)
    assert out[n_scen] == worst and int(out[n_scen + 2]) == arg and out[n_scen + 2] == float(arg)
    assert out[n_scen + 1] == expected
    for A in mats:
        A.close()


def test_single_scenario_single_beam_equals_objective(dev):
    """One scenario of one beam is the plain objective, bit for bit; the epilogue
    is repeatable bit for bit and works without its optional outputs."""
    specs, mats, host, xs, p, w = _scenario_case(1, 1)
    n = specs[0].n_rows
    part = _beam_doses(mats, xs, 1, 1, n)
    pd, wd = torch.from_numpy(p).cuda(), torch.from_numpy(w).cuda()
    d_out = torch.empty(1, n, dtype=torch.float32, device=dev)
    seed = torch.empty(1, n, dtype=torch.float32, device=dev)
    out = dm.scenario_objective(part, pd, wd, d_out=d_out, seed=seed).cpu().numpy()
    seed1 = torch.empty(n, dtype=torch.float32, device=dev)
    f1 = dm.objective(part[0, 0], pd, wd, seed=seed1).item()
    assert out[0] == f1 and out[1] == f1 and out[2] == f1 and out[3] == 0.0
    np.testing.assert_array_equal(_bits(d_out.cpu().numpy()[0]), _bits(part.cpu().numpy()[0, 0]))
    np.testing.assert_array_equal(_bits(seed.cpu().numpy()[0]), _bits(seed1.cpu().numpy()))
    again = dm.scenario_objective(part, pd, wd).cpu().numpy()
    np.testing.assert_array_equal(again, out)
    mats[0].close()


def test_worst_case_ties_and_empty_grid(dev):
    """Identical scenarios tie: the first is the worst; an empty grid gives zeros."""
    n = 5000
    g = np.random.default_rng(3)
    one = g.uniform(0, 70, n).astype(np.float32)
    part = torch.from_numpy(np.stack([np.stack([one * 0.5, one * 0.5])] * 3)).cuda()  # 3 x 2 x n
    p = torch.from_numpy(np.full(n, 30.0, np.float32)).cuda()
    w = torch.ones(n, device=dev)
    out = dm.scenario_objective(part, p, w).cpu().numpy()
    assert out[0] == out[1] == out[2] and out[3] == out[0] and out[5] == 0.0
    assert out[4] == (out[0] + out[1] + out[2]) / 3.0
    z = torch.empty(4, 2, 0, device=dev)
    e = torch.empty(0, device=dev)
    out = dm.scenario_objective(z, e, e).cpu().numpy()
    np.testing.assert_array_equal(out, np.zeros(7))


def test_scenario_argument_errors(dev):
    n = 1000
    part = torch.ones(2, 3, n, device=dev)
    p, w = torch.zeros(n, device=dev), torch.ones(n, device=dev)
    d_out = torch.empty(2, n, device=dev)
    with pytest.raises(dm.DoseError):  # no scenario
        dm.scenario_objective(torch.ones(0, 3, n, device=dev), p, w)
    with pytest.raises(dm.DoseError):  # seed and dose written to the same memory
        dm.scenario_objective(part, p, w, d_out=d_out, seed=d_out)
    out = torch.empty(8, dtype=torch.float64, device=dev)
    # scenario doses written over the beam doses
    st = _lib.load().dose_scenario_objective(2, 3, n, part.data_ptr(), p.data_ptr(), w.data_ptr(), None,
                                             part.data_ptr(), None, out.data_ptr(), None)
    assert st == -1
    for bad in [
        (0, 3, n, part.data_ptr()),          # no scenario
        (2, 0, n, part.data_ptr()),          # no beam
        (2, 3, -1, part.data_ptr()),         # negative size
        (65537, 1, 1, part.data_ptr()),      # too many scenarios
        (2, 3, n, part.data_ptr() + 2),      # misaligned beam doses
        (2, 3, n, None),                     # null beam doses
    ]:
        st = _lib.load().dose_scenario_objective(*bad, p.data_ptr(), w.data_ptr(), None, None, None,
                                                 out.data_ptr(), None)
        assert st == -1, bad
    st = _lib.load().dose_scenario_objective(2, 3, n, part.data_ptr(), p.data_ptr(), w.data_ptr(), None, None,
                                             None, out.data_ptr() + 4, None)  # misaligned doubles
    assert st == -1
    torch.cuda.synchronize()


def _random_epilogue_inputs(n_scen, n_beams, n, seed=11):
    g = np.random.default_rng(seed)
    part = g.uniform(0, 30, (n_scen, n_beams, n)).astype(np.float32)
    part[:, :, g.random(n) < 0.3] = 0.0  # voxels outside every beam
    p = g.choice([0.0, 20.0, 60.0], size=n).astype(np.float32)
    w = g.choice([1.0, 10.0], size=n).astype(np.float32)
    return part, p, w


def _offset(a: np.ndarray, floats: int):
    """A contiguous device copy of a whose data starts `floats` floats into its buffer."""
    buf = torch.empty(a.size + floats, dtype=torch.float32, device="cuda")
    t = buf[floats:].view(a.shape)
    t.copy_(torch.from_numpy(a))
    return t


@pytest.mark.parametrize("n", [10003, 4097, 6])
def test_ragged_grid_parity(dev, n):
    """A voxel count that is not a multiple of 4 takes the 4-byte path: the same
    checks against the oracle as above."""
    n_scen, n_beams = 5, 3
    _say(f"scenario epilogue ragged grid: n={n}")
    part_h, p, w = _random_epilogue_inputs(n_scen, n_beams, n)
    prob_h = np.array([0.1, 0.3, 0.2, 0.25, 0.15])
    d_out = torch.empty(n_scen, n, dtype=torch.float32, device=dev)
    seed = torch.empty(n_scen, n, dtype=torch.float32, device=dev)
    out = dm.scenario_objective(torch.from_numpy(part_h).cuda(), torch.from_numpy(p).cuda(),
                                torch.from_numpy(w).cuda(), prob=torch.from_numpy(prob_h).cuda(),
                                d_out=d_out, seed=seed).cpu().numpy()
    d_h, seed_h = d_out.cpu().numpy(), seed.cpu().numpy()
    for s in range(n_scen):
        acc = part_h[s, 0].copy()
        for b in range(1, n_beams):
            acc = acc + part_h[s, b]
        np.testing.assert_array_equal(_bits(d_h[s]), _bits(acc))
        assert oracle.max_rel_err(d_h[s], oracle.beam_sum(part_h[s].astype(np.float64))) <= 2.0001 * 2.0 ** -24
        d64 = d_h[s].astype(np.float64)
        f_ref = oracle.objective(d64, p, w)
        assert abs(out[s] - f_ref) <= 1e-13 * abs(f_ref)
        np.testing.assert_array_equal(_bits(seed_h[s]), _bits(oracle.objective_seed(d64, p, w).astype(np.float32)))
    worst, arg, expected = oracle.robust(out[:n_scen], prob_h)
    assert out[n_scen] == worst and out[n_scen + 1] == expected and int(out[n_scen + 2]) == arg


@pytest.mark.parametrize("n_beams", [3, 9])
def test_aligned_and_misaligned_arrays_agree_bitwise(dev, n_beams):
    """The 16-byte path (aligned arrays, n a multiple of 4; the beam count a
    template argument up to 8 beams, a loop beyond) and the 4-byte path add the
    same terms in the same order: every output is bitwise equal, and the
    scenario doses are the FP32 sums in ascending beam order."""
    n_scen, n = 4, 12288
    _say(f"scenario epilogue aligned vs misaligned: {n_beams} beams")
    part_h, p, w = _random_epilogue_inputs(n_scen, n_beams, n, seed=12)
    res = []
    for off in (0, 1):
        d_out = _offset(np.zeros((n_scen, n), np.float32), off)
        seed = _offset(np.zeros((n_scen, n), np.float32), off)
        out = dm.scenario_objective(_offset(part_h, off), _offset(p, off), _offset(w, off), d_out=d_out,
                                    seed=seed).cpu().numpy()
        res.append((out, d_out.cpu().numpy(), seed.cpu().numpy()))
    np.testing.assert_array_equal(res[0][0], res[1][0])
    np.testing.assert_array_equal(_bits(res[0][1]), _bits(res[1][1]))
    np.testing.assert_array_equal(_bits(res[0][2]), _bits(res[1][2]))
    for s in range(n_scen):
        acc = part_h[s, 0].copy()
        for b in range(1, n_beams):
            acc = acc + part_h[s, b]
        np.testing.assert_array_equal(_bits(res[0][1][s]), _bits(acc))
        f_ref = oracle.objective(res[0][1][s].astype(np.float64), p, w)
        assert abs(res[0][0][s] - f_ref) <= 1e-13 * abs(f_ref)
    # the plain objective takes the same two paths
    d = part_h[0, 0]
    f_al = dm.objective(_offset(d, 0), _offset(p, 0), _offset(w, 0)).item()
    f_mis = dm.objective(_offset(d, 1), _offset(p, 1), _offset(w, 1)).item()
    assert f_al == f_mis == dm.scenario_objective(_offset(part_h[:1, :1].copy(), 0), _offset(p, 0),
                                                  _offset(w, 0)).cpu().numpy()[0]


@pytest.mark.parametrize("mode", ["expected", "worst"])
def test_robust_gradient_through_autograd(dev, mode):
    """x_b -> beam doses (DoseSpMV) -> robust objective (ScenarioObjective): the
    spot-weight gradient of beam b must be sum_s c_s A_sb^T seed_s, with the
    GPU's own seeds and c_s the probabilities (expected) or the worst
    scenario's indicator (worst), each adjoint within 1e-5 of |A|^T |c seed|
    (the adjoint's bound) plus the FP32 sum over scenarios."""
    n_scen, n_beams = 3, 2
    _say(f"robust gradient: mode={mode}")
    specs = dosegen.robust_scenarios(7 / 64, n_scen, n_beams, nx=41, ny=40, spots_per_line=20)
    mats, host = [], []
    for sp in specs:
        rp, cols, vals = dosegen.csr(sp)
        mats.append(dm.DoseMatrix(rp, cols, vals, sp.n_cols, "fp16", transpose=True))
        host.append((rp, cols, vals))
    n = specs[0].n_rows
    g = np.random.default_rng(78)
    pd = torch.from_numpy(g.choice([0.0, 20.0, 60.0], size=n).astype(np.float32)).cuda()
    wd = torch.from_numpy(g.choice([1.0, 10.0], size=n).astype(np.float32)).cuda()
    prob_h = np.array([0.5, 0.2, 0.3])
    prob = torch.from_numpy(prob_h).cuda()
    xs = [torch.from_numpy(dosegen.spot_weights(dosegen.SEED0 + 6, b, specs[b].n_cols)).cuda().requires_grad_(True)
          for b in range(n_beams)]
    part = torch.stack([torch.stack([dm.dose(xs[b], mats[s * n_beams + b]) for b in range(n_beams)])
                        for s in range(n_scen)])
    f = dm.ScenarioObjective.apply(part, pd, wd, prob if mode == "expected" else None, mode)
    f.backward()

    seed = torch.empty(n_scen, n, dtype=torch.float32, device=dev)
    out = dm.scenario_objective(part.detach(), pd, wd, prob=prob, seed=seed).cpu().numpy()
    seed_h = seed.cpu().numpy().astype(np.float64)
    if mode == "expected":
        assert f.item() == out[n_scen + 1]
    else:
        assert f.item() == out[n_scen]
    c = oracle.robust_weights(out[:n_scen], prob_h if mode == "expected" else None, mode)
    for b in range(n_beams):
        n_cols = specs[b].n_cols
        g_ref = np.zeros(n_cols)
        scale = np.zeros(n_cols)
        for s in range(n_scen):
            rp, cols, vals = host[s * n_beams + b]
            dec, _ = oracle.decode_matrix("fp16", rp, vals)
            g_ref += c[s] * oracle.spmv_T(rp, cols, dec, seed_h[s], n_cols)
            scale += abs(c[s]) * oracle.spmv_T(rp, cols, np.abs(dec), np.abs(seed_h[s]), n_cols)
        grad = xs[b].grad.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(grad - g_ref) <= (TOL + (n_scen + 1) * 2.0 ** -24) * scale + 1e-30)
    for A in mats:
        A.close()


def test_robust_step_at_bench_size(dev):
    """The robust-plan step as the bench times it: 9 scenarios x 4 beams on the
    128 x 128 x 6 grid (98,304 voxels, about 4.8e8 stored entries), all beam
    doses in one autotuned graph plan, then the epilogue.  Every beam dose is
    checked against the oracle's product (relative 1e-5), the epilogue against
    the oracle on the GPU's beam doses as above."""
    n_scen, n_beams = 9, 4
    specs = dosegen.robust_scenarios(0.1, n_scen, n_beams)
    n = specs[0].n_rows
    _say(f"robust step at bench size: {n} voxels, {len(specs)} matrices")
    xs_h = [dosegen.spot_weights(dosegen.SEED0 + 6, b, specs[b].n_cols) for b in range(n_beams)]
    xs = [torch.from_numpy(x).cuda() for x in xs_h]
    part = torch.empty(n_scen, n_beams, n, dtype=torch.float32, device=dev)
    mats, entries, y_ref = [], [], []
    for m, sp in enumerate(specs):
        rp, cols, vals = dosegen.csr(sp)
        A = dm.DoseMatrix(rp, cols, vals, sp.n_cols, "fp16")
        mats.append(A)
        s, b = divmod(m, n_beams)
        entries.append((A, xs[b], part[s, b]))
        dec, _ = oracle.decode_matrix("fp16", rp, vals)
        y_ref.append(oracle.spmv(rp, cols, dec, xs_h[b]))
        del rp, cols, vals, dec
    plan = dm.BatchPlan(entries, autotune=True)
    plan.launch()
    g = np.random.default_rng(6)
    p = g.choice([0.0, 20.0, 60.0], size=n).astype(np.float32)
    w = g.choice([1.0, 10.0], size=n).astype(np.float32)
    d_out = torch.empty(n_scen, n, dtype=torch.float32, device=dev)
    out = dm.scenario_objective(part, torch.from_numpy(p).cuda(), torch.from_numpy(w).cuda(),
                                d_out=d_out).cpu().numpy()
    part_h, d_h = part.cpu().numpy(), d_out.cpu().numpy()
    for m in range(len(specs)):
        s, b = divmod(m, n_beams)
        assert oracle.max_rel_err(part_h[s, b], y_ref[m]) <= TOL, specs[m].name
    for s in range(n_scen):
        acc = part_h[s, 0].copy()
        for b in range(1, n_beams):
            acc = acc + part_h[s, b]
        np.testing.assert_array_equal(_bits(d_h[s]), _bits(acc))
        f_ref = oracle.objective(d_h[s].astype(np.float64), p, w)
        assert abs(out[s] - f_ref) <= 1e-13 * abs(f_ref)
    worst, arg, expected = oracle.robust(out[:n_scen])
    assert out[n_scen] == worst and out[n_scen + 1] == expected and int(out[n_scen + 2]) == arg
    plan.close()
    for A in mats:
        A.close()


@pytest.mark.parametrize("n_scen,n_beams", [(3, 2), (9, 4)])
@pytest.mark.parametrize("autotune", [False, True])
def test_scenario_plan_sums_beams_in_the_products(n_scen, n_beams, autotune, dev):
    """The scenario plan (one launch per beam, the first storing, the others
    adding) gives each scenario's dose bit for bit as the beam products
    followed by the epilogue's FP32 beam sum, on every graph replay (with
    eager work between replays), and so the same objectives."""
    specs, mats, host, xs, p, w = _scenario_case(n_scen, n_beams)
    n = specs[0].n_rows
    pd, wd = torch.from_numpy(p).cuda(), torch.from_numpy(w).cuda()
    part = _beam_doses(mats, xs, n_scen, n_beams, n)
    d_ref = torch.empty(n_scen, n, device=dev)
    out_ref = dm.scenario_objective(part, pd, wd, d_out=d_ref)
    torch.cuda.synchronize()
    xd = [torch.from_numpy(x).cuda() for x in xs]
    d = torch.full((n_scen, n), float("nan"), device=dev)
    plan = dm.ScenarioPlan([[mats[s * n_beams + b] for b in range(n_beams)] for s in range(n_scen)],
                           [[xd[b] for b in range(n_beams)] for _ in range(n_scen)], d, autotune=autotune)
    for rep in range(3):
        d.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        assert np.array_equal(_bits(d.cpu().numpy()), _bits(d_ref.cpu().numpy())), rep
        junk = torch.rand(1 << 20, device=dev).sum()  # eager work between replays
        del junk
    out = dm.scenario_objective(d.view(n_scen, 1, n), pd, wd)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint64), out_ref.cpu().numpy().view(np.uint64))
    plan.close()
    for A in mats:
        A.close()


def test_scenario_plan_argument_errors(dev):
    specs, mats, host, xs, p, w = _scenario_case(2, 2)
    n = specs[0].n_rows
    xd = [torch.from_numpy(x).cuda() for x in xs]
    grid = [[mats[s * 2 + b] for b in range(2)] for s in range(2)]
    with pytest.raises(ValueError):
        dm.ScenarioPlan(grid, [[xd[0], xd[1]]], torch.empty(2, n, device=dev))
    with pytest.raises(ValueError):
        dm.ScenarioPlan(grid, [[xd[0], xd[1]]] * 2, torch.empty(3, n, device=dev))
    lib = _lib.load()
    import ctypes
    ha = (ctypes.c_void_p * 4)(*[A.handle for s in grid for A in s])
    hx = (ctypes.c_void_p * 4)(*[x.data_ptr() for x in (xd[0], xd[1], xd[0], xd[1])])
    h = ctypes.c_void_p()
    d = torch.empty(2, n, device=dev)
    assert lib.dose_scenario_plan_create(ha, hx, 0, 2, d.data_ptr(), 0, None, ctypes.byref(h)) == _lib.ERR_INVALID_ARGUMENT
    assert lib.dose_scenario_plan_create(None, hx, 2, 2, d.data_ptr(), 0, None, ctypes.byref(h)) == _lib.ERR_INVALID_ARGUMENT
    # d overlapping a spot-weight vector
    hx2 = (ctypes.c_void_p * 4)(*[d.data_ptr()] * 4)
    assert lib.dose_scenario_plan_create(ha, hx2, 2, 2, d.data_ptr(), 0, None, ctypes.byref(h)) == _lib.ERR_INVALID_ARGUMENT
    for A in mats:
        A.close()
