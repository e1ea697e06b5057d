"""The entry point that allocates nothing (dose_scenario_objective_noalloc:
its partial sums live in the library's static scratch array) against the
allocating dose_scenario_objective, bit for bit, through the C ABI: two calls
in a row, the second with a smaller input (the scratch keeps the first call's
partial sums), then an empty grid; and the size limit of the scratch."""
import numpy as np
import pytest
import torch

from paper_2103_09683_amd import _lib

pytestmark = pytest.mark.gpu


def _case(n_scen, n_beams, n, seed):
    g = torch.Generator().manual_seed(seed)
    part = torch.rand(n_scen, n_beams, n, generator=g).cuda()
    p = (torch.randint(0, 3, (n,), generator=g).float() * 20.0).cuda()
    w = torch.where(torch.rand(n, generator=g) < 0.5, 1.0, 10.0).float().cuda()
    prob = torch.rand(n_scen, generator=g, dtype=torch.float64)
    prob = (prob / prob.sum()).cuda()
    return part, p, w, prob


def _run(fn, part, p, w, prob):
    n_scen, n_beams, n = part.shape
    d_out = torch.full((n_scen, n), float("nan"), device=part.device)
    seed = torch.full((n_scen, n), float("nan"), device=part.device)
    out = torch.full((n_scen + 3,), float("nan"), dtype=torch.float64, device=part.device)
    st = getattr(_lib.load(), fn)(n_scen, n_beams, n, part.data_ptr(), p.data_ptr(), w.data_ptr(),
                                 prob.data_ptr() if prob is not None else None, d_out.data_ptr(),
                                 seed.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return st, d_out, seed, out


def _bits32(t):
    return t.cpu().numpy().view(np.uint32)


def _bits64(t):
    return t.cpu().numpy().view(np.uint64)


def test_noalloc_equals_allocating_call_twice(dev):
    cases = [(9, 4, 1_048_576 + 13, 1, True), (3, 2, 5_000, 2, False), (2, 1, 0, 3, True)]
    for n_scen, n_beams, n, sd, with_prob in cases:
        print(f"no-alloc case {n_scen} x {n_beams} x {n}", flush=True)
        part, p, w, prob = _case(n_scen, n_beams, n, sd)
        prob = prob if with_prob else None
        st_a, d_a, s_a, o_a = _run("dose_scenario_objective", part, p, w, prob)
        st_b, d_b, s_b, o_b = _run("dose_scenario_objective_noalloc", part, p, w, prob)
        torch.cuda.synchronize()
        assert st_a == _lib.OK and st_b == _lib.OK
        assert np.array_equal(_bits32(d_a), _bits32(d_b))
        assert np.array_equal(_bits32(s_a), _bits32(s_b))
        assert np.array_equal(_bits64(o_a), _bits64(o_b))
        assert np.all(np.isfinite(o_b.cpu().numpy()))


def test_noalloc_rejects_sizes_beyond_the_scratch(dev):
    # n = 4 Mi voxels takes 1,024 partial sums per scenario: 64 scenarios fit
    # the 65,536-double scratch, 65 do not
    n = 4 * 1024 * 1024
    part, p, w, _ = _case(65, 1, n, 4)
    st, _, _, _ = _run("dose_scenario_objective_noalloc", part, p, w, None)
    assert st == _lib.ERR_INVALID_ARGUMENT
    st, _, _, o = _run("dose_scenario_objective_noalloc", part[:64].contiguous(), p, w, None)
    torch.cuda.synchronize()
    assert st == _lib.OK
    st_a, _, _, o_a = _run("dose_scenario_objective", part[:64].contiguous(), p, w, None)
    torch.cuda.synchronize()
    assert np.array_equal(_bits64(o), _bits64(o_a))
