"""The boundary's contracts beyond plain parity.

* dose_spmv_batched is asynchronous: its item tables go through a ring of
  pinned slots, so many calls in a row without a synchronisation (cycling the
  ring several times, each call with its own inputs and outputs) must each
  give the plain products bit for bit; items without rows or entries are
  accepted; more items than one slot holds are refused.
* The binding refuses strided or misshapen x / y for batched items.
* dose_robust_seed forms the robust gradient's seeds c_s g seed_s (c_s from
  the oracle's robust weights of the GPU's own scenario objectives), rounded
  once from FP64.
* FP64 spot weights run the FP64 adjoint in autograd (the paper's
  half/double arithmetic end to end).
"""
import numpy as np
import pytest
import torch

import dosegen
import oracle
import paper_2103_09683_amd as dm

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def _mats(fmt="fp16", n=3, scale=0.02):
    specs = dosegen.robust_batch(scale)[:n]
    out = []
    for s in specs:
        rp, cols, vals = dosegen.csr(s)
        out.append((s, dm.DoseMatrix(rp, cols, vals, s.n_cols, fmt, transpose=True)))
    return out


def test_batched_calls_in_a_row_without_sync(dev):
    mats = _mats()
    n_calls = 40  # more than twice the ring's 16 slots
    _say(f"batched async: {n_calls} calls, {len(mats)} items each")
    xs, ys = [], []
    for c in range(n_calls):
        e = []
        for s, A in mats:
            X = torch.from_numpy(np.stack([dosegen.spot_weights(s.seed, 100 * c + r, s.n_cols)
                                           for r in range(4)], 1)).cuda()
            Y = torch.full((s.n_rows, 4), np.nan, device=dev)
            e.append((A, X, Y))
        xs.append(e)
    for e in xs:
        dm.spmv_batched(e)  # no synchronisation between calls
    torch.cuda.synchronize()
    for c in (0, 1, 15, 16, 17, 39):
        for A, X, Y in xs[c]:
            for r in range(4):
                y_plain = A.spmv(X[:, r].contiguous()).cpu().numpy()
                np.testing.assert_array_equal(_bits(Y[:, r].cpu().numpy()), _bits(y_plain))
    for _, A in mats:
        A.close()


def test_batched_accepts_items_without_rows_or_entries(dev):
    (s, A), = _mats(n=1)
    empty_rows = dm.DoseMatrix(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 7)
    no_entries = dm.DoseMatrix(np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 3)
    x = torch.from_numpy(dosegen.spot_weights(s.seed, 1, s.n_cols)).cuda()
    y = torch.full((s.n_rows,), np.nan, device=dev)
    y0 = torch.full((0,), np.nan, device=dev)
    y5 = torch.full((5,), np.nan, device=dev)
    dm.spmv_batched([(empty_rows, torch.zeros(7, device=dev), y0), (A, x, y),
                     (no_entries, torch.zeros(3, device=dev), y5)])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_bits(y.cpu().numpy()), _bits(A.spmv(x).cpu().numpy()))
    np.testing.assert_array_equal(_bits(y5.cpu().numpy()), np.zeros(5, np.uint32))
    for M in (A, empty_rows, no_entries):
        M.close()


def test_batched_refuses_more_items_than_a_slot_holds(dev):
    rp = np.array([0, 1, 2], np.int64)
    A = dm.DoseMatrix(rp, np.array([0, 1], np.int32), np.array([1.0, 2.0], np.float32), 2)
    x = torch.ones(2, device=dev)
    ys = torch.zeros(2049, 2, device=dev)
    ok = [(A, x, ys[i]) for i in range(2048)]
    dm.spmv_batched(ok)
    torch.cuda.synchronize()
    assert torch.equal(ys[:2048], torch.tensor([1.0, 2.0], device=dev).expand(2048, 2))
    with pytest.raises(dm.DoseError) as err:
        dm.spmv_batched(ok + [(A, x, ys[2048])])
    assert err.value.code == dm._lib.ERR_UNSUPPORTED
    A.close()


def test_batched_binding_refuses_strided_or_misshapen_vectors(dev):
    (s, A), = _mats(n=1)
    xt = torch.rand(4, s.n_cols, device=dev).T  # [n_cols][4] as a transposed view
    Y = torch.zeros(s.n_rows, 4, device=dev)
    with pytest.raises(TypeError):
        dm.spmv_batched([(A, xt, Y)])
    with pytest.raises(TypeError):
        dm.BatchPlan([(A, xt, Y)])
    X = xt.contiguous()
    with pytest.raises(TypeError):
        dm.spmv_batched([(A, X, torch.zeros(4, s.n_rows, device=dev).T)])
    with pytest.raises(ValueError):
        dm.spmv_batched([(A, X, torch.zeros(s.n_rows, 2, device=dev))])
    with pytest.raises(ValueError):
        dm.spmv_batched([(A, X.reshape(-1), torch.zeros(s.n_rows * 4, device=dev))])
    A.close()


@pytest.mark.parametrize("mode,with_prob", [("expected", True), ("expected", False), ("worst", False)])
def test_robust_seed_against_oracle_weights(dev, mode, with_prob):
    n_scen, n = 7, 3001
    g = np.random.default_rng(31)
    seed_h = (g.standard_normal((n_scen, n)) * 10).astype(np.float32)
    f_h = g.random(n_scen) * 100
    f_h[4] = f_h.max() + 1.0
    f_h[5] = f_h[4]  # a tie: the first of them is the worst
    out_h = np.concatenate([f_h, [f_h.max(), 0.0, 4.0]])
    prob_h = g.random(n_scen)
    prob_h /= prob_h.sum()
    gs = 0.75
    seed, out = torch.from_numpy(seed_h).cuda(), torch.from_numpy(out_h).cuda()
    prob = torch.from_numpy(prob_h).cuda() if with_prob else None
    gscale = torch.tensor([gs], dtype=torch.float64, device=dev)
    w = dm.robust_seed(seed, mode, out=out, prob=prob, grad_scale=gscale).cpu().numpy()
    c = oracle.robust_weights(f_h, prob_h if with_prob else None, mode)
    ref = c[:, None] * gs * seed_h.astype(np.float64)
    # one rounding of the FP64 product to FP32
    assert np.all(np.abs(w - ref) <= 2.0 ** -24 * np.abs(ref))
    if mode == "worst":
        assert np.count_nonzero(w[[0, 1, 2, 3, 5, 6]]) == 0 and np.all(w[4] == (gs * seed_h[4]).astype(np.float32))
    # in place, and without an outer derivative
    s2 = seed.clone()
    dm.robust_seed(s2, mode, out=out, prob=prob, wseed=s2)
    ref1 = (c[:, None] * seed_h.astype(np.float64)).astype(np.float32)
    np.testing.assert_array_equal(_bits(s2.cpu().numpy()), _bits(ref1))


def test_robust_seed_argument_errors(dev):
    seed = torch.zeros(3, 10, device=dev)
    out = torch.zeros(6, dtype=torch.float64, device=dev)
    lib = dm._lib.load()
    st = torch.cuda.current_stream().cuda_stream
    p, q = seed.data_ptr(), torch.zeros(3, 10, device=dev).data_ptr()
    assert lib.dose_robust_seed(0, 10, 0, None, None, None, p, q, st) == dm._lib.ERR_INVALID_ARGUMENT
    assert lib.dose_robust_seed(3, 10, 2, None, None, None, p, q, st) == dm._lib.ERR_INVALID_ARGUMENT
    assert lib.dose_robust_seed(3, 10, 1, None, None, None, p, q, st) == dm._lib.ERR_INVALID_ARGUMENT
    assert lib.dose_robust_seed(3, 10, 0, None, None, None, p, p + 4, st) == dm._lib.ERR_INVALID_ARGUMENT
    assert lib.dose_robust_seed(3, 10, 0, None, None, None, p + 2, q, st) == dm._lib.ERR_INVALID_ARGUMENT
    assert lib.dose_robust_seed(3, 10, 1, out.data_ptr(), None, None, p, q, st) == dm._lib.OK
    assert lib.dose_robust_seed(3, 0, 0, None, None, None, None, None, st) == dm._lib.OK
    torch.cuda.synchronize()


def test_fp64_weights_run_the_fp64_adjoint_in_autograd(dev):
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16", transpose=True)
    x_h = dosegen.spot_weights(spec.seed, 0, spec.n_cols)
    v_h = dosegen.signed_values(spec.seed, 5, spec.n_rows)
    x = torch.from_numpy(x_h.astype(np.float64)).cuda().requires_grad_(True)
    v = torch.from_numpy(v_h.astype(np.float64)).cuda()
    d = dm.dose(x, A)
    assert d.dtype == torch.float64
    (d * v).sum().backward()
    assert x.grad.dtype == torch.float64
    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    g_ref = oracle.spmv_T(rp, cols, dec, v_h, spec.n_cols)
    scale = oracle.spmv_T(rp, cols, np.abs(dec), np.abs(v_h), spec.n_cols)
    # FP64 sums: far inside what an FP32 adjoint (about 2^-24 of the scale) could reach
    assert oracle.max_scaled_err(x.grad.cpu().numpy(), g_ref, scale) <= 1e-12
    # and the forward pass in FP64 against the oracle
    assert oracle.max_rel_err(d.detach().cpu().numpy(), oracle.spmv(rp, cols, dec, x_h)) <= 1e-12
    A.close()


def test_objective_backward_scales_the_seed_in_the_library(dev):
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16", transpose=True)
    p_h, w_h = dosegen.objective_masks(spec.nx, spec.ny, spec.nz)
    p, w = torch.from_numpy(p_h).cuda(), torch.from_numpy(w_h).cuda()
    x = torch.from_numpy(dosegen.spot_weights(spec.seed, 0, spec.n_cols)).cuda().requires_grad_(True)
    d = dm.dose(x, A)
    f = dm.DoseObjective.apply(d, p, w)
    (3.0 * f).backward()
    seed = torch.empty_like(d)
    dm.objective(d.detach(), p, w, seed=seed)
    seed_h = seed.cpu().numpy().astype(np.float64)
    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    g_ref = oracle.spmv_T(rp, cols, dec, 3.0 * seed_h, spec.n_cols)
    scale = oracle.spmv_T(rp, cols, np.abs(dec), np.abs(3.0 * seed_h), spec.n_cols)
    assert oracle.max_scaled_err(x.grad.cpu().numpy(), g_ref, scale) <= 1e-5 + 2.0 ** -24
    A.close()
