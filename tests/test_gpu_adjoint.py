"""GPU parity of the adjoint g = A^T v, the stored transpose, the FP64
objective reductions and the autograd path, against the CPU oracle.

The adjoint's seed v is signed, so its error is measured componentwise
against |A|^T |v|: |g_j - g*_j| <= 1e-5 (|A|^T |v|)_j, and g_j must be
exactly 0 where that scale is 0.
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


@pytest.mark.parametrize("fmt", FORMATS)
def test_transpose_decodes_to_transpose_of_decoded(fmt, dev):
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    _say("transpose", fmt)
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, fmt, transpose=True)
    dec, _ = oracle.decode_matrix(fmt, rp, vals)
    t_rp, t_c, t_d = oracle.transpose(rp, cols, dec, spec.n_cols)
    rp_d, c_d, v_d = A.decode(part="AT")
    np.testing.assert_array_equal(rp_d, t_rp)
    np.testing.assert_array_equal(c_d, t_c)
    np.testing.assert_array_equal(_bits(v_d), _bits(t_d))
    A.close()


@pytest.mark.parametrize("fmt", FORMATS)
def test_adjoint_parity_small(fmt, dev):
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    v = dosegen.signed_values(spec.seed, 3, spec.n_rows)
    _say("adjoint", fmt)
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, fmt, transpose=True)
    g = A.adjoint(torch.from_numpy(v).cuda()).cpu().numpy()
    dec, _ = oracle.decode_matrix(fmt, rp, vals)
    g_ref = oracle.spmv_T(rp, cols, dec, v, spec.n_cols)
    scale = oracle.spmv_T(rp, cols, np.abs(dec), np.abs(v), spec.n_cols)
    assert oracle.max_scaled_err(g, g_ref, scale) <= TOL
    A.close()


def test_adjoint_long_rows_and_empty_columns(dev):
    """A^T rows of about 3,000 entries: split groups shared by four waves
    (group sizes 1024 and 8192) or rows summed by one wave (65536).  Both
    must meet the bound and give the same bits; empty columns give +0."""
    rng = np.random.default_rng(5)
    n_rows, n_cols = 30000, 150
    lens = rng.integers(0, 60, size=n_rows)
    lens[rng.random(n_rows) < 0.6] = 0
    rp = np.zeros(n_rows + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    cols = np.empty(rp[-1], np.int32)
    for i in range(n_rows):
        if lens[i]:
            # columns 120.. stay empty
            cols[rp[i]:rp[i + 1]] = np.sort(rng.choice(120, size=lens[i], replace=False))
    vals = np.exp(rng.normal(-3, 1, size=rp[-1])).astype(np.float32)
    v = rng.uniform(-1, 1, n_rows).astype(np.float32)
    A = dm.DoseMatrix(rp, cols, vals, n_cols, "fp16", transpose=True)
    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    g_ref = oracle.spmv_T(rp, cols, dec, v, n_cols)
    scale = oracle.spmv_T(rp, cols, np.abs(dec), np.abs(v), n_cols)
    col_len = np.bincount(cols, minlength=n_cols)
    gs = []
    for group_nnz_t in (1024, 8192, 65536):
        _say("adjoint long rows", group_nnz_t)
        A.set_partition(8192, group_nnz_t)
        n_split = A.info()["n_groups_split_t"]
        assert n_split == int(np.sum(col_len > max(group_nnz_t // 4, 2048)))
        g = A.adjoint(torch.from_numpy(v).cuda()).cpu().numpy()
        assert oracle.max_scaled_err(g, g_ref, scale) <= TOL
        assert np.all(_bits(g[120:]) == 0)
        # deterministic
        g2 = A.adjoint(torch.from_numpy(v).cuda()).cpu().numpy()
        np.testing.assert_array_equal(_bits(g), _bits(g2))
        gs.append(g)
    assert A.info()["n_groups_split_t"] == 0
    for g in gs[1:]:
        np.testing.assert_array_equal(_bits(g), _bits(gs[0]))
    A.close()


def test_adjointness(dev):
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "bf16", transpose=True)
    x = torch.from_numpy(dosegen.spot_weights(spec.seed, 0, spec.n_cols)).cuda()
    v = torch.from_numpy(dosegen.signed_values(spec.seed, 4, spec.n_rows)).cuda()
    lhs = torch.dot(v.double(), A.spmv(x).double()).item()
    rhs = torch.dot(A.adjoint(v).double(), x.double()).item()
    dec, _ = oracle.decode_matrix("bf16", rp, vals)
    bound = np.dot(np.abs(v.cpu().numpy()), oracle.spmv(rp, cols, np.abs(dec), x.cpu().numpy()))
    assert abs(lhs - rhs) <= 2e-6 * bound
    A.close()


def _objective_case():
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    p, w = dosegen.objective_masks(spec.nx, spec.ny, spec.nz)
    x = dosegen.spot_weights(spec.seed, 0, spec.n_cols) * np.float32(8.0)
    return spec, rp, cols, vals, p, w, x


def test_objective_seed_and_norm_parity(dev):
    spec, rp, cols, vals, p, w, x = _objective_case()
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16", transpose=True)
    d = A.spmv(torch.from_numpy(x).cuda())
    pd, wd = torch.from_numpy(p).cuda(), torch.from_numpy(w).cuda()
    seed = torch.empty_like(d)
    f = dm.objective(d, pd, wd, seed=seed).item()
    d_h = d.cpu().numpy().astype(np.float64)
    f_ref = oracle.objective(d_h, p, w)  # same FP32 dose, FP64 reduction
    assert abs(f - f_ref) <= 1e-13 * abs(f_ref)
    s_ref = oracle.objective_seed(d_h, p, w).astype(np.float32)
    np.testing.assert_array_equal(_bits(seed.cpu().numpy()), _bits(s_ref))
    g = A.adjoint(seed)
    n = dm.norm2(g).item()
    n_ref = oracle.norm2(g.cpu().numpy().astype(np.float64))
    assert abs(n - n_ref) <= 1e-14 * n_ref
    # fixed-order reductions are bitwise repeatable
    assert dm.objective(d, pd, wd).item() == f and dm.norm2(g).item() == n
    # empty input
    z = torch.empty(0, device=dev)
    assert dm.objective(z, z, z).item() == 0.0 and dm.norm2(z).item() == 0.0
    A.close()


def test_objective_gradient_autograd_vs_oracle_and_finite_differences(dev):
    """f(x) = sum w (A x - p)^2 through DoseSpMV and DoseObjective; the
    gradient must match the oracle's A^T (2 w (A x - p)) and central finite
    differences of the oracle objective over 64 seeded spots."""
    spec, rp, cols, vals, p, w, x = _objective_case()
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16", transpose=True)
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    f = dm.DoseObjective.apply(dm.dose(xt, A), torch.from_numpy(p).cuda(), torch.from_numpy(w).cuda())
    f.backward()
    g = xt.grad.cpu().numpy().astype(np.float64)

    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    d_ref = oracle.spmv(rp, cols, dec, x)
    f_ref = oracle.objective(d_ref, p, w)
    seed_ref = oracle.objective_seed(d_ref, p, w)
    # oracle gradient in FP64: A^T seed, with the seed kept in FP64
    dense = np.zeros((spec.n_rows, spec.n_cols))
    dense[np.repeat(np.arange(spec.n_rows), np.diff(rp)), cols] = dec
    g_ref = dense.T @ seed_ref
    g_scale = np.abs(dense).T @ np.abs(seed_ref)
    # dose error <= 1e-5 relative enters the seed through 2w(d - p)
    d_abs = oracle.spmv(rp, cols, np.abs(dec), x)
    seed_err = 2 * w * (TOL * d_abs)
    bound = TOL * g_scale + np.abs(dense).T @ seed_err
    assert np.all(np.abs(g - g_ref) <= bound + 1e-30)
    assert abs(f.item() - f_ref) <= 2 * TOL * np.sum(w * 2 * np.abs(d_ref - p) * d_abs) + 1e-9

    rng = np.random.default_rng(64)
    spots = rng.choice(spec.n_cols, size=64, replace=False)
    h = np.float32(0.5)
    for j in spots:
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (oracle.objective(oracle.spmv(rp, cols, dec, xp), p, w)
              - oracle.objective(oracle.spmv(rp, cols, dec, xm), p, w)) / (float(xp[j]) - float(xm[j]))
        # f is quadratic: the central difference equals the FP64 gradient up to
        # the FP64 rounding of f; the GPU gradient carries the bound above
        assert abs(fd - g_ref[j]) <= 1e-9 * f_ref
        assert abs(fd - g[j]) <= bound[j] + 1e-9 * f_ref
    A.close()
