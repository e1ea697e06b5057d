"""FP32 matrix values (the paper's Single control, Sec. V): the stored values
are the FP32 inputs themselves, 4 bytes per entry.  Parity with the oracle as
for the reduced formats, bitwise invariance under any partition, batched
equal to plain, 16-bit indices equal to 32-bit, and FP64 products."""
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
    a = np.ascontiguousarray(a)
    return a.view(np.uint32 if a.dtype == np.float32 else np.uint64)


def _long_rows(seed, n_rows=3000, n_cols=6000):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 40, n_rows)
    lens[rng.random(n_rows) < 0.3] = 0
    lens[[7, 1500, 2999]] = [5900, 2100, 4097]
    rp = np.zeros(n_rows + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    cols = np.concatenate([np.sort(rng.choice(n_cols, l, replace=False)) for l in lens]).astype(np.int32)
    vals = rng.lognormal(-3, 1, rp[-1]).astype(np.float32)
    return rp, cols, vals, n_cols


def test_fp32_values_decode_forward_adjoint(dev):
    spec = dosegen.small_plain()
    rp0, cols0, vals0 = dosegen.csr(spec)
    for name, (rp, cols, vals, n_cols) in [("small_plain", (rp0, cols0, vals0, spec.n_cols)),
                                           ("long_rows", _long_rows(21))]:
        _say("fp32 values", name)
        A = dm.DoseMatrix(rp, cols, vals, n_cols, "fp32", transpose=True)
        r_rp, r_cols, r_vals = A.decode()
        np.testing.assert_array_equal(_bits(r_vals), _bits(vals))
        np.testing.assert_array_equal(r_cols, cols)
        dec, _ = oracle.decode_matrix("fp32", rp, vals)
        x = dosegen.spot_weights(spec.seed, 3, n_cols)
        y = A.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
        assert oracle.max_rel_err(y, oracle.spmv(rp, cols, dec, x)) <= TOL
        v = dosegen.signed_values(spec.seed, 4, rp.size - 1)
        g = A.adjoint(torch.from_numpy(v).cuda()).cpu().numpy()
        scale = oracle.spmv_T(rp, cols, np.abs(dec), np.abs(v), n_cols)
        assert oracle.max_scaled_err(g, oracle.spmv_T(rp, cols, dec, v, n_cols), scale) <= TOL
        # FP64 vectors: FP64 products and sums
        y64 = A.spmv(torch.from_numpy(x.astype(np.float64)).cuda()).cpu().numpy()
        assert oracle.max_rel_err(y64, oracle.spmv(rp, cols, dec, x)) <= 1e-12
        A.close()


def test_fp32_values_partitions_batched_u16(dev):
    rp, cols, vals, n_cols = _long_rows(22)
    A = dm.DoseMatrix(rp, cols, vals, n_cols, "fp32", transpose=True)
    A16 = dm.DoseMatrix(rp, cols, vals, n_cols, "fp32", index_format="u16")
    rng = np.random.default_rng(8)
    x = torch.from_numpy(rng.random(n_cols).astype(np.float32)).cuda()
    v = torch.from_numpy(rng.standard_normal(rp.size - 1).astype(np.float32)).cuda()
    ref_y, ref_g = A.spmv(x).cpu().numpy(), A.adjoint(v).cpu().numpy()
    for g in [1024, 4096, 65536]:
        _say("fp32 partition", g)
        A.set_partition(g, g)
        np.testing.assert_array_equal(_bits(A.spmv(x).cpu().numpy()), _bits(ref_y))
        np.testing.assert_array_equal(_bits(A.adjoint(v).cpu().numpy()), _bits(ref_g))
    A.set_partition(A16.info()["group_nnz"], A.info()["group_nnz_t"])
    np.testing.assert_array_equal(_bits(A16.spmv(x).cpu().numpy()), _bits(A.spmv(x).cpu().numpy()))
    # batched, 4 vectors, against plain products of each vector
    X = torch.from_numpy(rng.random((n_cols, 4)).astype(np.float32)).cuda()
    Y = torch.full((rp.size - 1, 4), float("nan"), device=dev)
    dm.spmv_batched([(A, X, Y)])
    torch.cuda.synchronize()
    for r in range(4):
        np.testing.assert_array_equal(_bits(Y[:, r].cpu().numpy()),
                                      _bits(A.spmv(X[:, r].contiguous()).cpu().numpy()))
    A.close()
    A16.close()
