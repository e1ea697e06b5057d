"""16-bit column indices: the same products as with 32-bit indices.

The kernels only widen the indices they load, so every result must equal the
32-bit path bit for bit (forward, adjoint through the transpose built from
the 16-bit indices, batched), besides meeting the oracle's bound.
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
def test_u16_equals_i32_forward_adjoint_decode(fmt, dev):
    spec = dosegen.robust_batch(0.03)[2]
    rp, cols, vals = dosegen.csr(spec)
    _say("u16", fmt, spec.name, rp[-1])
    A32 = dm.DoseMatrix(rp, cols, vals, spec.n_cols, fmt, transpose=True)
    A16 = dm.DoseMatrix(rp, cols, vals, spec.n_cols, fmt, transpose=True, index_format="u16")
    assert A16.info()["index_format"] == 2
    assert A16.info()["spmv_bytes"] == A32.info()["spmv_bytes"] - 2 * int(rp[-1])
    assert A16.info()["adjoint_bytes"] == A32.info()["adjoint_bytes"]
    # decode: the same columns
    r_rp, r_cols, r_vals = A16.decode(0, 3000)
    np.testing.assert_array_equal(r_cols, cols[:rp[3000]])
    x = torch.from_numpy(dosegen.spot_weights(spec.seed, 0, spec.n_cols)).cuda()
    y16 = A16.spmv(x).cpu().numpy()
    y32 = A32.spmv(x).cpu().numpy()
    np.testing.assert_array_equal(_bits(y16), _bits(y32))
    dec, _ = oracle.decode_matrix(fmt, rp, vals)
    y_ref = oracle.spmv(rp, cols, dec, x.cpu().numpy())
    assert oracle.max_rel_err(y16, y_ref) <= TOL
    v = torch.from_numpy(dosegen.signed_values(spec.seed, 5, spec.n_rows)).cuda()
    np.testing.assert_array_equal(_bits(A16.adjoint(v).cpu().numpy()), _bits(A32.adjoint(v).cpu().numpy()))
    A16.close()
    A32.close()


def test_u16_batched_equals_plain(dev):
    specs = dosegen.robust_batch(0.03)[:4]
    entries, mats = [], []
    for s in specs:
        rp, cols, vals = dosegen.csr(s)
        A = dm.DoseMatrix(rp, cols, vals, s.n_cols, "bf16", index_format="u16")
        X = np.stack([dosegen.spot_weights(s.seed, 10 * s.matrix_id + r, s.n_cols) for r in range(4)], 1)
        Y = torch.full((s.n_rows, 4), np.nan, device=dev)
        mats.append((A, X))
        entries.append((A, torch.from_numpy(np.ascontiguousarray(X)).cuda(), Y))
    _say("u16 batched")
    dm.spmv_batched(entries)
    torch.cuda.synchronize()
    for (A, X), (_, _, Y) in zip(mats, entries):
        for r in range(4):
            y = A.spmv(torch.from_numpy(np.ascontiguousarray(X[:, r])).cuda()).cpu().numpy()
            np.testing.assert_array_equal(_bits(Y[:, r].cpu().numpy()), _bits(y))
        A.close()


def test_u16_rejects_wide_matrices_and_mixed_batches(dev):
    rp = np.array([0, 2], np.int64)
    cols = np.array([5, 70000], np.int32)
    vals = np.ones(2, np.float32)
    with pytest.raises(dm.DoseError):
        dm.DoseMatrix(rp, cols, vals, 70001, "fp16", index_format="u16")
    A = dm.DoseMatrix(rp, cols[:1].repeat(2) + np.array([0, 1], np.int32), vals, 65536, "fp16", index_format="u16")
    B = dm.DoseMatrix(rp, cols[:1].repeat(2) + np.array([0, 1], np.int32), vals, 65536, "fp16")
    x = torch.ones(65536, device=dev)
    y1 = torch.empty(1, device=dev)
    y2 = torch.empty(1, device=dev)
    with pytest.raises(dm.DoseError):
        dm.spmv_batched([(A, x, y1), (B, x, y2)])
    A.close()
    B.close()


def test_misaligned_vectors_rejected(dev):
    """x, y, v, g must be 4-byte aligned: the C ABI rejects others before any
    launch."""
    from paper_2103_09683_amd import _lib
    rp = np.array([0, 2, 3], np.int64)
    cols = np.array([0, 3, 1], np.int32)
    vals = np.ones(3, np.float32)
    A = dm.DoseMatrix(rp, cols, vals, 4, "fp16", transpose=True)
    buf = torch.zeros(64, device=dev)
    lib = _lib.load()
    base = buf.data_ptr()
    assert lib.dose_spmv(A.handle, base + 2, base + 128, None) == _lib.ERR_INVALID_ARGUMENT
    assert lib.dose_spmv(A.handle, base, base + 130, None) == _lib.ERR_INVALID_ARGUMENT
    assert lib.dose_spmv_adjoint(A.handle, base + 1, base + 128, None) == _lib.ERR_INVALID_ARGUMENT
    assert lib.dose_spmv(A.handle, base, base + 128, None) == _lib.OK
    torch.cuda.synchronize()
    A.close()


@pytest.mark.parametrize("fmt", ["fp16", "fp8e4m3_rowscale"])
def test_u16_columns_up_to_65535(fmt, dev):
    """16-bit indices at their limit: n_cols = 65536, columns up to 65535 in
    both halves of the packed index words; equal to the 32-bit path."""
    rng = np.random.default_rng(16)
    n_rows, n_cols = 700, 65536
    lens = rng.integers(0, 300, n_rows)
    lens[::7] = 0
    rp = np.zeros(n_rows + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    cols = np.concatenate([np.sort(rng.choice(np.arange(65000, 65536), l, replace=False)) if i % 2
                           else np.sort(rng.choice(n_cols, l, replace=False)) for i, l in enumerate(lens)]).astype(np.int32)
    vals = rng.lognormal(-3, 1, rp[-1]).astype(np.float32)
    assert cols.max() >= 65500
    A32 = dm.DoseMatrix(rp, cols, vals, n_cols, fmt, transpose=True)
    A16 = dm.DoseMatrix(rp, cols, vals, n_cols, fmt, transpose=True, index_format="u16")
    np.testing.assert_array_equal(A16.decode()[1], cols)
    x = torch.from_numpy(rng.random(n_cols).astype(np.float32)).cuda()
    v = torch.from_numpy(rng.standard_normal(n_rows).astype(np.float32)).cuda()
    np.testing.assert_array_equal(_bits(A16.spmv(x).cpu().numpy()), _bits(A32.spmv(x).cpu().numpy()))
    np.testing.assert_array_equal(_bits(A16.adjoint(v).cpu().numpy()), _bits(A32.adjoint(v).cpu().numpy()))
    dec, _ = oracle.decode_matrix(fmt, rp, vals)
    assert oracle.max_rel_err(A16.spmv(x).cpu().numpy(), oracle.spmv(rp, cols, dec, x.cpu().numpy())) <= TOL
    A16.close()
    A32.close()
