"""Parity at the workloads' full sizes, in the launch configurations the
benchmark times, on seeded row samples the oracle computes one by one.

* Half/double (Sec. II-D: FP16 values, FP64 spot weights, FP64 sums and
  dose) on the clinical beam (2,097,152 x 25,000) and on the largest
  workload (8,388,608 x 60,000): spot weights hi + lo (both exact in FP32,
  lo below hi's last bit), reference oracle(hi) + oracle(lo) on a 1% sample
  stratified to hold the longest rows and empty rows; bound 1e-12 of
  sum |a| |x| per row (the kernel's FP64 error is below 50 * 2^-53).
* The robust batch at full size: 36 matrices of 0.5M-2.1M rows (7.5e9
  stored entries), 4 spot-weight vectors each, one autotuned graph plan, in
  FP16 and BF16: every matrix's product on a 1% row sample against the
  oracle (1e-5 relative), and every output bit for bit equal to the plain
  product of each vector.
* The paper-irregular row lengths (sigma 1.0, rows of up to 16,000 entries)
  at the clinical beam's width (25,000 columns): sampled rows, the longest
  ones among them, against the oracle.
"""
import time

import numpy as np
import pytest
import torch

import dosegen
import oracle
import paper_2103_09683_amd as dm

pytestmark = pytest.mark.gpu

TOL = 1e-5
TOL64 = 1e-12


def _say(*a):
    print(*a, flush=True)


def _sub_csr(rp, cols, vals, rows):
    lens = rp[rows + 1] - rp[rows]
    srp = np.zeros(rows.size + 1, np.int64)
    np.cumsum(lens, out=srp[1:])
    idx = np.repeat(rp[rows] - srp[:-1], lens) + np.arange(srp[-1], dtype=np.int64)
    return srp, cols[idx], vals[idx]


def _sample_rows(rp, seed, frac=0.01, n_long=200, n_empty=200):
    lens = np.diff(rp)
    rng = np.random.default_rng(seed)
    empty = np.nonzero(lens == 0)[0]
    parts = [np.argsort(lens, kind="stable")[-n_long:], rng.integers(0, lens.size, max(1, int(lens.size * frac)))]
    if empty.size:
        parts.append(empty[rng.integers(0, empty.size, n_empty)])
    return np.unique(np.concatenate(parts))


def _with_low_bits(hi32, rng):
    hi = np.asarray(hi32, np.float32)
    e = np.frexp(hi.astype(np.float64))[1]
    u = (rng.choice([-1.0, 1.0], hi.size) * rng.uniform(0.5, 1.0, hi.size)).astype(np.float32)
    lo = np.ldexp(u.astype(np.float64), e - 26).astype(np.float32)
    x = hi.astype(np.float64) + lo.astype(np.float64)
    assert np.array_equal(x - hi.astype(np.float64), lo.astype(np.float64))
    return x, hi, lo


@pytest.mark.timeout(600)
@pytest.mark.parametrize("which", ["clinical_beam", "sweep_large"])
def test_half_double_full_size_sampled(which, dev):
    spec = getattr(dosegen, which)()
    t0 = time.time()
    rp, cols, vals = dosegen.csr(spec)
    _say(f"half/double {spec.name}: {rp[-1]} entries generated in {time.time() - t0:.1f}s")
    rows = _sample_rows(rp, 2103)
    srp, scols, svals = _sub_csr(rp, cols, vals, rows)
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16")
    del cols, vals
    rng = np.random.default_rng(65)
    x, hi, lo = _with_low_bits(dosegen.spot_weights(spec.seed, 0, spec.n_cols), rng)
    y = A.spmv(torch.from_numpy(x).cuda())
    assert y.dtype == torch.float64
    y = y.cpu().numpy()
    _say("forward done")
    dec, _ = oracle.decode_matrix("fp16", srp, svals)
    y_ref = oracle.spmv(srp, scols, dec, hi) + oracle.spmv(srp, scols, dec, lo)
    scale = oracle.spmv(srp, scols, np.abs(dec), np.abs(hi)) + oracle.spmv(srp, scols, np.abs(dec), np.abs(lo))
    err = oracle.max_scaled_err(y[rows], y_ref, scale)
    _say(f"{spec.name} half/double: max scaled error {err:.3e} on {rows.size} rows")
    assert err <= TOL64
    lens = np.diff(rp)
    assert np.all(y[lens == 0].view(np.uint64) == 0)
    A.close()


def _robust_batch_format(fmt, dev):
    specs = dosegen.robust_batch(1.0)
    mats, entries, checks = [], [], []
    nnz = 0
    t0 = time.time()
    for s in specs:
        rp, cols, vals = dosegen.csr(s)
        nnz += int(rp[-1])
        rows = _sample_rows(rp, 3000 + s.matrix_id, n_long=20, n_empty=20)
        checks.append((rows, _sub_csr(rp, cols, vals, rows)))
        A = dm.DoseMatrix(rp, cols, vals, s.n_cols, fmt)
        del rp, cols, vals
        X = torch.from_numpy(np.stack([dosegen.spot_weights(s.seed, 4 * s.matrix_id + r, s.n_cols)
                                       for r in range(4)], 1)).cuda()
        mats.append(A)
        entries.append((A, X, torch.full((s.n_rows, 4), np.nan, device=dev)))
    _say(f"robust batch {fmt}: 36 matrices, {nnz} entries, created in {time.time() - t0:.1f}s")
    return specs, mats, entries, checks, nnz


@pytest.mark.timeout(900)
@pytest.mark.parametrize("fmt", ["fp16", "bf16"])
def test_robust_batch_full_size(fmt, dev):
    specs, mats, entries, checks, nnz = _robust_batch_format(fmt, dev)
    assert nnz > 7e9
    plan = dm.BatchPlan(entries, autotune=True)
    plan.launch()
    torch.cuda.synchronize()
    _say("plan launched")
    worst = 0.0
    for s, (A, X, Y), (rows, (srp, scols, svals)) in zip(specs, entries, checks):
        for r in range(4):
            y_plain = A.spmv(X[:, r].contiguous())
            assert torch.equal(Y[:, r].contiguous().view(torch.int32), y_plain.view(torch.int32)), (s.name, r)
        dec, _ = oracle.decode_matrix(fmt, srp, svals)
        Y_ref = oracle.spmv_multi(srp, scols, dec, X.cpu().numpy())
        Y_s = Y.cpu().numpy()[rows]
        for r in range(4):
            err = oracle.max_rel_err(Y_s[:, r], Y_ref[:, r])
            worst = max(worst, err)
            assert err <= TOL, (s.name, r, err)
    _say(f"robust batch {fmt}: max relative error {worst:.3e} over 36 x 4 sampled products")
    plan.close()
    for A in mats:
        A.close()
    del entries
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
def test_paper_irregular_at_clinical_width(dev):
    spec = dosegen.paper_irregular(dosegen.clinical_beam())
    rp, cols, vals = dosegen.csr(spec)
    lens = np.diff(rp)
    assert spec.n_cols == 25000 and lens.max() == 16000
    rows = _sample_rows(rp, 2104)
    assert lens[rows].max() == 16000
    srp, scols, svals = _sub_csr(rp, cols, vals, rows)
    x_h = dosegen.spot_weights(spec.seed, 0, spec.n_cols)
    for idx in ("i32", "u16"):
        A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16", index_format=idx)
        assert A.info()["n_groups_split"] > 0
        y = A.spmv(torch.from_numpy(x_h).cuda()).cpu().numpy()
        dec, _ = oracle.decode_matrix("fp16", srp, svals)
        err = oracle.max_rel_err(y[rows], oracle.spmv(srp, scols, dec, x_h))
        _say(f"{spec.name} ({idx}): max rel err {err:.3e} on {rows.size} rows, longest {lens[rows].max()}")
        assert err <= TOL
        assert np.all(y[lens == 0].view(np.uint32) == 0)
        A.close()
