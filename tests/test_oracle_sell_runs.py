"""Pins of the oracle's SELL-C-sigma layout and run-length column indices.

SELL-C-sigma (Kreutzer et al., SIAM J. Sci. Comput. 2014; named by the paper
as the next storage format to investigate, Sec. II-C and Sec. VII): rows
sorted by descending length inside windows of sigma rows (stable), cut into
chunks of C rows, each chunk as wide as its longest row, stored column-major
and padded.  Pinned by a hand-worked example, by numpy's stable argsort (the
layout reduces to it window by window), by the special cases sigma = 1 and
C = 1, and by the product over the packed arrays, which must equal the CSR
oracle's product bit for bit (every row is summed over the same entries in
the same order; padding is skipped).

Run-length indices: the maximal runs of consecutive columns of every row.
Pinned by a hand-worked example, by a run count computed independently with
numpy (one run plus one per break in a row), by maximality, and by decoding.
"""
import numpy as np

import dosegen
import oracle


def _rp(lengths):
    rp = np.zeros(len(lengths) + 1, np.int64)
    np.cumsum(lengths, out=rp[1:])
    return rp


def test_sell_layout_hand_worked_example():
    # lengths 1, 3, 0, 2 | 2, 5 with sigma = 4, C = 2: the first window sorts
    # to rows 1 (3), 3 (2), 0 (1), 2 (0); the second to 5 (5), 4 (2); chunks
    # [1, 3], [0, 2], [5, 4] have widths 3, 1, 5.
    perm, width = oracle.sell_layout(_rp([1, 3, 0, 2, 2, 5]), 2, 4)
    assert perm.tolist() == [1, 3, 0, 2, 5, 4]
    assert width.tolist() == [3, 1, 5]


def test_sell_layout_ties_keep_row_order():
    perm, width = oracle.sell_layout(_rp([2, 7, 2, 7, 0, 2]), 4, 8)
    assert perm.tolist() == [1, 3, 0, 2, 5, 4]
    assert width.tolist() == [7, 2]


def test_sell_layout_is_windowed_stable_argsort():
    rng = np.random.default_rng(5)
    for n, C, sigma in [(1000, 64, 256), (777, 64, 128), (5000, 32, 1024), (300, 8, 300), (64, 64, 4096), (50, 4, 3), (97, 8, 12)]:
        lens = rng.integers(0, 12, n)  # many ties
        rp = _rp(lens)
        perm, width = oracle.sell_layout(rp, C, sigma)
        ref = np.concatenate([w0 + np.argsort(-lens[w0:w0 + sigma], kind="stable") for w0 in range(0, n, sigma)])
        assert np.array_equal(perm, ref)
        padded = np.zeros(-(-n // C) * C, np.int64)
        padded[:n] = lens[ref]
        assert np.array_equal(width, padded.reshape(-1, C).max(1))


def test_sell_layout_special_cases():
    lens = np.array([3, 0, 5, 1, 1, 4, 0, 2])
    rp = _rp(lens)
    perm, width = oracle.sell_layout(rp, 2, 1)  # sigma = 1: no sorting
    assert perm.tolist() == list(range(8))
    assert width.tolist() == [3, 5, 4, 2]
    perm, width = oracle.sell_layout(rp, 1, 8)  # C = 1: widths are the sorted lengths
    assert width.tolist() == sorted(lens.tolist(), reverse=True)


def _dose_rows(seed=3):
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    x = dosegen.spot_weights(spec.seed, seed, spec.n_cols)
    return spec, rp, cols, dec, x


def test_sell_pack_holds_every_entry_once_and_product_equals_csr_bitwise():
    spec, rp, cols, dec, x = _dose_rows()
    lens = np.diff(rp)
    for C, sigma in [(64, 4096), (64, 64), (16, 1000)]:
        perm, width = oracle.sell_layout(rp, C, sigma)
        sval, scol = oracle.sell_pack(rp, cols, dec, C, perm, width)
        assert sval.size == C * width.sum()
        assert np.count_nonzero(scol >= 0) == rp[-1]
        assert np.all(sval[scol < 0] == 0.0)
        # chunk 0, position 0 holds the first window's longest row, column-major
        r0 = perm[0]
        j = np.arange(lens[r0])
        assert np.array_equal(scol[j * C], cols[rp[r0]:rp[r0 + 1]])
        assert np.array_equal(sval[j * C], dec[rp[r0]:rp[r0 + 1]])
        y = oracle.sell_spmv(spec.n_rows, C, perm, width, sval, scol, x)
        assert np.array_equal(y.view(np.uint64), oracle.spmv(rp, cols, dec, x).view(np.uint64))


def test_runs_hand_worked_example():
    rp = _rp([6, 0, 1, 3])
    cols = np.array([3, 4, 5, 9, 10, 20, 7, 0, 2, 3], np.int32)
    run_ptr, start, length = oracle.runs_encode(rp, cols)
    assert run_ptr.tolist() == [0, 3, 3, 4, 6]
    assert start.tolist() == [3, 9, 20, 7, 0, 2]
    assert length.tolist() == [3, 2, 1, 1, 1, 2]
    assert np.array_equal(oracle.runs_decode(run_ptr, start, length), cols)


def test_runs_count_maximality_and_decode_on_dose_rows():
    for spec in (dosegen.small_plain(), dosegen.paper_irregular(dosegen.small_plain())):
        rp, cols, _ = dosegen.csr(spec)
        run_ptr, start, length = oracle.runs_encode(rp, cols)
        lens = np.diff(rp)
        # independent count: one run per non-empty row plus one per break
        brk = np.diff(cols.astype(np.int64)) != 1
        row_of = np.repeat(np.arange(lens.size), lens)
        same_row = row_of[1:] == row_of[:-1]
        expect = (lens > 0).astype(np.int64)
        np.add.at(expect, row_of[1:][brk & same_row], 1)
        assert np.array_equal(np.diff(run_ptr), expect)
        assert np.all(length >= 1)
        # maximal: within a row no run continues the previous one
        for i in np.nonzero(np.diff(run_ptr) > 1)[0][:2000]:
            a, b = run_ptr[i], run_ptr[i + 1]
            assert np.all(start[a + 1:b] != start[a:b - 1] + length[a:b - 1])
        assert np.array_equal(oracle.runs_decode(run_ptr, start, length), cols)
        # the ray structure: a few runs per non-empty row
        per_row = np.diff(run_ptr)[lens > 0]
        assert per_row.mean() < 8
