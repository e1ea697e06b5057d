"""Host-only tests of the SELL-C-sigma layout the library builds (C = 64):
the sigma-sorted row order and the chunk widths must equal the oracle's
(Kreutzer et al.'s definition, pinned in test_oracle_sell_runs.py) exactly.
No GPU is touched."""
import numpy as np
import pytest

import oracle
import paper_2103_09683_amd as dm
from paper_2103_09683_amd import _lib


def _rp(lengths):
    rp = np.zeros(len(lengths) + 1, np.int64)
    np.cumsum(lengths, out=rp[1:])
    return rp


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 255, 256, 1000, 4097])
@pytest.mark.parametrize("sigma", [1, 7, 64, 100, 256, 1000, 1 << 20])
def test_layout_equals_oracle(n, sigma):
    rng = np.random.default_rng(n * 31 + sigma)
    lens = rng.integers(0, 20, n)  # many ties
    lens[rng.random(n) < 0.5] = 0   # empty rows, as outside a beam
    rp = _rp(lens)
    perm, width = dm.sell_layout(rp, sigma)
    perm_o, width_o = oracle.sell_layout(rp, 64, sigma)
    assert np.array_equal(perm, perm_o)
    assert np.array_equal(width, width_o)


def test_layout_of_dose_rows():
    import dosegen
    spec = dosegen.small_plain()
    rp, _, _ = dosegen.csr(spec)
    for sigma in (64, 256, 2048):
        perm, width = dm.sell_layout(rp, sigma)
        perm_o, width_o = oracle.sell_layout(rp, 64, sigma)
        assert np.array_equal(perm, perm_o) and np.array_equal(width, width_o)


def test_layout_rejects_bad_arguments():
    rp = _rp([1, 2, 3])
    perm = np.empty(3, np.int64)
    width = np.empty(1, np.int64)
    lib = _lib.load()
    assert lib.dose_sell_layout(rp.ctypes.data, 3, 0, perm.ctypes.data, width.ctypes.data) == _lib.ERR_INVALID_ARGUMENT
    assert lib.dose_sell_layout(rp.ctypes.data, 3, -5, perm.ctypes.data, width.ctypes.data) == _lib.ERR_INVALID_ARGUMENT
    bad = np.array([0, 3, 2, 4], np.int64)
    assert lib.dose_sell_layout(bad.ctypes.data, 3, 4, perm.ctypes.data, width.ctypes.data) == _lib.ERR_BAD_CSR
    assert lib.dose_sell_layout(rp.ctypes.data, 3, 4, None, width.ctypes.data) == _lib.ERR_INVALID_ARGUMENT
