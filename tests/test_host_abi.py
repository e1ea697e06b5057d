"""Host-only tests of libdose: exported symbols, CSR validation, the row-block
partition and the byte model.  None of these touch a GPU."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

import paper_2103_09683_amd as dm
from paper_2103_09683_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "dose.h")).read()
    return sorted(set(re.findall(r"^\s*(?:dose_status|const char\*)\s+(dose_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    names = _header_functions()
    assert len(names) >= 19
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    # the binding declares exactly the header's entry points
    assert sorted(_lib.SIGNATURES) == names


def test_status_strings():
    lib = _lib.load()
    assert lib.dose_status_string(0) == b"ok"
    assert lib.dose_status_string(_lib.ERR_BAD_CSR) == b"malformed CSR matrix"
    assert lib.dose_status_string(-99) == b"unknown status"


# ------------------------------------------------------------------ validation
def _good():
    rp = np.array([0, 2, 2, 5], np.int64)
    c = np.array([0, 3, 1, 2, 4], np.int32)
    v = np.array([0.5, 1.0, 0.25, 2.0, 3.0], np.float32)
    return rp, c, v


def test_validate_accepts_good_and_empty():
    rp, c, v = _good()
    assert dm.csr_validate(rp, c, v, 5) == 0
    assert dm.csr_validate(np.array([0], np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 0) == 0
    assert dm.csr_validate(np.zeros(4, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 7) == 0


@pytest.mark.parametrize("mutate,code", [
    (lambda rp, c, v: rp.__setitem__(0, 1), _lib.ERR_BAD_CSR),              # row_ptr[0] != 0
    (lambda rp, c, v: rp.__setitem__(1, 6), _lib.ERR_BAD_CSR),              # decreasing / out of range
    (lambda rp, c, v: c.__setitem__(1, 5), _lib.ERR_BAD_CSR),               # column out of range
    (lambda rp, c, v: c.__setitem__(1, -1), _lib.ERR_BAD_CSR),              # negative column
    (lambda rp, c, v: c.__setitem__(3, 1), _lib.ERR_BAD_CSR),               # duplicate column
    (lambda rp, c, v: c.__setitem__(2, 3), _lib.ERR_BAD_CSR),               # not ascending
    (lambda rp, c, v: v.__setitem__(0, np.nan), _lib.ERR_BAD_CSR),
    (lambda rp, c, v: v.__setitem__(4, -np.inf), _lib.ERR_BAD_CSR),
    (lambda rp, c, v: v.__setitem__(4, 65520.0), _lib.ERR_UNSUPPORTED),     # rounds to inf in FP16
])
def test_validate_rejects(mutate, code):
    rp, c, v = _good()
    mutate(rp, c, v)
    assert dm.csr_validate(rp, c, v, 5) == code


def test_validate_format_ranges():
    rp, c, v = _good()
    v[4] = 65519.0  # rounds to 65504: representable
    assert dm.csr_validate(rp, c, v, 5, "fp16") == 0
    v[4] = 3.0e38
    assert dm.csr_validate(rp, c, v, 5, "fp16") == _lib.ERR_UNSUPPORTED
    assert dm.csr_validate(rp, c, v, 5, "bf16") == 0
    v[4] = np.float32(3.4e38)  # rounds past the largest bfloat16
    assert dm.csr_validate(rp, c, v, 5, "bf16") == _lib.ERR_UNSUPPORTED
    assert dm.csr_validate(rp, c, v, 5, "fp8e4m3_rowscale") == 0


def test_validate_rejects_nnz_mismatch_and_unknown_format():
    rp, c, v = _good()
    rp[-1] = 4
    assert dm.csr_validate(rp, c[:4], v[:4], 5) == 0
    lib = _lib.load()
    cs, keep = dm._csr_struct(*_good(), 5)
    cs.nnz = 4
    assert lib.dose_csr_validate(ctypes.byref(cs), 1, 1) == _lib.ERR_BAD_CSR
    cs, keep = dm._csr_struct(*_good(), 5)
    assert lib.dose_csr_validate(ctypes.byref(cs), 9, 1) == _lib.ERR_INVALID_ARGUMENT
    assert lib.dose_csr_validate(ctypes.byref(cs), 1, 7) == _lib.ERR_INVALID_ARGUMENT
    assert lib.dose_csr_validate(None, 1, 1) == _lib.ERR_INVALID_ARGUMENT
    assert b"null" in lib.dose_last_error()


# ------------------------------------------------------------------ partition
def _random_row_ptr(rng, n_rows, long_rows=()):
    lens = rng.integers(0, 300, size=n_rows)
    lens[rng.random(n_rows) < 0.5] = 0
    for i, L in long_rows:
        lens[i] = L
    rp = np.zeros(n_rows + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    return rp


@pytest.mark.parametrize("group_nnz", [1024, 4096, 32768, 1 << 20])
def test_partition_groups_tile_the_rows(group_nnz):
    rng = np.random.default_rng(group_nnz)
    rp = _random_row_ptr(rng, 50000, long_rows=[(7, 30000), (4000, 8193), (4001, 2049), (49999, 100000)])
    G = dm.partition_preview(rp, group_nnz)
    assert G.shape[1] == 6
    assert G[0, 0] == 0 and G[-1, 4] == rp.size - 1
    assert np.all(G[1:, 0] == G[:-1, 4]), "groups must tile the rows in order"
    assert np.all(np.diff(G[:, :5], axis=1) >= 0)
    long_row = max(group_nnz // 4, 2048)
    lens = np.diff(rp)
    for r0, r1, r2, r3, r4, split in G:
        nnz = rp[r4] - rp[r0]
        assert 1 <= r4 - r0 <= 16384
        if split:
            # a split group is one row, longer than a wave's share
            assert r4 == r0 + 1 and r1 == r2 == r3 == r4
            assert lens[r0] > long_row
            continue
        assert np.all(lens[r0:r4] <= long_row), "long rows must form split groups"
        assert nnz <= group_nnz
        # wave shares balance entries + 16 per row, up to one row's cost
        cost = [(rp[b] - rp[a]) + 16 * (b - a) for a, b in ((r0, r1), (r1, r2), (r2, r3), (r3, r4))]
        biggest_row = max((rp[i + 1] - rp[i]) + 16 for i in range(r0, r4))
        assert max(cost) - min(cost) <= 2 * biggest_row + (nnz + 16 * (r4 - r0)) // 4 + 1
    n_split = int(G[:, 5].sum())
    assert n_split == int(np.sum(lens > long_row))


def test_partition_is_deterministic():
    rng = np.random.default_rng(3)
    rp = _random_row_ptr(rng, 20000)
    np.testing.assert_array_equal(dm.partition_preview(rp, 8192), dm.partition_preview(rp, 8192))


def test_partition_empty_inputs():
    assert dm.partition_preview(np.array([0], np.int64), 1024).shape == (0, 6)
    G = dm.partition_preview(np.zeros(40001, np.int64), 1024)
    assert (G[:, 4] - G[:, 0]).tolist() == [16384, 16384, 7232]


def test_partition_rejects_bad_group_size():
    for bad in (3000, 512, 1 << 21):
        with pytest.raises(dm.DoseError):
            dm.partition_preview(np.array([0, 1], np.int64), bad)


# ------------------------------------------------------------------ byte model
def _table1():
    with open(os.path.join(ROOT, "tests", "golden", "paper_table1.json")) as f:
        return json.load(f)


def test_byte_model_reproduces_paper_oi_bound():
    t = _table1()
    liver1 = t["table1"][0]
    b = dm.byte_model(liver1["nnz"], liver1["rows"], liver1["cols"], value_bytes=2, index_bytes=4,
                      row_ptr_bytes=4, x_bytes=8, y_bytes=8)
    assert b == 6 * liver1["nnz"] + 12 * liver1["rows"] + 8 * liver1["cols"]
    assert round(2 * liver1["nnz"] / b, 3) == t["oi_upper_bound_liver1"]


def test_storage_model_reproduces_table1_sizes():
    """Table I's sizes fit FP16 values + int32 columns + int32 row offsets:
    solving size = 6 nnz + 4 rows for nnz gives the printed non-zeros to
    three significant figures on all six matrices, while 6 nnz alone (no row
    offsets) or 8 B/nnz (FP32 values) do not."""
    def sig3(v):
        return float(f"{v:.2e}")

    rows = _table1()["table1"]
    for r in rows:
        assert abs(dm.storage_bytes(r["nnz"], r["rows"]) / 1e9 - r["size_gb"]) <= 6 * 0.005 * 10 ** np.floor(
            np.log10(r["nnz"])) / 1e9 + 1e-9
        nnz_fit = (r["size_gb"] * 1e9 - 4 * r["rows"]) / 6
        assert sig3(nnz_fit) == r["nnz"], r["beam"]
        assert round(r["nnz"] / (r["rows"] * r["cols"]) * 100, 2) == r["ratio_pct"], r["beam"]
    assert any(sig3(r["size_gb"] * 1e9 / 6) != r["nnz"] for r in rows)
    assert all(sig3((r["size_gb"] * 1e9 - 4 * r["rows"]) / 8) != r["nnz"] for r in rows)


def test_u16_index_validation():
    rp = np.array([0, 2], np.int64)
    vals = np.ones(2, np.float32)
    assert dm.csr_validate(rp, np.array([0, 65535], np.int32), vals, 65536, "fp16", "u16") == 0
    assert dm.csr_validate(rp, np.array([0, 65535], np.int32), vals, 65537, "fp16", "u16") == _lib.ERR_UNSUPPORTED
    assert dm.csr_validate(rp, np.array([0, 65536], np.int32), vals, 65537, "fp16", "i32") == 0


def test_row_length_limit_in_partition():
    """A row of 2^28 or more entries is rejected by the partition (positions in
    a group are 32-bit byte offsets); one entry fewer is a split group."""
    ok = np.array([0, (1 << 28) - 1], np.int64)
    p = dm.partition_preview(ok, 16384)
    assert p.shape[0] == 1 and p[0, 5] == 1
    bad = np.array([0, 1 << 28], np.int64)
    with pytest.raises(dm.DoseError):
        dm.partition_preview(bad, 16384)


def test_scenario_objective_rejects_bad_arguments_before_any_device_work():
    """Argument checks of the robust-plan epilogue run on the host first: bad
    counts, sizes, null or misaligned arrays, overlapping outputs and inputs
    return INVALID_ARGUMENT (the pointers below are never dereferenced)."""
    lib = _lib.load()
    f = lib.dose_scenario_objective
    buf = np.zeros(4096, np.float64)  # host memory, only used as distinct addresses
    base = buf.ctypes.data
    part, p, w, out = base, base + 8192, base + 12288, base + 16384
    ok = dict(n_scen=2, n_beams=2, n=64, part=part, p=p, w=w, prob=None, d_out=None, seed=None, out=out)

    def call(**kw):
        a = dict(ok, **kw)
        return f(a["n_scen"], a["n_beams"], a["n"], a["part"], a["p"], a["w"], a["prob"], a["d_out"],
                 a["seed"], a["out"], None)

    bad = [dict(n_scen=0), dict(n_beams=0), dict(n_scen=65537), dict(n_beams=65537), dict(n=-1),
           dict(out=None), dict(part=None), dict(p=None), dict(w=None), dict(part=part + 2),
           dict(out=out + 4), dict(prob=out + 4 + 8 * 64), dict(d_out=part),
           dict(d_out=base + 20480, seed=base + 20480 + 4), dict(seed=p),
           dict(n=2 ** 61)]
    for kw in bad:
        assert call(**kw) == _lib.ERR_INVALID_ARGUMENT, kw
        assert lib.dose_last_error()
