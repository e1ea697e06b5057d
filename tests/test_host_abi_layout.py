"""The binding's ctypes structures and constants against the C header: small
C programs, compiled with gcc against include/dose.h, print every
structure's size and each field's offset, and every enumerator the binding
mirrors; the ctypes declarations and constants must agree one by one, so a
reordered, resized or missing field, or a flag renumbered on one side, is
caught without a GPU."""
import ctypes
import os
import subprocess

import pytest

from paper_2103_09683_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# C name of each ctypes structure (the ctypes field names are the C ones)
STRUCTS = {
    "dose_csr_host": _lib.CsrHost,
    "dose_matrix_info_t": _lib.MatrixInfo,
    "dose_batch_item": _lib.BatchItem,
    "dose_sell_info_t": _lib.SellInfo,
    "dose_sell_batch_item": _lib.SellBatchItem,
    "dose_adjoint_item": _lib.AdjointItem,
}


def _c_source():
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "dose.h"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    return "\n".join(lines) + "\n"


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    d = tmp_path_factory.mktemp("abi")
    src, exe = d / "layout.c", d / "layout"
    src.write_text(_c_source())
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe)], check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    layout = {}
    for line in out.splitlines():
        name, field, value = line.split()
        layout[(name, field)] = int(value)
    return layout


@pytest.mark.parametrize("cname", list(STRUCTS))
def test_struct_layout_matches_header(cname, c_layout):
    cls = STRUCTS[cname]
    assert ctypes.sizeof(cls) == c_layout[(cname, "sizeof")], cname
    for field, _ in cls._fields_:
        assert getattr(cls, field).offset == c_layout[(cname, field)], (cname, field)


def test_header_compiles_as_c_and_cxx(tmp_path):
    # the header is plain C (the boundary takes no C++ or HIP types) and
    # also compiles as C++
    src = tmp_path / "h.c"
    src.write_text('#include "dose.h"\nint main(void) { return DOSE_OK; }\n')
    for compiler, std in (("gcc", "-std=c11"), ("g++", "-std=c++17")):
        subprocess.run([compiler, std, "-Wall", "-Werror", "-x", "c" if compiler == "gcc" else "c++",
                        "-I", os.path.join(ROOT, "include"), str(src), "-o", str(tmp_path / "h")],
                       check=True, capture_output=True, text=True)


# every constant of the binding against the header's enumerator of that name
# (the binding drops the DOSE_ prefix)
CONSTANTS = ["OK", "ERR_INVALID_ARGUMENT", "ERR_BAD_CSR", "ERR_UNSUPPORTED", "ERR_NO_TRANSPOSE",
             "ERR_OUT_OF_MEMORY", "ERR_HIP", "ERR_INTERNAL", "VAL_FP16", "VAL_BF16", "VAL_FP8E4M3_ROWSCALE",
             "VAL_FP32", "IDX_I32", "IDX_U16", "IDX_RUNS", "CREATE_TRANSPOSE", "CREATE_AUTOTUNE",
             "CREATE_TRANSPOSE_SLABS", "ADJOINT_ACCUMULATE", "PART_A", "PART_AT", "PLAN_AUTOTUNE",
             "ROBUST_EXPECTED", "ROBUST_WORST"]


def test_constants_match_header(tmp_path):
    lines = ['#include <stdio.h>', '#include "dose.h"', "int main(void) {"]
    lines += [f'  printf("{c} %lld\\n", (long long)DOSE_{c});' for c in CONSTANTS]
    lines += ["  return 0;", "}"]
    src, exe = tmp_path / "consts.c", tmp_path / "consts"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe)], check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    header = {name: int(value) for name, value in (line.split() for line in out.splitlines())}
    for c in CONSTANTS:
        assert getattr(_lib, c) == header[c], (c, getattr(_lib, c), header[c])
    # create flags and plan flags are single bits, distinct within each family
    create = [header[c] for c in ("CREATE_TRANSPOSE", "CREATE_AUTOTUNE", "CREATE_TRANSPOSE_SLABS")]
    plan = [header[c] for c in ("PLAN_AUTOTUNE", "ADJOINT_ACCUMULATE")]
    for family in (create, plan):
        assert all(f > 0 and f & (f - 1) == 0 for f in family) and len(set(family)) == len(family)
