"""The binding's ctypes structures against the C header: a small C program,
compiled with gcc against include/dose.h, prints every structure's size and
each field's offset; the ctypes declarations must agree field by field, so a
reordered, resized or missing field in either is caught without a GPU."""
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
