"""Builds of the native host code with AddressSanitizer and
UndefinedBehaviorSanitizer, for tests/test_sanitizers.py.

libdose is compiled by hipcc with the sanitizers on its host side only
(-Xarch_host before each -fsanitize=; the device code is built as usual);
the oracle and the input generator are compiled by the same clang, so that
one sanitizer runtime serves the whole process.  Builds are cached in
tests/_build/asan/, keyed by a hash of the sources and flags."""
from __future__ import annotations

import glob
import hashlib
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "tests", "_build", "asan")
CSRC = os.path.join(ROOT, "paper_2103_09683_amd", "csrc")
LIB_SOURCES = ["dose_api.cpp", "spmv_kernels.hip", "setup_kernels.hip", "reduce_kernels.hip", "sell_kernels.hip",
               "slab_kernels.hip"]
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
SAN_C = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined",
         "-shared-libsan"]


def runtime() -> str:
    """The clang AddressSanitizer runtime to preload."""
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not libs:
        raise RuntimeError("clang's AddressSanitizer runtime is not installed")
    return libs[-1]


def _hash(paths, flags) -> str:
    h = hashlib.sha256(" ".join(flags).encode())
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _cached(name, srcs, flags, build_fn) -> str:
    key = _hash(srcs, flags)
    path = os.path.join(OUT, f"{name}-{key}.so")
    if not os.path.exists(path):
        os.makedirs(OUT, exist_ok=True)
        build_fn(path + ".tmp")
        os.replace(path + ".tmp", path)
        # older builds of the same library
        import shutil
        for old in glob.glob(os.path.join(OUT, f"{name}-*")):
            if not old.startswith(path):
                shutil.rmtree(old, ignore_errors=True) if os.path.isdir(old) else os.remove(old)
    return path


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd[:3])} ... failed:\n{r.stderr[-4000:]}")


def libdose() -> str:
    srcs = [os.path.join(CSRC, f) for f in LIB_SOURCES] + glob.glob(os.path.join(CSRC, "*.h")) + \
        [os.path.join(ROOT, "include", "dose.h")]
    flags = ["-O1", "-g", "--offload-arch=gfx950", "-fPIC", "-std=c++17", *SAN_HOST,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

    def build(out):
        objdir = out + ".obj"
        os.makedirs(objdir, exist_ok=True)

        def one(f):
            obj = os.path.join(objdir, os.path.splitext(f)[0] + ".o")
            _run([HIPCC, *flags, "-x", "hip", "-c", os.path.join(CSRC, f), "-o", obj])
            return obj

        with ThreadPoolExecutor(max_workers=min(5, os.cpu_count() or 1)) as ex:
            objs = list(ex.map(one, LIB_SOURCES))
        _run([HIPCC, "-shared", "-fPIC", "-shared-libsan", "--offload-arch=gfx950",
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", *objs, "-o", out])

    return _cached("libdose", srcs, flags, build)


def c_library(name: str, src: str, extra=()) -> str:
    flags = ["-O1", "-g", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11",
             *SAN_C, *extra]
    return _cached(name, [src], flags, lambda out: _run([CLANG, *flags, "-o", out, src, "-lm",
                                                         "-Wl,-rpath,/opt/rocm/llvm/lib"]))


def oracle_lib() -> str:
    return c_library("liboracle", os.path.join(ROOT, "oracle", "dose_oracle.c"))


def dosegen_lib() -> str:
    return c_library("libdosegen", os.path.join(ROOT, "dosegen", "dosegen.c"))
