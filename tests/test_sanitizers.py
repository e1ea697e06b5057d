"""The native host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): libdose's host side (validation, the row-group partition, the
SELL-C-sigma layout, argument checks of every entry point that fails before
touching a GPU), the oracle and the input generator, built with the
sanitizers (tests/sanitize_build.py) and driven by the host and oracle test
modules in a child process that preloads the sanitizer runtime.  Any
sanitizer report fails the child (halt on the first error)."""
import os
import subprocess
import sys

import pytest

import sanitize_build

ROOT = sanitize_build.ROOT
MODULES = ["tests/test_host_abi.py", "tests/test_host_sell.py", "tests/test_oracle_pins.py",
           "tests/test_oracle_sell_runs.py", "tests/test_oracle_metrics.py"]


@pytest.mark.timeout(900)
def test_host_code_under_sanitizers():
    dose = sanitize_build.libdose()
    orc = sanitize_build.oracle_lib()
    gen = sanitize_build.dosegen_lib()
    driver = "\n".join([
        "import sys",
        f"sys.path.insert(0, {ROOT!r})",
        f"sys.path.insert(0, {os.path.join(ROOT, 'tests')!r})",
        "import paper_2103_09683_amd._lib as L",
        f"L.LIB_PATH = {dose!r}",
        "import oracle, dosegen",
        f"oracle._LIB_PATH = {orc!r}",
        f"dosegen._LIB_PATH = {gen!r}",
        "import pytest",
        f"rc = pytest.main(['-q', '-x', '-m', 'not gpu', '-p', 'no:cacheprovider', *{MODULES!r}])",
        "assert L.load()._name == L.LIB_PATH and oracle._lib._name == oracle._LIB_PATH",
        "assert dosegen._lib._name == dosegen._LIB_PATH",
        "sys.exit(int(rc))",
    ])
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": sanitize_build.runtime(),
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "LD_LIBRARY_PATH": "/opt/rocm/llvm/lib:" + env.get("LD_LIBRARY_PATH", ""),
        "OMP_NUM_THREADS": "4",
    })
    r = subprocess.run([sys.executable, "-c", driver], env=env, cwd=ROOT, capture_output=True, text=True,
                       timeout=850)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert " passed" in r.stdout
