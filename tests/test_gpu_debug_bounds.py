"""The debug kernel build (paper_2512_23183_amd/build_debug.py: the same
sources with SV_DEBUG_BOUNDS) on the GPU: its context creation proves that
the index checks report (a one-thread probe forms an out-of-range index,
which the check clamps and flags), then tile passes of every engine,
sweeps, the QFT's permutation pass, expectation passes and gradients run
through it without a flagged index and match the oracle
(tests/debug_bounds_driver.py, in a child process that loads the debug
library).  The CPU test checks that the debug library exports what the
regular one does."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEBUG_LIB = os.path.join(ROOT, "paper_2512_23183_amd", "libsv_debug.so")
REG_LIB = os.path.join(ROOT, "paper_2512_23183_amd", "libsv.so")
DRIVER = os.path.join(ROOT, "tests", "debug_bounds_driver.py")


def _declared():
    text = open(os.path.join(ROOT, "include", "sv.h")).read()
    return sorted(set(re.findall(r"\b(sv_[a-z0-9_]+)\s*\(", text)))


def test_debug_library_exports_the_abi():
    if not os.path.exists(DEBUG_LIB):
        pytest.skip("debug library not built (python paper_2512_23183_amd/build_debug.py)")
    dbg = ctypes.CDLL(DEBUG_LIB)
    reg = ctypes.CDLL(REG_LIB)
    for name in _declared():
        if hasattr(reg, name):
            assert hasattr(dbg, name), name


@pytest.mark.gpu
def test_workloads_under_debug_index_checks():
    assert os.path.exists(DEBUG_LIB), "build it with python paper_2512_23183_amd/build_debug.py"
    env = dict(os.environ, SV_LIBRARY=DEBUG_LIB)
    print("[debug-bounds] child process", flush=True)
    r = subprocess.run([sys.executable, "-u", DRIVER], capture_output=True, text=True, timeout=240, env=env)
    print(r.stdout[-3000:], flush=True)
    assert r.returncode == 0 and "debug-bounds ok" in r.stdout, r.stderr[-3000:]
