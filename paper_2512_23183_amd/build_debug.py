"""Build the debug kernel variant of ``libsv.so``: the same sources
compiled with SV_DEBUG_BOUNDS, under which the tile, permutation, sweep and
expectation kernels check every HBM and LDS index they form against its
array.  An index outside its array is replaced by 0 (the access stays in
bounds, nothing traps) and sets a flag; the API call that launched the
kernel synchronises and returns SV_EDEVICE.  Objects go to
``_build_debug/``, the library to ``paper_2512_23183_amd/libsv_debug.so``;
tests/test_gpu_debug_bounds.py runs workloads through it (SV_LIBRARY).
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, HERE)
import build as _b  # noqa: E402  (the regular build's flags and sources)

OUT = os.path.join(ROOT, "_build_debug")
LIB = os.path.join(HERE, "libsv_debug.so")


def _compile(src: str) -> str:
    obj = os.path.join(OUT, src + ".o")
    cmd = [_b.HIPCC, "-DSV_DEBUG_BOUNDS"] + _b.COMMON + _b.DEVICE + ["-x", "hip"]
    cmd += ["-c", os.path.join(_b.CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    return obj


def build() -> str:
    os.makedirs(OUT, exist_ok=True)
    srcs = _b.sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    cmd = [_b.HIPCC, f"--offload-arch={_b.ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs + ["-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build())
