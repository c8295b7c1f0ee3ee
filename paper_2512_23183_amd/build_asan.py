"""Build a CPU-checking variant of ``libsv.so``: the same sources with the
host code compiled under AddressSanitizer and UndefinedBehaviorSanitizer
(device code unchanged, never run by it), linked to ``_build_asan/``.

It serves the host-only entry points (validation, lowering, planning, the
device-plan build behind ``sv_plan_info`` / ``sv_plan_dump``, the
parameter-shift expansion behind ``sv_psr_info``) run on the CPU by
``tests/test_host_sanitized.py``, in a child process that preloads the
sanitizer runtime.  Not used by anything that runs on a GPU.
"""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, HERE)
import build as _b  # noqa: E402  (the regular build's flags and sources)

OUT = os.path.join(ROOT, "_build_asan")
LIB = os.path.join(OUT, "libsv_asan.so")
# host side only: each sanitizer flag applies to the host compilation
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def runtime() -> str:
    """The toolchain's AddressSanitizer runtime (preloaded by the test)."""
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("AddressSanitizer runtime not found under /opt/rocm/llvm")
    return hits[-1]


def _compile(src: str) -> str:
    obj = os.path.join(OUT, src + ".o")
    cmd = [_b.HIPCC] + [f for f in _b.COMMON if f != "-O3"] + ["-O1", "-g"] + _b.DEVICE + SAN + ["-x", "hip"]
    cmd += ["-c", os.path.join(_b.CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    return obj


def stale() -> bool:
    """True when the library is missing or older than a source or header."""
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = glob.glob(os.path.join(_b.CSRC, "*")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    return any(os.path.getmtime(f) > t for f in deps)


def build() -> str:
    os.makedirs(OUT, exist_ok=True)
    srcs = _b.sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    cmd = [_b.HIPCC, f"--offload-arch={_b.ARCH}", "-shared", "-fPIC", "-shared-libsan",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-o", LIB + ".tmp"] + objs + ["-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build())
