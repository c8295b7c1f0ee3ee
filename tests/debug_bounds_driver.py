"""Child process of test_gpu_debug_bounds.py: workloads through the debug
kernel library (SV_LIBRARY = libsv_debug.so, built with SV_DEBUG_BOUNDS).
Every API call synchronises and returns SV_EDEVICE if a kernel formed an
index outside its array, so a clean run means every checked index of these
workloads stayed in bounds; each result is also compared with the oracle.
Prints one line per case and "debug-bounds ok" at the end."""
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2512_23183_amd import inputs as I  # noqa: E402
from paper_2512_23183_amd import sv  # noqa: E402

C64, C128 = sv.C64, sv.C128


def close(got, want, dtype, what):
    got = got.astype(np.complex128)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    tol = 1e-12 if dtype == C128 else 2e-5
    assert rel <= tol, (what, dtype, rel)
    print(f"[debug-bounds] {what} dtype={dtype}: rel {rel:.2e}", flush=True)


def run(ctx, circ, psi0, dtype, flags=0, params=None):
    st = ctx.alloc(circ.n, dtype)
    st.set_amplitudes(psi0)
    st.apply(circ, params, flags)
    out = st.get_amplitudes()
    st.free()
    return out


def main():
    assert os.environ.get("SV_LIBRARY", "").endswith("libsv_debug.so")
    ctx = sv.Context(0)  # sv_init runs the debug build's self-probe
    try:
        for dtype in (C64, C128):
            # rotation-layer tile passes (four-bit stages), several tiles
            n = 16
            circ = I.deep_random_circuit(n, 6, 5)
            psi0 = I.gaussian_state(n, 6)
            close(run(ctx, circ, psi0, dtype), oracle.run_circuit(circ, None, psi0), dtype, "deep tile passes")
            # the same gates one launch per gate (sweep kernels)
            close(run(ctx, circ, psi0, dtype, sv.FLAG_UNFUSED), oracle.run_circuit(circ, None, psi0), dtype,
                  "deep sweeps")
            # QFT: Hadamard / ladder stages and the permutation pass
            n = 18
            psi0 = I.gaussian_state(n, 7)
            st = ctx.alloc(n, dtype)
            st.set_amplitudes(psi0)
            st.qft()
            got = st.get_amplitudes()
            st.free()
            close(got, math.sqrt(1 << n) * np.fft.ifft(psi0), dtype, "qft")
            # ansatz gradient: three-bit engine with layout maps, expectation
            # tiles, wide X/Y supports straight from HBM
            n = 14
            c = I.hea_circuit(n, 2)
            params = I.uniform_params(c.n_params, 8)
            terms = [(0.7, "X" + "I" * (n - 2) + "Y"), (-0.4, "Z" * n)]
            ham = I.PauliSum.from_strings(n, terms)
            ham2 = I.random_2local(n, 30, 9)
            for h, name in ((ham, "wide terms"), (ham2, "2-local")):
                e, g = ctx.param_shift_grad(c, params, h, dtype)
                e_ref, g_ref = oracle.param_shift(c, params, h)
                tol = 1e-10 if dtype == C128 else 1e-5
                assert abs(e - e_ref) <= tol and np.max(np.abs(g - g_ref)) <= tol, (name, dtype)
                print(f"[debug-bounds] gradient {name} dtype={dtype}: ok", flush=True)
        # forced dense blocks (MFMA stages, complex64)
        kc = sv.Context(0, dense_fuse=4)
        try:
            n = 14
            circ = I.deep_random_circuit(n, 4, 11)
            psi0 = I.gaussian_state(n, 12)
            close(run(kc, circ, psi0, C64), oracle.run_circuit(circ, None, psi0), C64, "dense blocks")
        finally:
            kc.close()
    finally:
        ctx.close()
    print("debug-bounds ok", flush=True)


if __name__ == "__main__":
    main()
