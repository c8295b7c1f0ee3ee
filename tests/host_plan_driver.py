"""Drives the host-only entry points (validation, lowering, planning,
device-plan build, parameter-shift expansion) over seeded random circuits
of every gate kind and size, and over invalid arguments.  Run by the CPU
tests in a child process, against the regular library or the sanitizer
build of the host code (SV_LIBRARY); it prints one summary line and exits
0, or raises.  No device is touched."""
import os
import sys

import numpy as np

sys.modules.setdefault("torch", None)  # the host entry points need no torch runtime
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_2512_23183_amd import inputs as I  # noqa: E402
from paper_2512_23183_amd import sv  # noqa: E402

def main(rounds):
    rng = np.random.default_rng(2024)
    plans = psrs = refused = 0
    for it in range(rounds):
        n = int(rng.choice([1, 2, 3, 4, 5, 7, 9, 12, 13, 14, 17, 20, 24, 28, 30, 33, 34]))
        if rng.random() < 0.25:
            # layered circuits: the rotation-layer planning path
            c = I.deep_random_circuit(n, int(rng.integers(1, 8)), it) if n >= 2 else \
                I.random_circuit(n, 10, it)
        else:
            c = I.random_circuit(n, int(rng.integers(0, 120)), it, n_params=int(rng.integers(0, 6)))
        params = rng.uniform(0, 2 * np.pi, c.n_params)
        for dtype in (sv.C64, sv.C128):
            widths = {}
            if rng.random() < 0.5:
                widths = {"tile_bits_c64": int(rng.integers(6, 15)), "tile_bits_c128": int(rng.integers(6, 13)),
                          "dense_fuse": int(rng.choice([-1, 1]))}
            info = sv.plan_info(c, params, dtype, **widths)
            assert sum(info["tile_passes_by_engine"]) == info["tile_passes"], info
            if info["tile_passes"]:
                assert 0.0 < info["min_pass_scale"] <= info["max_pass_scale"] < float("inf"), info
            text = sv.plan_dump(c, params, dtype, **widths)
            assert text.count("pass ") == info["tile_passes"] + info["perm_passes"] + info["sweep_passes"]
            plans += 1
        if c.n_params and n <= 24:
            ham = I.random_2local(n, 10, it) if n >= 2 else I.PauliSum.from_strings(1, [(1.0, "Z")])
            nc, sh = sv.psr_info(c, params, ham)
            assert nc == 1 + int(sh.sum()), (nc, sh)
            psrs += 1
        # invalid variants must be refused with SV_EINVAL, before any work
        for bad in ("params", "qubit"):
            try:
                if bad == "params":
                    sv.plan_info(c, np.zeros(c.n_params + 1), sv.C64)
                else:
                    g = c.gates.copy()
                    if g.size == 0:
                        raise sv.SvError(-1, "no gate to corrupt")
                    g[0]["q"][0] = n + 3
                    sv.plan_info(I.Circuit(c.n, g, c.mats, c.n_params), params, sv.C64)
                raise AssertionError("invalid circuit accepted")
            except sv.SvError as e:
                assert e.code == -1, e
                refused += 1
    print(f"host plans {plans}, gradients {psrs}, refusals {refused}", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 60)
