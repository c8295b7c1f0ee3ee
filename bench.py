"""Benchmark: state-vector hot path on one MI355X.

Headline workload (one "step"): the deep random circuit of 40 layers (U3
with angles U[0, 2 pi)^3 on each of 30 qubits, then CZ on a fresh random
perfect matching; 1800 logical gates, seed 4) applied to a resident
30-qubit complex128 state (16 GiB, the paper's FP64 complex amplitudes),
reset to |0...0> at the start of every step.  Metric: amplitude updates per
second = logical gates x 2^n per step / time.  The roofline block describes
the fused tile pass that carries the whole circuit: algorithmic bytes (one
read and one write of the state per pass) over its average launch time
(HIP events on its stream), against 8 TB/s HBM; the arithmetic it issues
per amplitude and its fraction of the FP64 vector peak go beside it.

Extras in the same JSON line (each bounded in time):
  deep30_c64      the same circuit on a complex64 state (the precision the
                  configuration names): fused and one launch per gate, with
                  the fused pass's roofline block
  qft28_c64/c128  gate-based QFT of the seeded 28-qubit Gaussian state: time,
                  passes and the tile pass's roofline block
  qft             20/24/28 qubits at complex64 and complex128, fused and one
                  launch per gate, GB/s per pass (states of at most 256 MiB
                  stay in the Infinity Cache: marked cache_resident)
  grad10          10-qubit complex128 VQE gradient (161 circuits): batched vs one
                  circuit at a time
  vqe10           the same ansatz and Hamiltonian minimised by Adam (lr 1e-2, at
                  most 350 iterations, tolerance 1e-7), one gradient per iteration
  grad20          20-qubit complex64 gradient, 8 layers (641 circuits), 200-term
                  random 2-local Hamiltonian: batched vs one circuit at a time
  sweeps          single-gate sweeps on an 8 GiB state: GB/s per gate and bit
  trotter         26-qubit XYZ-chain time evolution (20 first-order Trotter steps)
  serving         Poisson stream of mixed requests through the serving queue
                  (bounded sample), p50/p99 latency vs a serial loop
  cpu_oracle_1thread  the oracle QFT at 24 qubits on one host thread
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector (256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz)
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector with packed FP32 (the library does not emit packed FP32)
DEEP_N, DEEP_DEPTH, DEEP_SEED = 30, 40, 4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def qft_touched(n):
    """Amplitudes a gate-based QFT touches: 2^n per H, 2^(n-2) per CP (one
    quarter of the index set has both bits set), 2^(n-1) per SWAP."""
    return n * (1 << n) + n * (n - 1) // 2 * (1 << (n - 2)) + (n // 2) * (1 << (n - 1))


def qft_gates(n):
    return n + n * (n - 1) // 2 + n // 2


def sync_all(ctx):
    import torch
    ctx.synchronize()
    torch.cuda.synchronize()


def time_qft(ctx, sv, n, dtype, steps, warmup, flags=0, psi=None, profile=False):
    st = ctx.alloc(n, dtype)
    if psi is not None:
        st.set_amplitudes(psi)
    for _ in range(warmup):
        st.qft(flags)
    sync_all(ctx)
    if profile:
        ctx.profile_reset()
        ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        st.qft(flags)
    sync_all(ctx)
    dt = time.perf_counter() - t0
    prof = {}
    if profile:
        for name in ("tile", "perm"):
            prof[name] = ctx.profile_get(name)
        ctx.profile(False)
        ctx.profile_reset()
    return st, dt, prof


def deep_pass_profile(ctx, st, c):
    """One more application with per-kernel HIP-event timing: tile and
    permutation passes (count, total ms)."""
    ctx.synchronize()
    ctx.profile_reset()
    ctx.profile(True)
    st.reset()
    st.apply(c)
    ctx.synchronize()
    out = {k: ctx.profile_get(k) for k in ("tile", "perm")}
    ctx.profile(False)
    ctx.profile_reset()
    return out


def roofline_block(S, prof, kernel, steps_passes=None):
    """HBM roofline of a fused tile pass: 2S algorithmic bytes per launch
    over its average HIP-event duration."""
    tile_ms, tile_n, _ = prof["tile"]
    avg_ms = tile_ms / max(tile_n, 1)
    achieved = 2.0 * S / (avg_ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": kernel,
            "bytes_per_launch": 2.0 * S, "avg_launch_ms": avg_ms, "launches_per_step": tile_n}


def bench_deep_headline(ctx, sv, inputs, args, tuned, dtype=None):
    """The deep random circuit (30 qubits, depth 40) at complex128: reset + fused apply per
    step on a resident state."""
    dtype = sv.C128 if dtype is None else dtype
    n = DEEP_N
    c = inputs.deep_random_circuit(n, DEEP_DEPTH, DEEP_SEED)
    log(f"[bench] headline: deep random circuit n={n} depth={DEEP_DEPTH} {'c128' if dtype == sv.C128 else 'c64'}")
    st = ctx.alloc(n, dtype)
    for _ in range(args.warmup):
        st.reset()
        st.apply(c)
    sync_all(ctx)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st.reset()
        st.apply(c)
    sync_all(ctx)
    dt = time.perf_counter() - t0
    prof = deep_pass_profile(ctx, st, c)
    norm_err = st.norm2() - 1.0
    st.free()
    amp = 16 if dtype == sv.C128 else 8
    S = float(amp << n)
    G = c.n_gates
    info = sv.plan_info(c, dtype=dtype, **(tuned or {}))
    return {"value": G * float(1 << n) * args.steps / dt, "ms_per_step": dt / args.steps * 1e3, "n": n,
            "gates": G, "S": S, "prof": prof, "norm2_minus_1": norm_err, "plan": info}


def bench_qft_headline(ctx, sv, inputs, args, dtype=None, steps=None, warmup=None):
    n = 28
    dtype = sv.C64 if dtype is None else dtype
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    log(f"[bench] QFT n={n} {'c64' if dtype == sv.C64 else 'c128'}, generating input")
    psi = inputs.gaussian_state(n, 2)
    if dtype == sv.C64:
        psi = psi.astype(np.complex64)
    st, dt, prof = time_qft(ctx, sv, n, dtype, steps, warmup, psi=psi, profile=True)
    del psi
    G = qft_gates(n)
    au = G * float(1 << n) * steps
    S = (8.0 if dtype == sv.C64 else 16.0) * (1 << n)
    tile_ms, tile_n, tile_bytes = prof["tile"]
    perm_ms, perm_n, _ = prof["perm"]
    avg_tile_s = tile_ms / 1e3 / max(tile_n, 1)
    achieved = (2.0 * S) / avg_tile_s / 1e9
    st.free()
    return {
        "value": au / dt, "ms_per_step": dt / steps * 1e3, "n": n, "gates": G,
        "touched_au_per_s": qft_touched(n) * float(steps) / dt,
        "passes_per_step": (tile_n + perm_n) / steps,
        "tile_avg_ms": tile_ms / max(tile_n, 1), "perm_avg_ms": perm_ms / max(perm_n, 1),
        "tile_launches": tile_n, "achieved_gbs": achieved, "S": S,
        "pass_gbs": 2.0 * S * (tile_n + perm_n) / (dt) / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_tile (fused LDS tile pass; four-bit Hadamard/ladder stages)",
                     "bytes_per_launch": 2.0 * S, "avg_launch_ms": tile_ms / max(tile_n, 1)},
    }


def bench_qft_table(ctx, sv, inputs, oracle_mod):
    out = {}
    for n in (20, 24, 28):
        for dtype, name in ((sv.C64, "c64"), (sv.C128, "c128")):
            psi = inputs.gaussian_state(n, 2) if n <= 24 else None
            st = ctx.alloc(n, dtype)
            if psi is not None:
                st.set_amplitudes(psi)
                st.qft()
                got = st.get_amplitudes().astype(np.complex128)
                ref = math.sqrt(1 << n) * np.fft.ifft(psi)
                rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            else:
                rel = None
            st.free()
            reps = 3 if n <= 24 else 2
            st, dt, prof = time_qft(ctx, sv, n, dtype, reps, 1, profile=True)
            st.free()
            amp = 8 if dtype == sv.C64 else 16
            S = float(amp << n)
            G = qft_gates(n)
            tile_ms, tile_n, _ = prof["tile"]
            perm_ms, perm_n, _ = prof["perm"]
            passes = (tile_n + perm_n) / reps
            rec = {"au_per_s": G * float(1 << n) * reps / dt, "ms": dt / reps * 1e3,
                   "touched_au_per_s": qft_touched(n) * float(reps) / dt,
                   # a state of at most 256 MiB stays in the Infinity Cache
                   # between passes: not an HBM roofline measurement
                   "cache_resident": S <= 256.0 * 2 ** 20,
                   "passes": passes,
                   "gbs_per_pass": 2 * S * (tile_n + perm_n) / ((tile_ms + perm_ms) / 1e3) / 1e9
                   if tile_n + perm_n else None,
                   "rel_l2_vs_inverse_dft": rel}
            # one launch per gate (every size): GB/s per gate sweep, from the
            # algorithmic bytes and HIP-event times of the sweep launches
            st = ctx.alloc(n, dtype)
            sync_all(ctx)
            ctx.profile_reset()
            ctx.profile(True)
            t0 = time.perf_counter()
            st.qft(sv.FLAG_UNFUSED)
            sync_all(ctx)
            dt1 = time.perf_counter() - t0
            st.free()
            sw_ms = sw_n = sw_b = 0.0
            for k in ("sweep_u1", "sweep_phase", "sweep_xperm", "sweep_diag", "sweep_u2", "sweep_swap",
                      "sweep_ladder"):
                a, b, cb = ctx.profile_get(k)
                sw_ms += a
                sw_n += b
                sw_b += cb
            ctx.profile(False)
            ctx.profile_reset()
            rec["unfused_ms"] = dt1 * 1e3
            rec["unfused_au_per_s"] = G * float(1 << n) / dt1
            rec["unfused_sweeps"] = int(sw_n)
            rec["unfused_gbs_per_sweep"] = sw_b / (sw_ms / 1e3) / 1e9 if sw_ms else None
            out[f"n{n}_{name}"] = rec
            log(f"[bench] qft n={n} {name}: {rec['ms']:.3f} ms, {rec['au_per_s']:.3e} AU/s")
    return out


def bench_grad(ctx, sv, inputs, n, layers, dtype, ham, reps, seq_reps=1, seq_flags=None, direct_ctx=None):
    c = inputs.hea_circuit(n, layers)
    params = inputs.uniform_params(c.n_params, 1 if n == 10 else 3)
    circuits = 2 * c.n_params + 1
    ctx.param_shift_grad(c, params, ham, dtype)  # warm-up
    l0, i0 = ctx.graph_stats()
    t0 = time.perf_counter()
    for _ in range(reps):
        e, g = ctx.param_shift_grad(c, params, ham, dtype)
    dt = (time.perf_counter() - t0) / reps
    l1, i1 = ctx.graph_stats()
    rec = {"n": n, "params": c.n_params, "circuits": circuits, "gates_per_circuit": c.n_gates,
           "batched_ms": dt * 1e3, "batched_grads_per_s": 1.0 / dt,
           "au_per_s": circuits * c.n_gates * float(1 << n) / dt,
           "graph_launches": l1 - l0, "graph_instantiations": i1 - i0}
    if direct_ctx is not None:
        # the same batch launched kernel by kernel (no graph)
        direct_ctx.param_shift_grad(c, params, ham, dtype)
        t0 = time.perf_counter()
        for _ in range(reps):
            e3, g3 = direct_ctx.param_shift_grad(c, params, ham, dtype)
        dt3 = (time.perf_counter() - t0) / reps
        rec["batched_direct_launch_ms"] = dt3 * 1e3
        rec["batched_direct_launch_bitwise_equal"] = bool(e3 == e and np.array_equal(g3, g))
    for name, fl in (seq_flags or {}).items():
        t0 = time.perf_counter()
        for _ in range(seq_reps):
            e2, g2 = ctx.param_shift_grad(c, params, ham, dtype, fl)
        dts = (time.perf_counter() - t0) / seq_reps
        rec[f"{name}_ms"] = dts * 1e3
        rec[f"{name}_grads_per_s"] = 1.0 / dts
        rec[f"{name}_max_abs_diff_vs_batched"] = float(np.max(np.abs(g2 - g)))
    # one more call with per-kernel timing (launched directly): tile passes,
    # expectation passes and the shared-prefix copies; state_passes counts
    # (state, tile pass) pairs, each moving 2 x 2^n amplitudes
    ctx.profile_reset()
    ctx.profile(True)
    ctx.param_shift_grad(c, params, ham, dtype)
    amp = 8 if dtype == sv.C64 else 16
    for name in ("tile", "expect_tile", "share"):
        ms, nl, nbytes = ctx.profile_get(name)
        rec[f"{name}_ms"] = ms
        rec[f"{name}_launches"] = int(nl)
        if name == "tile":
            rec["state_passes"] = nbytes / (2.0 * amp * (1 << n))
            rec["tile_gbs"] = nbytes / (ms / 1e3) / 1e9 if ms > 0 else None
    ctx.profile(False)
    ctx.profile_reset()
    rec["energy"] = e
    return rec, (c, params, e, g)


def bench_deep30(ctx, sv, inputs, n=DEEP_N, depth=DEEP_DEPTH):
    c = inputs.deep_random_circuit(n, depth, DEEP_SEED)
    rec = {"n": n, "depth": depth, "gates": c.n_gates}
    st = ctx.alloc(n, sv.C64)
    for name, fl in (("fused", 0), ("unfused", sv.FLAG_UNFUSED)):
        st.reset()
        ctx.synchronize()
        ctx.profile_reset()
        ctx.profile(True)
        t0 = time.perf_counter()
        st.apply(c, None, fl)
        ctx.synchronize()
        dt = time.perf_counter() - t0
        names = ["tile", "perm"] if fl == 0 else ["sweep_u1", "sweep_phase", "sweep_xperm", "sweep_diag",
                                                  "sweep_u2", "sweep_swap", "sweep_ladder"]
        ms = nl = by = 0.0
        for k in names:
            a, b, cb = ctx.profile_get(k)
            ms += a
            nl += b
            by += cb
        ctx.profile(False)
        rec[name] = {"ms": dt * 1e3, "au_per_s": c.n_gates * float(1 << n) / dt, "launches": int(nl),
                     "kernel_ms": ms, "algorithmic_gbs": by / (ms / 1e3) / 1e9 if ms else None,
                     "norm2_minus_1": st.norm2() - 1.0}
        if fl == 0 and nl:
            achieved = by / (ms / 1e3) / 1e9
            rec[name]["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                                     "kernel": "k_tile (rotation-layer stages)",
                                     "bytes_per_launch": 2.0 * 8 * (1 << n), "avg_launch_ms": ms / nl}
        log(f"[bench] deep30 {name}: {dt*1e3:.1f} ms")
    st.free()
    rec["dense_blocks"] = bench_deep30_blocks(sv, c, n)
    return rec


def bench_deep30_blocks(sv, c, n):
    """The same complex64 circuit with every run of at least two fixed gates
    on at most k qubits forced into a dense block (dense_fuse = k, MFMA
    16 x 16 stages), k = 2, 3, 4: one warm-up and one timed application
    each.  The default policy forms no blocks on these layers."""
    out = {}
    for k in (2, 3, 4):
        info = sv.plan_info(c, dtype=sv.C64, dense_fuse=k)
        kc = sv.Context(0, dense_fuse=k)
        try:
            st = kc.alloc(n, sv.C64)
            st.apply(c)
            kc.synchronize()
            t0 = time.perf_counter()
            st.apply(c)
            kc.synchronize()
            dt = time.perf_counter() - t0
            st.free()
        finally:
            kc.close()
        out[f"k{k}"] = {"ms": dt * 1e3, "blocks": info["dense_blocks"], "stages": info["stages"],
                        "tile_passes": info["tile_passes"]}
        log(f"[bench] deep30 c64 forced k={k} blocks: {dt*1e3:.1f} ms ({info['dense_blocks']} blocks)")
    return out


def bench_vqe(ctx, sv, inputs):
    """VQE of the 10-qubit XYZ chain at the paper's optimiser settings (Adam, lr 1e-2, at most
    350 iterations, tolerance 1e-7), one batched gradient per iteration."""
    c = inputs.hea_circuit(10, 4)
    ham = inputs.xyz_chain(10)
    p0 = inputs.uniform_params(c.n_params, 1)
    ctx.vqe_adam(c, p0, ham, sv.C128, max_iters=3)  # warm-up
    t0 = time.perf_counter()
    th, e = ctx.vqe_adam(c, p0, ham, sv.C128)
    dt = time.perf_counter() - t0
    e0 = -9.161997432407  # exact diagonalisation of the 10-site chain
    rec = {"n": 10, "dtype": "c128", "iterations": int(len(e)), "ms": dt * 1e3,
           "ms_per_iteration": dt * 1e3 / len(e), "energy_first": float(e[0]), "energy_final": float(e[-1]),
           "exact_ground_energy": e0, "gap_to_ground": float(e[-1] - e0)}
    log(f"[bench] vqe10: {len(e)} iterations in {dt*1e3:.1f} ms, E {e[0]:.6f} -> {e[-1]:.6f} (E0 {e0})")
    return rec


def bench_trotter(ctx, sv, inputs, n=26, steps=20, t_total=2.0):
    """Time evolution of the XYZ chain (first-order Trotter, field
    h(t) = 2 sin t) on a resident complex64 state, and its final energy."""
    c = inputs.trotter_xyz_circuit(n, steps, t_total)
    st = ctx.alloc(n, sv.C64)
    st.apply(c)  # warm-up
    st.reset()
    ctx.synchronize()
    t0 = time.perf_counter()
    st.apply(c)
    ctx.synchronize()
    dt = time.perf_counter() - t0
    e = st.expectation(inputs.xyz_chain(n, h=inputs.xyz_field(t_total)))
    st.free()
    rec = {"n": n, "steps": steps, "t": t_total, "gates": c.n_gates, "ms": dt * 1e3,
           "au_per_s": c.n_gates * float(1 << n) / dt, "energy_final": e}
    log(f"[bench] trotter n={n}: {dt*1e3:.1f} ms, {rec['au_per_s']:.3e} AU/s")
    return rec


def bench_sweeps(ctx, sv, inputs):
    """GB/s of single-gate sweeps (the plain path: one launch per gate) on an
    8 GiB state, per gate and target position: algorithmic bytes (the
    amplitudes the gate reads and writes) over the kernel's own time."""
    out = {}
    I = inputs
    for n, dtype, dname in ((30, sv.C64, "c64"), (29, sv.C128, "c128")):
        st = ctx.alloc(n, dtype)
        cases = []
        for q in (0, n // 2, n - 5, n - 2, n - 1):
            cases.append((f"u3_q{q}", I.U3, [q], [0.3, 0.7, 1.1], "sweep_u1"))
        cases += [("cnot_q0_q%d" % (n - 1), I.CNOT, [0, n - 1], [], "sweep_xperm"),
                  ("cz_q0_q%d" % (n // 2), I.CZ, [0, n // 2], [], "sweep_phase"),
                  ("swap_q1_q%d" % (n - 3), I.SWAP, [1, n - 3], [], "sweep_swap")]
        rec = {}
        for name, kind, qs, ang, kname in cases:
            b = I.CircuitBuilder(n)
            b.add(kind, qs, angles=ang)
            c = b.build()
            st.apply(c, None, sv.FLAG_UNFUSED)  # warm-up
            ctx.synchronize()
            ctx.profile_reset()
            ctx.profile(True)
            for _ in range(5):
                st.apply(c, None, sv.FLAG_UNFUSED)
            ctx.synchronize()
            ms, cnt, by = ctx.profile_get(kname)
            ctx.profile(False)
            rec[name] = {"kernel": kname, "ms": ms / cnt, "gbs": by / (ms / 1e3) / 1e9,
                         "frac_of_8tbs": by / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}
        st.free()
        out[f"n{n}_{dname}"] = rec
        log("[bench] sweeps n=%d %s: %s" % (n, dname, ", ".join(f"{k} {v['gbs']:.0f}" for k, v in rec.items())))
    return out


SERVE_N = (8, 24)
SERVE_DEPTH = (2, 10)


def bench_serving(ctx, sv, inputs, count, seed=5, serial_count=48, small_n=16, tick_budget=None, loads=None,
                  progress=0):
    """The serving request mix (qubits 8..24, depth 2..10, 20-200 terms, half
    gradients, complex64) through the queue at 0.8x and 2x the serial rate
    and in a burst (or the (load, count) pairs in loads).  The serial
    plain-GPU rate mu comes from the first serial_count requests of the same
    list run one at a time; p50 / p99 are reported over all requests and
    over those of at most small_n qubits.  progress > 0 logs a line every
    that many submissions and completions."""
    # the generator is prefix-stable: the first serial_count requests of any
    # longer list are these
    reqs = inputs.serving_requests(serial_count, seed, rate_per_s=0.0, n_range=SERVE_N, depth_range=SERVE_DEPTH)
    t0 = time.perf_counter()
    for r in reqs[:serial_count]:
        if r.grad:
            ctx.param_shift_grad(r.circuit, r.params, r.hamiltonian, sv.C64, sv.FLAG_SEQUENTIAL)
        else:
            st = ctx.alloc(r.circuit.n, sv.C64)
            st.apply(r.circuit, r.params)
            st.expectation(r.hamiltonian)
            st.free()
    serial_dt = (time.perf_counter() - t0) / serial_count
    mu = 1.0 / serial_dt
    out = {"serial_requests": serial_count, "serial_req_per_s": mu, "n_range": list(SERVE_N),
           "depth_range": list(SERVE_DEPTH), "small_n_max": small_n}
    if loads is None:
        loads = ((0.8, min(count, 200)), (2.0, count), ("burst", count))
    log(f"[bench] serving: serial rate {mu:.2f} requests/s over {serial_count} requests")
    for load, cnt in loads:
        # burst: every request arrives at once (peak queue throughput)
        lam = 0.0 if load == "burst" else load * mu
        reqs = inputs.serving_requests(cnt, seed, rate_per_s=lam, n_range=SERVE_N, depth_range=SERVE_DEPTH)
        q = ctx.queue(64 << 30)
        if tick_budget is not None:
            q.set_tick_budget(tick_budget)
        tickets = []
        t_start = time.perf_counter()
        for r in reqs:
            now = time.perf_counter() - t_start
            if r.arrival_s > now:
                time.sleep(r.arrival_s - now)
            tickets.append(q.submit(r.circuit, r.params, r.hamiltonian, r.grad, sv.C64))
            if progress and len(tickets) % progress == 0:
                log(f"[bench] serving load {load}: {len(tickets)} submitted at {time.perf_counter() - t_start:.0f} s")
        lat = []
        for t in tickets:
            _, _, l = q.wait(t)
            lat.append(l)
            if progress and len(lat) % progress == 0:
                log(f"[bench] serving load {load}: {len(lat)} completed at {time.perf_counter() - t_start:.0f} s")
        total = time.perf_counter() - t_start
        st = q.stats()
        q.close()
        lat = np.array(lat)
        small = np.array([r.circuit.n <= small_n for r in reqs])
        rec = {"requests": cnt, "arrival_rate": lam, "req_per_s": cnt / total,
               "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
               "small_requests": int(small.sum()),
               "small_p50_ms": float(np.percentile(lat[small], 50) * 1e3) if small.any() else None,
               "small_p99_ms": float(np.percentile(lat[small], 99) * 1e3) if small.any() else None,
               "launches": st["launches"], "circuits": st["circuits_run"]}
        out[f"load_{load}"] = rec
        log(f"[bench] serving load {load}: {cnt} requests, {rec['req_per_s']:.1f}/s, p50 {rec['p50_ms']:.1f} ms, "
            f"p99 {rec['p99_ms']:.1f} ms (n <= {small_n}: p99 {rec['small_p99_ms']:.1f} ms)")
    return out


# Sources that decide what the headline tile kernel reads, writes and
# issues; recorded counter figures are reported only while they are
# unchanged.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_tile_deep30_c128_traffic.md")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_tile_deep30_c128_counters.md")
TRAFFIC_SOURCES = ["paper_2512_23183_amd/csrc/kernels.hip", "paper_2512_23183_amd/csrc/tile_kernel.h",
                   "paper_2512_23183_amd/csrc/device_common.h", "paper_2512_23183_amd/csrc/plan.cpp",
                   "paper_2512_23183_amd/csrc/lower.cpp", "paper_2512_23183_amd/csrc/sv_internal.h",
                   "paper_2512_23183_amd/csrc/tune.cpp", "paper_2512_23183_amd/csrc/tile_h4.h"]


def traffic_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _recorded(path, key):
    """A figure from a committed counter summary, or None when the summary
    is missing or was taken from other sources than the current ones."""
    try:
        with open(path) as f:
            text = f.read()
    except OSError:
        return None
    vals = dict(line.split(":", 1) for line in text.splitlines()
                if line.startswith((key + ":", "source_sha256:")))
    if vals.get("source_sha256", "").strip() != traffic_sources_sha():
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def recorded_traffic(path):
    """HBM bytes per tile launch (FETCH_SIZE + WRITE_SIZE, calibrated)."""
    return _recorded(path, "traffic_bytes_per_launch")


def recorded_valu(path):
    """VALU wave instructions per tile launch (SQ_INSTS_VALU)."""
    return _recorded(path, "valu_wave_instr_per_launch")


def copy_ceiling_gbs(nbytes=2 << 30, reps=5):
    """Read + write GB/s of plain device streams over nbytes (torch's copy
    and its out-of-place negation, HIP events; the faster one): the
    practical streaming ceiling beside the 8 TB/s peak."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    best = (0.0, None)
    for name, f in (("copy", lambda: dst.copy_(src)), ("neg", lambda: torch.neg(src, out=dst))):
        f()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        e1.synchronize()
        gbs = 2.0 * nbytes / (e0.elapsed_time(e1) / reps / 1e3) / 1e9
        best = max(best, (gbs, name))
    del src, dst
    torch.cuda.empty_cache()
    return best


def copy_calibration():
    """A plain streaming kernel of known size (read 1 GiB, write 1 GiB per
    dispatch) whose FETCH_SIZE / WRITE_SIZE scale the counter readings."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": src.numel() * 4, "dispatches": 3}), flush=True)


def cpu_baseline(oracle_mod, inputs, layers=3):
    """The oracle on a bounded sample of the headline workload: the first
    `layers` layers (U3 on every qubit, CZ matching) of the 30-qubit depth-40
    circuit from |0...0>, FP64 complex, on the host's cores (about ten
    seconds)."""
    c = inputs.deep_random_circuit(DEEP_N, DEEP_DEPTH, DEEP_SEED)
    per_layer = DEEP_N + DEEP_N // 2
    sub = inputs.Circuit(c.n, c.gates[: layers * per_layer].copy(), c.mats, 0)
    t0 = time.perf_counter()
    psi = oracle_mod.run_circuit(sub)
    dt = time.perf_counter() - t0
    del psi
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": sub.n_gates * float(1 << DEEP_N) / dt, "unit": "amplitude-updates/s", "cores": cores,
            "kind": "oracle",
            "sample": f"FP64 oracle gate by gate, first {layers} of {DEEP_DEPTH} layers ({sub.n_gates} gates) "
                      f"of the {DEEP_N}-qubit circuit from |0...0> ({dt:.1f} s)"}


def cpu_baseline_1thread(n=24):
    """The same oracle QFT on one host thread (OMP_NUM_THREADS=1, a child
    process that never touches the GPU), on a smaller state."""
    code = ("import sys, time; sys.path.insert(0, %r); import oracle; "
            "from paper_2512_23183_amd import inputs; psi = inputs.gaussian_state(%d, 2); "
            "t0 = time.perf_counter(); oracle.qft(psi); print(time.perf_counter() - t0)" % (ROOT, n))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    if r.returncode != 0:
        return None
    dt = float(r.stdout.strip().splitlines()[-1])
    return {"value": qft_gates(n) * float(1 << n) / dt, "unit": "amplitude-updates/s", "cores": 1,
            "kind": "oracle", "sample": f"FP64 oracle gate-by-gate QFT on one {n}-qubit Gaussian state "
                                        f"({qft_gates(n)} gates, {dt:.1f} s, one thread)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="headline only")
    ap.add_argument("--serving", type=int, default=1000, help="serving sample size at 2x and in a burst (0 = skip)")
    ap.add_argument("--stream-requests", type=int, default=10000,
                    help="requests of --only serving_stream (one stream at 2x the serial rate)")
    ap.add_argument("--skip-cpu", action="store_true", help="omit the CPU oracle baseline (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the plain streaming kernel used to scale HBM byte counters")
    ap.add_argument("--only", choices=["grad10", "grad20", "vqe10", "trotter", "deep30", "deep30_once",
                                       "qft28_once", "deep30_dense4_once", "serving_stream"],
                    help="profiling aid: run only this extra (no headline) and print its record")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the simulator runs one state per GPU; the measured path is one MI355X's)", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    import oracle
    from paper_2512_23183_amd import inputs
    from paper_2512_23183_amd import sv

    ctx = sv.Context(0)
    # tile widths from the library's autotuner (cache in the temp directory);
    # complex128 is tuned at the headline's 30 qubits: at 27 the 11- and
    # 12-bit rotation-layer passes time within 1% of each other, at 30 the
    # 12-bit ones are 8% faster
    import tempfile
    cache = os.path.join(tempfile.gettempdir(), "sv_autotune_cache.txt")
    t_tune = time.perf_counter()
    ctx.autotune(sv.C128, DEEP_N, cache)
    tuned = ctx.autotune(sv.C64, 28, cache)
    log(f"[bench] autotuned widths: {tuned} ({time.perf_counter() - t_tune:.1f} s)")
    if args.only:
        if args.only == "grad10":
            rec, _ = bench_grad(ctx, sv, inputs, 10, 4, sv.C128, inputs.xyz_chain(10), 20, 3)
        elif args.only == "grad20":
            rec, _ = bench_grad(ctx, sv, inputs, 20, 8, sv.C64, inputs.random_2local(20, 200, 3), 2, 1)
        elif args.only == "vqe10":
            rec = bench_vqe(ctx, sv, inputs)
        elif args.only == "trotter":
            rec = bench_trotter(ctx, sv, inputs)
        elif args.only == "serving_stream":
            # the full-length stream: 10k requests at twice the
            # serial rate (about 12 minutes on one GPU)
            rec = bench_serving(ctx, sv, inputs, args.stream_requests, loads=((2.0, args.stream_requests),),
                                progress=1000)
        elif args.only == "deep30_once":
            # one fused application at complex128 (counter collection)
            c = inputs.deep_random_circuit(DEEP_N, DEEP_DEPTH, DEEP_SEED)
            st = ctx.alloc(DEEP_N, sv.C128)
            st.apply(c)
            ctx.synchronize()
            st.free()
            rec = {"n": DEEP_N, "dtype": "c128", "gates": c.n_gates}
        elif args.only == "deep30_dense4_once":
            # one fused complex64 application with forced four-qubit dense
            # blocks (MFMA counter collection)
            c = inputs.deep_random_circuit(DEEP_N, DEEP_DEPTH, DEEP_SEED)
            kc = sv.Context(0, dense_fuse=4)
            st = kc.alloc(DEEP_N, sv.C64)
            st.apply(c)
            kc.synchronize()
            st.free()
            kc.close()
            rec = {"n": DEEP_N, "dtype": "c64", "dense_fuse": 4}
        elif args.only == "qft28_once":
            # one fused QFT of a 28-qubit state at each precision (counter
            # collection; the kernels' work does not depend on the values)
            for dt in (sv.C64, sv.C128):
                st = ctx.alloc(28, dt)
                st.qft()
                ctx.synchronize()
                st.free()
            rec = {"n": 28, "dtype": ["c64", "c128"]}
        else:
            rec = bench_deep30(ctx, sv, inputs)
        ctx.close()
        print(json.dumps({"only": args.only, "record": rec}), flush=True)
        return
    head = bench_deep_headline(ctx, sv, inputs, args, tuned)
    roof = roofline_block(head["S"], head["prof"], "k_tile (fused LDS tile pass; rotation-layer stages)")
    roof["traffic"] = recorded_traffic(TRAFFIC_FILE)
    valu = recorded_valu(COUNTERS_FILE)
    if valu is not None:
        # VALU issue: wave instructions x 4 cycles (wave64 on 16 lanes) over
        # the SIMD cycles of one launch (1024 SIMDs at 2.4 GHz); FP64 FMA
        # issues at the full rate, so this is the fraction of the FP64
        # vector peak the pass's instruction stream could use
        roof["valu_wave_instr_per_launch"] = valu
        roof["valu_issue_frac"] = valu * 4.0 / (1024 * 2.4e9 * roof["avg_launch_ms"] / 1e3)
        roof["fp64_vector_peak_tflops"] = FP64_PEAK_TFLOPS
    extras = {"headline": {"passes_per_step": head["prof"]["tile"][1] + head["prof"]["perm"][1],
                           "perm_launches": head["prof"]["perm"][1], "norm2_minus_1": head["norm2_minus_1"],
                           "plan": head["plan"]}}
    copy_gbs = copy_kernel = None
    if not args.quick:
        copy_gbs, copy_kernel = copy_ceiling_gbs()
        log(f"[bench] device stream ceiling: {copy_gbs:.0f} GB/s ({copy_kernel})")
        roof["copy_ceiling_gbs"] = copy_gbs
        roof["copy_ceiling_kernel"] = copy_kernel
        roof["frac_of_copy_ceiling"] = roof["achieved"] / copy_gbs
        extras["deep30_c64"] = bench_deep30(ctx, sv, inputs)
        for dt, nm in ((sv.C64, "qft28_c64"), (sv.C128, "qft28_c128")):
            q = bench_qft_headline(ctx, sv, inputs, args, dt, steps=10, warmup=2)
            extras[nm] = {"au_per_s": q["value"], "ms_per_step": q["ms_per_step"],
                          "touched_au_per_s": q["touched_au_per_s"], "passes_per_step": q["passes_per_step"],
                          "perm_avg_ms": q["perm_avg_ms"], "pass_gbs": q["pass_gbs"], "roofline": q["roofline"]}
            log(f"[bench] {nm}: {q['ms_per_step']:.2f} ms")
        extras["qft"] = bench_qft_table(ctx, sv, inputs, oracle)
        direct = sv.Context(0, graph_batch=-1, **tuned)
        rec10, _ = bench_grad(ctx, sv, inputs, 10, 4, sv.C128, inputs.xyz_chain(10), 20, 3,
                              {"sequential": sv.FLAG_SEQUENTIAL,
                               "sequential_unfused": sv.FLAG_SEQUENTIAL | sv.FLAG_UNFUSED}, direct)
        extras["grad10_c128"] = rec10
        extras["vqe10_c128"] = bench_vqe(ctx, sv, inputs)
        log(f"[bench] grad10: {rec10['batched_ms']:.3f} ms (direct launches "
            f"{rec10['batched_direct_launch_ms']:.3f} ms)")
        rec20, _ = bench_grad(ctx, sv, inputs, 20, 8, sv.C64, inputs.random_2local(20, 200, 3), 2, 1,
                              {"sequential": sv.FLAG_SEQUENTIAL}, direct)
        extras["grad20_c64"] = rec20
        log(f"[bench] grad20: {rec20['batched_ms']:.2f} ms (direct launches "
            f"{rec20['batched_direct_launch_ms']:.2f} ms)")
        direct.close()
        extras["sweeps"] = bench_sweeps(ctx, sv, inputs)
        extras["trotter_xyz_c64"] = bench_trotter(ctx, sv, inputs)
        if args.serving > 0:
            extras["serving"] = bench_serving(ctx, sv, inputs, args.serving)
    cpu = cpu_baseline(oracle, inputs) if rank == 0 and not args.skip_cpu else None
    if cpu is not None and not args.quick:
        extras["cpu_oracle_1thread"] = cpu_baseline_1thread()
    ctx.close()
    line = {
        "metric": "amplitude-updates/s", "value": head["value"], "unit": "amplitude-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"deep_random_circuit_n{DEEP_N}_depth{DEEP_DEPTH}_complex128",
                   "n_qubits": DEEP_N, "depth": DEEP_DEPTH, "logical_gates": head["gates"],
                   "circuit": "per layer U3(theta, phi, lambda) on every qubit, angles U[0, 2 pi)^3, "
                              "then CZ on a fresh random perfect matching (seed 4)",
                   "input": "|0...0>, reset every step", "state_bytes": head["S"],
                   "autotuned_widths": tuned},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    if rank == 0:
        print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
