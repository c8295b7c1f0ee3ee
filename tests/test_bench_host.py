"""Host logic of bench.py (no GPU): the touched-amplitude count of the QFT
against brute force over index sets, the traffic record's staleness check,
and the one-GPU guard."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _brute_touched_qft(n):
    # gate list of the gate-based QFT (H on q, then CP(q, j) for j > q; then
    # floor(n/2) SWAPs); a gate touches the indices it may change: all for
    # H, both bits set for CP, the two bits different for SWAP
    N = 1 << n
    bit = lambda q: 1 << (n - 1 - q)
    total = 0
    for q in range(n):
        total += N
        for j in range(q + 1, n):
            total += sum(1 for k in range(N) if k & bit(q) and k & bit(j))
    for q in range(n // 2):
        a, b = bit(q), bit(n - 1 - q)
        total += sum(1 for k in range(N) if bool(k & a) != bool(k & b))
    return total


def test_qft_touched_matches_brute_force():
    for n in range(2, 8):
        assert bench.qft_touched(n) == _brute_touched_qft(n), n
        assert bench.qft_gates(n) == n + n * (n - 1) // 2 + n // 2


def test_recorded_figures_require_matching_sources(tmp_path):
    good = tmp_path / "good.md"
    good.write_text("x\ntraffic_bytes_per_launch: 1.5e+09\nvalu_wave_instr_per_launch: 2.5e+08\n"
                    "source_sha256: %s\n" % bench.traffic_sources_sha())
    assert bench.recorded_traffic(str(good)) == 1.5e9
    assert bench.recorded_valu(str(good)) == 2.5e8
    stale = tmp_path / "stale.md"
    stale.write_text("traffic_bytes_per_launch: 1.5e+09\nsource_sha256: %s\n" % ("0" * 64))
    assert bench.recorded_traffic(str(stale)) is None
    assert bench.recorded_traffic(str(tmp_path / "missing.md")) is None


def test_roofline_block_from_launch_times():
    # two launches of 4 ms each moving 2 x 16 GiB: 8.59 TB/s algorithmic
    S = 16.0 * 2 ** 30
    r = bench.roofline_block(S, {"tile": (8.0, 2, 0.0), "perm": (0.0, 0, 0.0)}, "k")
    assert abs(r["avg_launch_ms"] - 4.0) < 1e-12
    assert abs(r["achieved"] - 2 * S / 4e-3 / 1e9) < 1e-6
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-12 and r["bound"] == "hbm"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_serving_requests_are_prefix_stable():
    # the serving bench takes the serial rate from a short list and runs the
    # loads on longer ones: their first requests must be the same circuits
    import numpy as np
    from paper_2512_23183_amd import inputs as I
    a = I.serving_requests(6, 5, rate_per_s=0.0, n_range=bench.SERVE_N, depth_range=bench.SERVE_DEPTH)
    b = I.serving_requests(15, 5, rate_per_s=3.0, n_range=bench.SERVE_N, depth_range=bench.SERVE_DEPTH)
    for x, y in zip(a, b):
        assert x.circuit.n == y.circuit.n and x.grad == y.grad and x.circuit.n_gates == y.circuit.n_gates
        assert np.array_equal(x.params, y.params)
        assert np.array_equal(x.hamiltonian.coeffs, y.hamiltonian.coeffs)
