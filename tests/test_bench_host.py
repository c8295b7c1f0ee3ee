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


def test_recorded_traffic_requires_matching_sources(tmp_path, monkeypatch):
    good = tmp_path / "good.md"
    good.write_text("x\ntraffic_bytes_per_launch: 1.5e+09\nsource_sha256: %s\n" % bench.traffic_sources_sha())
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(good))
    assert bench.recorded_traffic() == 1.5e9
    stale = tmp_path / "stale.md"
    stale.write_text("traffic_bytes_per_launch: 1.5e+09\nsource_sha256: %s\n" % ("0" * 64))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale))
    assert bench.recorded_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.recorded_traffic() is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
