"""Host-only planning through the C ABI (no device): the plan inspection
and parameter-shift expansion entry points on the regular library, and the
same driver under AddressSanitizer / UndefinedBehaviorSanitizer on the
sanitizer build of the host code.

  * The headline workload's plan: every tile pass of the 30-qubit depth-40
    circuit runs as rotation layers at both precisions (48 passes at the
    default widths), with no group-factor diagonal left in any stage.
  * The QFT's passes take the Hadamard/ladder stages; the ansatz layers
    (parameterised rotations and CNOT ladders) the three-bit engine.
  * Parameter-shift batches: 2 circuits per two-term occurrence, 4 per
    four-term one, plus the unshifted circuit.
  * Seeded random circuits of every gate kind and size 1..34, widths and
    dense blocks varied, and invalid arguments, through sv_plan_info /
    sv_plan_dump / sv_psr_info (tests/host_plan_driver.py), once on the
    regular library and once under the sanitizers in a child process that
    preloads the toolchain's AddressSanitizer runtime.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2512_23183_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "host_plan_driver.py")


@pytest.fixture(scope="module")
def sv():
    from paper_2512_23183_amd import sv as svmod
    return svmod


def test_deep_circuit_plans_as_rotation_layers(sv):
    # the planner searches the tile of each pass of a layered circuit
    # (uncontrolled one-qubit gates and diagonals only): 35 passes at the
    # default 12 bits where growing the tile in program order took 48
    c = I.deep_random_circuit(30, 40, 4)
    for dtype in (sv.C64, sv.C128):
        info = sv.plan_info(c, dtype=dtype)
        assert info["tile_passes"] == 35 and info["perm_passes"] == 0
        # list-scheduled passes reach ceil(rotations / 4) stages in every
        # pass (1200 rotations); program order took 336
        assert info["stages"] == 313
        assert info["tile_passes_by_engine"] == [0, 0, 0, 0, 35]
        dump = sv.plan_dump(c, dtype=dtype)
        assert "acc=1" not in dump  # every diagonal folded into a table or a tile factor


def test_layered_tile_width_and_search(sv):
    # layered circuits take tile_bits_layers, others tile_bits; the search
    # never takes fewer ops into a pass than growing the tile in program
    # order, so a layered plan never has more passes at a wider tile
    c = I.deep_random_circuit(24, 20, 9)
    p12 = sv.plan_info(c, dtype=sv.C64, tile_bits_c64=10, tile_bits_layers_c64=12)["tile_passes"]
    p10 = sv.plan_info(c, dtype=sv.C64, tile_bits_c64=12, tile_bits_layers_c64=10)["tile_passes"]
    assert p12 < p10
    hea = I.hea_circuit(20, 2)
    prm = I.uniform_params(hea.n_params, 1)
    a = sv.plan_info(hea, prm, dtype=sv.C64, tile_bits_c64=12, tile_bits_layers_c64=9)["tile_passes"]
    b = sv.plan_info(hea, prm, dtype=sv.C64, tile_bits_c64=12, tile_bits_layers_c64=12)["tile_passes"]
    assert a == b  # the ansatz (CNOTs, parameters) is not layered
    qft = I.CircuitBuilder(24)
    for j in range(24):
        qft.add(I.H, [j])
        for k in range(j + 1, 24):
            qft.add(I.CP, [k, j], angles=[np.pi / 2 ** (k - j)])
    q = qft.build(0)
    a = sv.plan_info(q, dtype=sv.C64, tile_bits_c64=12, tile_bits_layers_c64=9)["tile_passes"]
    b = sv.plan_info(q, dtype=sv.C64, tile_bits_c64=12, tile_bits_layers_c64=12)["tile_passes"]
    c9 = sv.plan_info(q, dtype=sv.C64, tile_bits_c64=9, tile_bits_layers_c64=12)["tile_passes"]
    assert a == b < c9  # the QFT's CP ladders follow the general width


def test_forced_dense_block_widths(sv):
    # dense_fuse = k in 2..4 (a measurement mode): every run of >= 2 fixed
    # gates on <= k qubits becomes a dense block; the default policy forms
    # none on U3 + CZ layers; complex128 never forms blocks; other values
    # are rejected before anything is planned or any device is touched
    c = I.deep_random_circuit(16, 8, 4)
    assert sv.plan_info(c, dtype=sv.C64)["dense_blocks"] == 0
    counts = {}
    for k in (2, 3, 4):
        info = sv.plan_info(c, dtype=sv.C64, dense_fuse=k)
        counts[k] = info["dense_blocks"]
        assert counts[k] > 0, k
        dump = sv.plan_dump(c, dtype=sv.C64, dense_fuse=k)
        assert "DENSE4" in dump
        assert sv.plan_info(c, dtype=sv.C128, dense_fuse=k)["dense_blocks"] == 0
    # wider blocks swallow more gates each: fewer of them
    assert counts[2] > counts[3] > counts[4], counts
    for bad in (5, -2):
        with pytest.raises(sv.SvError) as ei:
            sv.plan_info(c, dtype=sv.C64, dense_fuse=bad)
        assert ei.value.code == -1
        h = sv._vp()
        cfg = sv._config(dense_fuse=bad)
        assert sv.lib().sv_init(sv.ctypes.byref(h), 0, sv.ctypes.byref(cfg)) == -1
        assert not h


def test_qft_and_ansatz_engines(sv):
    from paper_2512_23183_amd import sv as S
    qft = I.CircuitBuilder(20)
    for j in range(20):
        qft.add(I.H, [j])
        for k in range(j + 1, 20):
            qft.add(I.CP, [k, j], angles=[np.pi / 2 ** (k - j)])
    info = S.plan_info(qft.build(0), dtype=S.C64)
    assert info["tile_passes_by_engine"][2] == info["tile_passes"] > 0
    hea = I.hea_circuit(20, 2)
    info = S.plan_info(hea, I.uniform_params(hea.n_params, 1), dtype=S.C64)
    assert info["tile_passes_by_engine"][0] == info["tile_passes"] > 0


def test_parameter_shift_expansion(sv):
    c = I.hea_circuit(10, 4)
    nc, sh = sv.psr_info(c, I.uniform_params(c.n_params, 1), I.xyz_chain(10))
    assert nc == 2 * 80 + 1 and np.all(sh == 2)
    b = I.CircuitBuilder(3)
    b.add(I.RY, [0], params=[0])
    b.add(I.CRX, [0, 1], params=[1])
    b.add(I.RZ, [2], params=[0])
    nc, sh = sv.psr_info(b.build(2), np.array([0.3, 0.7]), I.xyz_chain(3))
    assert list(sh) == [4, 4] and nc == 9


def test_host_driver_regular_library():
    r = subprocess.run([sys.executable, DRIVER, "30"], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "host plans 60" in r.stdout


def test_host_driver_under_sanitizers():
    sys.path.insert(0, os.path.join(ROOT, "paper_2512_23183_amd"))
    import build_asan
    if build_asan.stale():
        build_asan.build()
    env = dict(os.environ, LD_PRELOAD=build_asan.runtime(), SV_LIBRARY=build_asan.LIB,
               ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, DRIVER, "30"], capture_output=True, text=True, timeout=1200, env=env)
    assert r.returncode == 0 and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, \
        r.stderr[-4000:]
    assert "host plans 60" in r.stdout


def test_deep_small_circuit_plans_quickly(sv):
    # one pass holds every op of a circuit no wider than its tile: the stage
    # scheduler keeps its ready sets up to date instead of rescanning the
    # pass per stage, so 12 qubits x 4000 layers (48000 rotations) plan fast
    import time
    c = I.deep_random_circuit(12, 4000, 3)
    t0 = time.perf_counter()
    info = sv.plan_info(c, dtype=sv.C128)
    assert time.perf_counter() - t0 < 10.0
    assert info["tile_passes"] == 1 and info["stages"] == 12 * 4000 // 4
