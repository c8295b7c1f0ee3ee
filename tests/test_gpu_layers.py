"""Rotation-layer passes with searched tiles and reordered stages (through
the C ABI).  Circuits of fixed uncontrolled one-qubit gates and diagonals
(layered circuits) get a searched tile per pass, and each pass's ops are
list-scheduled into four-bit stages, so the order in which the device
applies them differs from the program order wherever ops commute.  Random
layered circuits -- U3, RX, X, H on random subsets of qubits, with CZ, CP,
RZZ and RZ on random (also far-apart) qubits between them -- against the
oracle at several layered tile widths, so that the circuits span one to
many passes; and a gradient whose shifted gates are parameterised RZs
inside such passes against the oracle's shifted energies.  Tolerances:
complex128 1e-12 (amplitudes, relative L2; energies and gradients 1e-10),
complex64 1e-5.
"""
import numpy as np
import pytest

import oracle
from paper_2512_23183_amd import inputs as I

pytestmark = pytest.mark.gpu

C64, C128 = 0, 1


@pytest.fixture(scope="module")
def sv():
    from paper_2512_23183_amd import sv as svmod
    return svmod


def layered_circuit(n, layers, seed, rz_params=0, x_prob=0.1):
    rng = np.random.default_rng(seed)
    b = I.CircuitBuilder(n)
    p = 0
    for _ in range(layers):
        for q in range(n):
            u = rng.random()
            if u < 0.5:
                b.add(I.U3, [q], angles=list(rng.uniform(0, 2 * np.pi, 3)))
            elif u < 0.65:
                b.add(I.RX, [q], angles=[float(rng.uniform(0, 2 * np.pi))])
            elif u < 0.65 + x_prob:
                b.add(I.X, [q])
            elif u < 0.75 + x_prob:
                b.add(I.H, [q])
        for _ in range(n // 2 + 1):
            q0, q1 = (int(x) for x in rng.choice(n, 2, replace=False))
            k = rng.integers(4)
            if k == 0:
                b.add(I.CZ, [q0, q1])
            elif k == 1:
                b.add(I.CP, [q0, q1], angles=[float(rng.uniform(0, 2 * np.pi))])
            elif k == 2:
                b.add(I.RZZ, [q0, q1], angles=[float(rng.uniform(0, 2 * np.pi))])
            elif p < rz_params:
                b.add(I.RZ, [q0], params=[p])
                p += 1
            else:
                b.add(I.RZ, [q0], angles=[float(rng.uniform(0, 2 * np.pi))])
    return b.build(p)


# with X gates the passes take the general four-bit stages; without them
# most take the rotation-layer stages
@pytest.mark.parametrize("x_prob", [0.1, 0.0])
@pytest.mark.parametrize("n,width", [(8, 6), (12, 7), (12, 10), (16, 8), (16, 12), (19, 11)])
@pytest.mark.parametrize("dtype", [C64, C128])
def test_layered_circuits_vs_oracle(sv, n, width, dtype, x_prob):
    c = layered_circuit(n, 8, 300 + n + width, x_prob=x_prob)
    kw = {("tile_bits_layers_c64" if dtype == C64 else "tile_bits_layers_c128"): width}
    info = sv.plan_info(c, dtype=dtype, **kw)
    assert info["tile_passes"] >= 1 and info["stages"] >= info["tile_passes"]
    want = oracle.run_circuit(c)
    with sv.Context(0, **kw) as ctx:
        st = ctx.alloc(n, dtype)
        st.apply(c)
        got = st.get_amplitudes().astype(np.complex128)
        st.free()
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert err <= (1e-12 if dtype == C128 else 1e-5), (err, info["tile_passes"], info["stages"])


@pytest.mark.parametrize("dtype", [C128, C64])
def test_gradient_of_layered_circuit_vs_oracle(sv, dtype):
    n = 14
    c = layered_circuit(n, 6, 77, rz_params=10)
    assert c.n_params == 10
    theta = np.random.default_rng(5).uniform(0, 2 * np.pi, c.n_params)
    ham = I.random_2local(n, 30, 7)
    e_want = oracle.energy(oracle.run_circuit(c, theta), ham)[0]
    g_want = np.empty(c.n_params)
    for i in range(c.n_params):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += np.pi / 2
        tm[i] -= np.pi / 2
        g_want[i] = 0.5 * (oracle.energy(oracle.run_circuit(c, tp), ham)[0] -
                           oracle.energy(oracle.run_circuit(c, tm), ham)[0])
    kw = {("tile_bits_layers_c64" if dtype == C64 else "tile_bits_layers_c128"): 8}
    with sv.Context(0, **kw) as ctx:
        e, g = ctx.param_shift_grad(c, theta, ham, dtype)
    tol = 1e-10 if dtype == C128 else 1e-5
    assert abs(e - e_want) <= tol, (e, e_want)
    assert np.max(np.abs(g - g_want)) <= tol, np.max(np.abs(g - g_want))
