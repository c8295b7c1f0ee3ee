"""Four-bit Hadamard/ladder stages (through the C ABI): tile passes made of
Hadamards, CP ladders and all-ones-pattern diagonals (CZ, CP) run in
stages of four register bits.  Random H / CZ / CP circuits (fixed angles, so
CP runs merge into ladders) against the oracle at sizes with one and with
several tile passes; a gradient whose shifted gates are parameterised CPs
inside such passes against the oracle and, bitwise, against the same
circuits run one at a time.  Tolerances: complex128 1e-12 (amplitudes,
relative L2) and 1e-10 (energies, gradients); complex64 1e-5.
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


def h_cz_cp_circuit(n, layers, seed):
    rng = np.random.default_rng(seed)
    b = I.CircuitBuilder(n)
    for _ in range(layers):
        for q in range(n):
            if rng.random() < 0.7:
                b.add(I.H, [q])
        # a QFT-like cascade from a random control (merges into a ladder)
        c = int(rng.integers(n))
        for t in range(c + 1, n):
            b.add(I.CP, [c, t], angles=[np.pi / 2 ** (t - c)])
        for _ in range(n // 2):
            q0, q1 = rng.choice(n, 2, replace=False)
            if rng.random() < 0.5:
                b.add(I.CZ, [int(q0), int(q1)])
            else:
                b.add(I.CP, [int(q0), int(q1)], angles=[float(rng.uniform(0, 2 * np.pi))])
    return b.build(0)


@pytest.mark.parametrize("n", [6, 9, 13, 14, 17, 20])
@pytest.mark.parametrize("dtype", [C64, C128])
def test_h_cz_cp_circuits_vs_oracle(sv, n, dtype):
    c = h_cz_cp_circuit(n, 4, 100 + n)
    want = oracle.run_circuit(c)
    with sv.Context(0) as ctx:
        st = ctx.alloc(n, dtype)
        st.apply(c)
        got = st.get_amplitudes().astype(np.complex128)
        st.free()
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert err <= (1e-12 if dtype == C128 else 1e-5), err


@pytest.mark.parametrize("dtype", [C128, C64])
def test_gradient_with_shifted_cp_in_hadamard_passes(sv, dtype):
    n = 15
    b = I.CircuitBuilder(n)
    k = 0
    for layer in range(2):
        for q in range(n):
            b.add(I.H, [q])
        for q in range(layer % 2, n - 1, 2):
            b.add(I.CP, [q, q + 1], params=[k])
            k += 1
    c = b.build(k)
    ham = I.random_2local(n, 20, 41)
    params = I.uniform_params(c.n_params, 43)
    with sv.Context(0) as ctx:
        e_b, g_b = ctx.param_shift_grad(c, params, ham, dtype)
        e_s, g_s = ctx.param_shift_grad(c, params, ham, dtype, flags=sv.FLAG_SEQUENTIAL)
    assert e_b == e_s and np.array_equal(g_b, g_s), np.max(np.abs(g_b - g_s))
    e_ref, g_ref = oracle.param_shift(c, params, ham)
    tol = 1e-10 if dtype == C128 else 1e-5
    assert abs(e_b - e_ref) <= tol
    assert np.max(np.abs(g_b - g_ref)) <= tol


@pytest.mark.parametrize("dtype", [C128, C64])
def test_gradient_with_zero_angle_rz_between_hadamard_layers(sv, dtype):
    # RZ(0) lowers to the identity diagonal, whose values alone would class
    # its pass as Hadamards and all-ones-pattern diagonals; its shifted
    # copies RZ(+-pi/2) are general diagonals and must still be applied as
    # such (15 qubits: the batched slab executor, not the LDS-resident one).
    # H RZ(t) H = RX(t), so <Y_q> = -sin t has derivative -1 at t = 0.
    n = 15
    b = I.CircuitBuilder(n)
    for q in range(n):
        b.add(I.H, [q])
    for q in range(n):
        b.add(I.RZ, [q], params=[q])
    for q in range(n):
        b.add(I.H, [q])
    c = b.build(n)
    params = np.zeros(n)
    rng = np.random.default_rng(77)
    terms = []
    for q in range(n):
        terms.append((float(rng.normal()), "I" * q + "Y" + "I" * (n - 1 - q)))
    for q in range(n - 1):
        s = ["I"] * n
        s[q], s[q + 1] = "XY"[q % 2], "Y"
        terms.append((float(rng.normal()), "".join(s)))
    ham = I.PauliSum.from_strings(n, terms)
    with sv.Context(0) as ctx:
        e_b, g_b = ctx.param_shift_grad(c, params, ham, dtype)
        e_s, g_s = ctx.param_shift_grad(c, params, ham, dtype, flags=sv.FLAG_SEQUENTIAL)
    assert e_b == e_s and np.array_equal(g_b, g_s), np.max(np.abs(g_b - g_s))
    e_ref, g_ref = oracle.param_shift(c, params, ham)
    tol = 1e-10 if dtype == C128 else 1e-5
    assert abs(e_b - e_ref) <= tol
    assert np.max(np.abs(g_b - g_ref)) <= tol
    # single-Y terms contribute -c_q to their parameter's derivative
    assert np.max(np.abs(g_ref)) > 0.1
