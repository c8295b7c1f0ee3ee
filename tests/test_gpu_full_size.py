"""Full-size checks (through the C ABI) at the benchmark's sizes and at the
largest states one GPU holds, on outputs computable one by one or on
properties that hold at any size.

  * QFT of a basis state |x> at 28 qubits (the headline size, same entry
    point): psi[k] = exp(+2 pi i x k / N) / sqrt(N) (the closed form the
    oracle is pinned to), on 4096 sampled indices and the norm.
    Tolerance: complex64 |sqrt(N) psi[k] - exp(...)| <= 2e-5 (420 gates of
    ~6e-8 rounding each on a unit-modulus value, as a random walk, plus the
    FP32 phase tables), complex128 <= 1e-11.
  * QFT of |0> at 33 qubits complex64 (64 GiB) and 32 qubits complex128
    (64 GiB): the uniform state |+>^n, so <X_q> = 1 for every qubit and the
    norm is 1 (FP64 reductions: 1e-4 for complex64, 1e-9 for complex128).
  * The config-3 gradient (20 qubits, 8 layers, 641 circuits, 200 terms,
    complex64): sampled components against the oracle's shifted energies
    (g_i = [E(theta + pi/2 e_i) - E(theta - pi/2 e_i)] / 2), <= 1e-5.
"""
import math

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


@pytest.mark.parametrize("dtype,tol", [(C64, 2e-5), (C128, 1e-11)])
def test_qft28_basis_state_sampled_closed_form(sv, dtype, tol):
    n = 28
    N = 1 << n
    x = 0x9E3779B & (N - 1)
    b = I.CircuitBuilder(n)
    for q in range(n):
        if (x >> (n - 1 - q)) & 1:  # qubit q is index bit n - 1 - q
            b.add(I.X, [q])
    with sv.Context(0) as ctx:
        st = ctx.alloc(n, dtype)
        st.apply(b.build(0))
        st.qft()
        assert abs(st.norm2() - 1.0) <= (1e-5 if dtype == C64 else 1e-12)
        psi = st.get_amplitudes()
        st.free()
    rng = np.random.default_rng(11)
    ks = np.concatenate([[0, 1, N - 1, N // 2], rng.integers(0, N, 4092)])
    # exact phase x k / N mod 1 in integer arithmetic
    turns = ((x * ks) % N).astype(np.float64) / N
    want = np.exp(2j * math.pi * turns)
    got = psi[ks].astype(np.complex128) * math.sqrt(N)
    assert np.max(np.abs(got - want)) <= tol


@pytest.mark.parametrize("n,dtype,tol", [(33, C64, 1e-4), (32, C128, 1e-9)])
def test_qft_of_zero_at_the_largest_sizes(sv, n, dtype, tol):
    ham = I.PauliSum.from_strings(n, [(1.0, "I" * q + "X" + "I" * (n - 1 - q)) for q in range(n)])
    with sv.Context(0) as ctx:
        st = ctx.alloc(n, dtype)
        st.qft()
        nn = st.norm2()
        e, vals = st.expectation(ham, terms=True)
        st.free()
    assert abs(nn - 1.0) <= tol
    assert np.max(np.abs(vals - 1.0)) <= tol
    assert abs(e - n) <= n * tol


def test_config3_gradient_sampled_components(sv):
    n = 20
    c = I.hea_circuit(n, 8)
    ham = I.random_2local(n, 200, 3)
    params = I.uniform_params(c.n_params, 3)
    with sv.Context(0) as ctx:
        e, g = ctx.param_shift_grad(c, params, ham, C64)
    assert abs(e - oracle.circuit_energy(c, params, ham)) <= 1e-5
    for i in (0, 157, c.n_params - 1):
        tp = params.copy()
        tp[i] += math.pi / 2
        tm = params.copy()
        tm[i] -= math.pi / 2
        gi = 0.5 * (oracle.circuit_energy(c, tp, ham) - oracle.circuit_energy(c, tm, ham))
        assert abs(g[i] - gi) <= 1e-5, (i, g[i], gi)
