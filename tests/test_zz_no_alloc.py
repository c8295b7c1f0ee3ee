"""The entry point that allocates nothing (sv_apply_circuit_noalloc, through
the C ABI) against the fused apply it varies (sv_apply_circuit) and the
oracle: two calls in a row, the second with a smaller input (fewer qubits,
fewer ops), so stale contents of the shared preallocated block from the
first call would show; and a circuit whose plan tables exceed the block is
refused before any device work.

Tolerances as for every apply: complex128 <= 1e-12 absolute per amplitude,
complex64 relative L2 error <= 1e-5 max(1, sqrt(G / 500)) for G gates; the
two entry points share plan and kernels, so their outputs must also be
bitwise equal.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2512_23183_amd import inputs as I

pytestmark = pytest.mark.gpu

C64, C128 = 0, 1
SV_EINVAL = -1


@pytest.fixture(scope="module")
def sv():
    from paper_2512_23183_amd import sv as svmod
    return svmod


def _check(got, want, dtype, G):
    got = got.astype(np.complex128)
    if dtype == C128:
        assert np.max(np.abs(got - want)) <= 1e-12
    else:
        rel = np.linalg.norm(got - want) / np.linalg.norm(want)
        assert rel <= 1e-5 * max(1.0, math.sqrt(G / 500.0)), rel


def _both(ctx, n, dtype, circuit, params, psi0):
    out = []
    for noalloc in (True, False):
        st = ctx.alloc(n, dtype)
        st.set_amplitudes(psi0)
        if noalloc:
            st.apply_noalloc(circuit, params)
        else:
            st.apply(circuit, params)
        out.append(st.get_amplitudes())
        st.free()
    return out


@pytest.mark.parametrize("dtype", [C64, C128])
def test_noalloc_apply_matches_apply_twice_second_smaller(sv, dtype):
    big = I.deep_random_circuit(18, 10, 21)           # 270 gates on 18 qubits
    small = I.hea_circuit(9, 2)                        # 53 gates on 9 qubits
    small_params = I.uniform_params(small.n_params, 22)
    psi_big = I.gaussian_state(18, 23)
    psi_small = I.gaussian_state(9, 24)
    with sv.Context(0) as ctx:
        a_na, a_ref = _both(ctx, 18, dtype, big, None, psi_big)
        b_na, b_ref = _both(ctx, 9, dtype, small, small_params, psi_small)
    assert np.array_equal(a_na, a_ref)
    assert np.array_equal(b_na, b_ref)
    _check(a_na, oracle.run_circuit(big, psi=psi_big), dtype, len(big.gates))
    _check(b_na, oracle.run_circuit(small, small_params, psi=psi_small), dtype, len(small.gates))


def test_noalloc_refuses_plans_beyond_the_block(sv):
    n = 10
    rng = np.random.default_rng(31)
    b = I.CircuitBuilder(n)
    for _ in range(20000):
        q0, q1 = (int(v) for v in rng.choice(n, 2, replace=False))
        m = np.linalg.qr(rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4)))[0]
        b.add_matrix([q0, q1], m)
    huge = b.build(0)
    psi = I.gaussian_state(n, 32)
    with sv.Context(0) as ctx:
        st = ctx.alloc(n, C128)
        st.set_amplitudes(psi)
        with pytest.raises(sv.SvError) as ei:
            st.apply_noalloc(huge)
        assert ei.value.code == SV_EINVAL
        assert np.array_equal(st.get_amplitudes(), psi)   # nothing ran
        # the entry point stays usable after the refusal
        small = I.hea_circuit(n, 1)
        p = I.uniform_params(small.n_params, 33)
        st.apply_noalloc(small, p)
        got = st.get_amplitudes()
        st.free()
    _check(got, oracle.run_circuit(small, p, psi=psi), C128, len(small.gates))
