"""Shared prefixes in batched gradients (through the C ABI): the circuits of
a parameter-shift batch differ from the unshifted one in a single op, so the
batch executor gives each shifted circuit a copy of the unshifted state at
the pass that holds its shifted op instead of recomputing the passes before
it.  That copy is the state the circuit would have computed itself, so the
batched gradient must equal, bitwise, the same circuits run one at a time
through the pass executor (which shares nothing), and the oracle within the
usual tolerance (complex128 1e-10, complex64 1e-5).
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


# 15-16 qubits: several tile passes per circuit, so shifted ops sit in
# different passes
@pytest.mark.parametrize("n,layers,dtype", [(15, 3, C64), (16, 2, C128)])
def test_shared_prefix_gradient_equals_one_at_a_time(sv, n, layers, dtype):
    c = I.hea_circuit(n, layers)
    ham = I.random_2local(n, 25, 17)
    params = I.uniform_params(c.n_params, 23)
    with sv.Context(0) as ctx:
        ctx.profile_reset()
        ctx.profile(True)
        e_b, g_b = ctx.param_shift_grad(c, params, ham, dtype)
        share_ms, share_launches, _ = ctx.profile_get("share")
        ctx.profile(False)
        e_s, g_s = ctx.param_shift_grad(c, params, ham, dtype, flags=sv.FLAG_SEQUENTIAL)
    assert share_launches > 0  # some circuits did join late
    assert e_b == e_s
    assert np.array_equal(g_b, g_s), np.max(np.abs(g_b - g_s))
    e_ref, g_ref = oracle.param_shift(c, params, ham)
    tol = 1e-10 if dtype == C128 else 1e-5
    assert abs(e_b - e_ref) <= tol
    assert np.max(np.abs(g_b - g_ref)) <= tol


def test_shared_prefix_with_controlled_rotations(sv):
    # four-term rule circuits (CRY) next to two-term ones, 14 qubits complex128
    n = 14
    b = I.CircuitBuilder(n)
    k = 0
    for q in range(n):
        b.add(I.RY, [q], params=[k])
        k += 1
    for q in range(0, n - 1, 2):
        b.add(I.CRY, [q, q + 1], params=[k])
        k += 1
    for q in range(n):
        b.add(I.RZ, [q], params=[k])
        k += 1
    c = b.build(k)
    ham = I.random_2local(n, 15, 5)
    params = I.uniform_params(c.n_params, 6)
    with sv.Context(0) as ctx:
        e_b, g_b = ctx.param_shift_grad(c, params, ham, C128)
        e_s, g_s = ctx.param_shift_grad(c, params, ham, C128, flags=sv.FLAG_SEQUENTIAL)
    assert e_b == e_s and np.array_equal(g_b, g_s)
    e_ref, g_ref = oracle.param_shift(c, params, ham)
    assert abs(e_b - e_ref) <= 1e-10
    assert np.max(np.abs(g_b - g_ref)) <= 1e-10


def test_shared_prefix_over_several_slab_chunks(sv):
    # 24 qubits complex64: 193 circuits of 128 MiB exceed one 16 GiB slab, so
    # the batch runs in two chunks (the unshifted circuit, and with it the
    # prefix sharing, in the first); bitwise equal to one circuit at a time,
    # and the energy against the oracle
    n = 24
    c = I.hea_circuit(n, 2)
    ham = I.random_2local(n, 20, 29)
    params = I.uniform_params(c.n_params, 31)
    assert 2 * c.n_params + 1 > (16 << 30) // (8 << n)
    with sv.Context(0) as ctx:
        e_b, g_b = ctx.param_shift_grad(c, params, ham, C64)
        e_s, g_s = ctx.param_shift_grad(c, params, ham, C64, flags=sv.FLAG_SEQUENTIAL)
    assert e_b == e_s
    assert np.array_equal(g_b, g_s), np.max(np.abs(g_b - g_s))
    assert abs(e_b - oracle.circuit_energy(c, params, ham)) <= 1e-5
