"""Batch graphs (through the C ABI): a gradient or batch of energies whose
launches are recorded and replayed as one hipGraph gives bitwise the results
of the same batch launched kernel by kernel, on every call of a sequence
with other work and synchronisations on the same stream in between, and the
executable graph is reused while the batch keeps its shape.  One call per
case is also checked against the FP64 oracle (energies and gradients:
complex128 <= 1e-10, complex64 <= 1e-5 absolute).
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


# (qubits, layers, dtype): 8 qubits run in the one-launch small-circuit
# kernel, 15 qubits in the slab passes + batched expectation
@pytest.mark.parametrize("n,layers,dtype", [(8, 2, C128), (15, 1, C64), (15, 1, C128)])
def test_gradient_graph_replays_match_direct_launches(sv, n, layers, dtype):
    c = I.hea_circuit(n, layers)
    ham = I.random_2local(n, 30, 11)
    tol = 1e-10 if dtype == C128 else 1e-5
    with sv.Context(0, graph_batch=1) as g, sv.Context(0, graph_batch=-1) as d:
        other = g.alloc(n, dtype)
        for it in range(4):
            params = I.uniform_params(c.n_params, 100 + it)
            e_g, g_g = g.param_shift_grad(c, params, ham, dtype)
            # other work on the graph context's stream between replays
            other.reset()
            other.apply(c, params)
            other.qft()
            _ = other.norm2()
            e_d, g_d = d.param_shift_grad(c, params, ham, dtype)
            assert e_g == e_d, (it, e_g, e_d)
            assert np.array_equal(g_g, g_d), (it, np.max(np.abs(g_g - g_d)))
            if it == 0:
                e_ref, g_ref = oracle.param_shift(c, params, ham)
                assert abs(e_g - e_ref) <= tol
                assert np.max(np.abs(g_g - g_ref)) <= tol
        other.free()
        launches, inst = g.graph_stats()
        assert launches == 4
        assert inst == 1  # same shape every call: updated in place
        assert d.graph_stats() == (0, 0)


def test_batch_energies_graph_mixed_groups_and_shapes(sv):
    # small and large circuits, several (circuit, Hamiltonian) groups of
    # large ones; then a batch of another shape (new instantiation), then
    # the first shape again
    ns = [3, 9, 14, 14, 16]
    circs, prms, hams = [], [], []
    for i, n in enumerate(ns):
        c = I.hea_circuit(n, 1 + i % 2)
        circs.append(c)
        prms.append(I.uniform_params(c.n_params, 200 + i))
        hams.append(I.random_2local(n, 20, 300 + i))
    refs = np.array([oracle.circuit_energy(c, p, h) for c, p, h in zip(circs, prms, hams)])
    with sv.Context(0) as g, sv.Context(0, graph_batch=-1) as d:
        for dtype, tol in ((C64, 1e-5), (C128, 1e-10)):
            e1 = g.batch_energies(circs, prms, hams, dtype)
            assert np.max(np.abs(e1 - refs)) <= tol
            e2 = g.batch_energies(circs[:2], prms[:2], hams[:2], dtype)
            e3 = g.batch_energies(circs, prms, hams, dtype)
            assert np.array_equal(e1, e3)
            assert np.array_equal(e1, d.batch_energies(circs, prms, hams, dtype))
            assert np.array_equal(e2, d.batch_energies(circs[:2], prms[:2], hams[:2], dtype))
        launches, inst = g.graph_stats()
        assert launches == 6
        assert 2 <= inst <= 6


def test_graph_update_with_changed_arguments(sv):
    # gradients of the same launch shape (small-circuit kernel, counter
    # clear, combination) but different sizes: the executable graph is
    # updated with new arguments (qubit count, LDS size, circuit count,
    # possibly new buffers) instead of re-instantiated; every result must
    # equal the direct launches
    with sv.Context(0) as g, sv.Context(0, graph_batch=-1) as d:
        for n, layers, dtype in ((6, 1, C128), (9, 2, C128), (7, 3, C128), (9, 2, C64), (11, 1, C64)):
            c = I.hea_circuit(n, layers)
            ham = I.random_2local(n, 12, 40 + n)
            params = I.uniform_params(c.n_params, 50 + n)
            e_g, g_g = g.param_shift_grad(c, params, ham, dtype)
            e_d, g_d = d.param_shift_grad(c, params, ham, dtype)
            assert e_g == e_d and np.array_equal(g_g, g_d), (n, layers, dtype)
        launches, inst = g.graph_stats()
        assert launches == 5
        assert inst <= 3  # one per dtype at most, plus a possible change of shape
