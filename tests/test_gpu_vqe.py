"""VQE loop on the GPU (sv_vqe_adam, through the C ABI) against the oracle's
Adam loop driven by oracle parameter-shift gradients (Sec. "Variational
Quantum Eigensolver": Adam at lr 1e-2, at most 350 iterations, tolerance
1e-7).  Energies per iteration: complex128 <= 1e-10 absolute; complex64
<= 1e-4 (gradient rounding of ~1e-6 perturbs each Adam step by at most
lr * 1e-6 / |g_i| per parameter, accumulated over the iterations).
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


@pytest.mark.parametrize("dtype,tol", [(C128, 1e-10), (C64, 1e-4)])
def test_vqe_trajectory_matches_oracle_10q_xyz_chain(sv, dtype, tol):
    n = 10
    c = I.hea_circuit(n, 4)
    ham = I.xyz_chain(n)
    p0 = I.uniform_params(c.n_params, 1)
    th_ref, e_ref = oracle.vqe_adam(c, p0, ham, max_iters=25)
    with sv.Context(0) as ctx:
        th, e = ctx.vqe_adam(c, p0, ham, dtype, max_iters=25)
        assert len(e) == len(e_ref) == 25
        assert np.max(np.abs(e - e_ref)) <= tol
        assert np.max(np.abs(th - th_ref)) <= (1e-9 if dtype == C128 else 1e-3)
        # every iteration is one gradient of the same shape: one graph
        launches, inst = ctx.graph_stats()
        assert launches == 25 and inst == 1


def test_vqe_runs_to_the_cap_below_its_start_and_above_the_ground_energy(sv):
    # the 10-qubit XYZ chain at the paper's settings; exact ground energy of the chain
    n = 10
    c = I.hea_circuit(n, 4)
    ham = I.xyz_chain(n)
    e0 = -9.161997432407
    with sv.Context(0) as ctx:
        th, e = ctx.vqe_adam(c, I.uniform_params(c.n_params, 1), ham, C128)
        assert 2 <= len(e) <= 350
        assert np.all(e >= e0 - 1e-9)
        assert e[-1] < e[0] - 5.0
        # the returned parameters are those of the last energy
        e_last, _ = ctx.param_shift_grad(c, th, ham, C128)
        assert abs(e_last - e[-1]) <= 1e-10


def test_vqe_stops_on_tolerance_and_checks_arguments(sv):
    n = 3
    c = I.hea_circuit(n, 1)
    const = I.PauliSum.from_strings(n, [(1.5, "III")])
    p0 = I.uniform_params(c.n_params, 2)
    with sv.Context(0) as ctx:
        th, e = ctx.vqe_adam(c, p0, const, C128, max_iters=50)
        assert len(e) == 2 and np.allclose(e, 1.5, atol=1e-12)
        one, e1 = ctx.vqe_adam(c, p0, const, C128, max_iters=1)
        assert len(e1) == 1 and np.array_equal(one, p0)
        for kw in ({"max_iters": 0}, {"lr": 0.0}, {"lr": float("nan")}, {"tol": -1.0}):
            with pytest.raises(sv.SvError):
                ctx.vqe_adam(c, p0, const, C128, **kw)
