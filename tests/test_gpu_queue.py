"""Serving queue on the GPU: results match the oracle, and each request's
result is identical alone and when it shares launches with other requests
(continuous batching of mixed qubit counts)."""
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


@pytest.fixture(scope="module")
def ctx(sv):
    c = sv.Context(0)
    yield c
    c.close()


def _requests():
    return I.serving_requests(24, 11, rate_per_s=0.0, n_range=(3, 15), depth_range=(1, 3),
                              terms_range=(5, 40))


def test_queue_matches_oracle_and_is_mix_invariant(ctx, sv):
    reqs = _requests()
    # alone: one request in flight at a time
    q = ctx.queue(1 << 30)
    alone = []
    for r in reqs:
        t = q.submit(r.circuit, r.params, r.hamiltonian, r.grad, C128)
        alone.append(q.wait(t, 60000))
    q.close()
    # in the mix: everything submitted at once, small budget forces piecewise
    # admission and several shared launches
    q = ctx.queue(8 << 20)
    tickets = [q.submit(r.circuit, r.params, r.hamiltonian, r.grad, C128) for r in reqs]
    mixed = [q.wait(t, 120000) for t in tickets]
    st = q.stats()
    q.close()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    for r, a, m in zip(reqs, alone, mixed):
        assert a[0] == m[0]                      # bitwise identical energy
        if r.grad:
            np.testing.assert_array_equal(a[1], m[1])
            e_ref, g_ref = oracle.param_shift(r.circuit, r.params, r.hamiltonian)
            assert np.max(np.abs(m[1] - g_ref)) <= 1e-10
        else:
            e_ref = oracle.circuit_energy(r.circuit, r.params, r.hamiltonian)
        assert abs(m[0] - e_ref) <= 1e-10
        assert m[2] >= 0.0


def test_queue_200_request_sample_matches_oracle(ctx):
    # a seeded sample of 200 requests of the serving mix (qubit counts kept
    # at 8..10 so the oracle finishes in seconds), submitted at once to a
    # queue whose budget forces continuous batching; every result against
    # the oracle (complex128: 1e-10)
    reqs = I.serving_requests(200, 5, rate_per_s=0.0, n_range=(8, 10), depth_range=(2, 4),
                              terms_range=(20, 60))
    q = ctx.queue(8 << 20)
    tickets = [q.submit(r.circuit, r.params, r.hamiltonian, r.grad, C128) for r in reqs]
    got = [q.wait(t, 120000) for t in tickets]
    st = q.stats()
    q.close()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    for r, (e, g, _) in zip(reqs, got):
        if r.grad:
            e_ref, g_ref = oracle.param_shift(r.circuit, r.params, r.hamiltonian)
            assert np.max(np.abs(g - g_ref)) <= 1e-10, r.rid
        else:
            e_ref = oracle.circuit_energy(r.circuit, r.params, r.hamiltonian)
        assert abs(e - e_ref) <= 1e-10, r.rid


def test_queue_c64_tolerance(ctx):
    reqs = _requests()[:8]
    q = ctx.queue(1 << 30)
    tickets = [q.submit(r.circuit, r.params, r.hamiltonian, r.grad, C64) for r in reqs]
    for r, t in zip(reqs, tickets):
        e, g, _ = q.wait(t, 60000)
        e_ref, g_ref = oracle.param_shift(r.circuit, r.params, r.hamiltonian)
        assert abs(e - e_ref) <= 1e-5
        if r.grad:
            assert np.max(np.abs(g - g_ref)) <= 1e-5
    q.close()


def test_queue_rejects_invalid_and_oversized(ctx, sv):
    q = ctx.queue(1 << 20)
    c = I.hea_circuit(4, 1)
    with pytest.raises(sv.SvError) as e:
        q.submit(c, np.zeros(3), I.xyz_chain(4), True)
    assert e.value.name == "SV_EINVAL"
    big = I.hea_circuit(20, 1)   # 8 MiB state > 1 MiB budget
    with pytest.raises(sv.SvError) as e:
        q.submit(big, I.uniform_params(big.n_params, 0), I.xyz_chain(20), False)
    assert e.value.name == "SV_EBUSY"
    q.close()


def test_queue_cancel(ctx, sv):
    q = ctx.queue(1 << 30)
    c = I.hea_circuit(12, 3)
    p = I.uniform_params(c.n_params, 1)
    ts = [q.submit(c, p, I.xyz_chain(12), True) for _ in range(6)]
    q.cancel(ts[-1])
    outcomes = []
    for t in ts:
        try:
            q.wait(t, 60000)
            outcomes.append("ok")
        except sv.SvError as e:
            outcomes.append(e.name)
    assert outcomes[0] == "ok"
    assert outcomes[-1] in ("ok", "SV_ECANCELED")
    q.close()


def test_queue_200_request_sample_matches_oracle_c64(ctx):
    # the same seeded 200-request sample at complex64, the precision the
    # serving configuration names: energies and gradients within 1e-5
    reqs = I.serving_requests(200, 5, rate_per_s=0.0, n_range=(8, 10), depth_range=(2, 4),
                              terms_range=(20, 60))
    q = ctx.queue(8 << 20)
    tickets = [q.submit(r.circuit, r.params, r.hamiltonian, r.grad, C64) for r in reqs]
    got = [q.wait(t, 120000) for t in tickets]
    st = q.stats()
    q.close()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    for r, (e, g, _) in zip(reqs, got):
        if r.grad:
            e_ref, g_ref = oracle.param_shift(r.circuit, r.params, r.hamiltonian)
            assert np.max(np.abs(g - g_ref)) <= 1e-5, r.rid
        else:
            e_ref = oracle.circuit_energy(r.circuit, r.params, r.hamiltonian)
        assert abs(e - e_ref) <= 1e-5, r.rid


def test_small_requests_overtake_a_large_gradient(ctx):
    # a 20-qubit gradient (2 x 80 + 1 circuits) admitted in pieces of a
    # bounded tick; energy requests submitted right after it complete
    # before it does, with the results they have alone
    big = I.hea_circuit(20, 2)
    bp = I.uniform_params(big.n_params, 8)
    ham = I.random_2local(20, 30, 8)
    small = [I.hea_circuit(10, 2) for _ in range(4)]
    sp = [I.uniform_params(c.n_params, 20 + i) for i, c in enumerate(small)]
    sh = I.xyz_chain(10)
    q = ctx.queue(1 << 30)
    q.set_tick_budget(2e9)
    alone = []
    for c, p in zip(small, sp):
        t = q.submit(c, p, sh, False, C64)
        alone.append(q.wait(t, 60000)[0])
    tb = q.submit(big, bp, ham, True, C64)
    ts = [q.submit(c, p, sh, False, C64) for c, p in zip(small, sp)]
    res = [q.wait(t, 60000) for t in ts]
    eb, gb, lb = q.wait(tb, 120000)
    q.close()
    for (e, _, l), a in zip(res, alone):
        assert e == a
        assert l < lb
    e_ref = oracle.circuit_energy(big, bp, ham)
    assert abs(eb - e_ref) <= 1e-5
