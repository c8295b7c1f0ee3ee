"""Handle lifetimes and error reporting on the device (through the C ABI).

  * sv_shutdown refuses (SV_EBUSY, nothing released) while a state or a
    queue made on the context is alive; the Python Context releases its live
    states and queues before shutting down, after which those objects are
    closed handles (no use of freed memory from a later free or __del__).
  * Fault injection (SV_FAULT_ALLOC=N, read at context creation): the
    context's N-th device allocation fails.  Whichever call makes it returns
    SV_ENOMEM, the context stays usable (the same call succeeds when
    repeated, with the results of a clean run), and closing it returns the
    device memory it took.  In the serving queue, a request whose tick meets
    the failure completes with SV_ENOMEM instead of leaving its waiter
    blocked, and the next request is served normally.
The paper's explicit-error stance (App. D, "Error Reporting") is what these
check on the library's side: a failure is a status, never a crash, hang or
silent wrong value.
"""
import gc

import numpy as np
import pytest

import oracle
from paper_2512_23183_amd import inputs as I
from paper_2512_23183_amd.sv import SvError

pytestmark = pytest.mark.gpu

C64, C128 = 0, 1
SV_ENOMEM, SV_EBUSY = -2, -4


@pytest.fixture(scope="module")
def sv():
    from paper_2512_23183_amd import sv as svmod
    return svmod


def test_shutdown_refused_while_state_or_queue_alive(sv):
    ctx = sv.Context(0)
    st = ctx.alloc(6, C64)
    q = ctx.queue(1 << 26)
    assert sv.lib().sv_shutdown(ctx.h) == SV_EBUSY
    st.free()
    assert sv.lib().sv_shutdown(ctx.h) == SV_EBUSY  # the queue is still alive
    q.close()
    assert sv.lib().sv_shutdown(ctx.h) == 0
    ctx.h = None


def test_context_close_releases_live_handles(sv):
    ctx = sv.Context(0)
    st = ctx.alloc(8, C128)
    c = I.hea_circuit(8, 1)
    st.apply(c, I.uniform_params(c.n_params, 3))
    q = ctx.queue(1 << 26)
    ctx.close()
    assert st.h is None and q.h is None
    st.free()   # no-ops on released handles
    q.close()
    del st, q
    gc.collect()
    with pytest.raises(sv.SvError):
        ctx.alloc(4, C64)


def _workload():
    c = I.hea_circuit(14, 2)
    params = I.uniform_params(c.n_params, 9)
    ham = I.random_2local(14, 30, 9)
    return c, params, ham


def _steps(ctx, c, params, ham):
    """Each step returns its result; the context's allocations happen in
    these calls (state, plan and term uploads, batch buffers)."""
    box = {}

    def alloc():
        box["st"] = ctx.alloc(14, C64)
        return None

    def apply():
        box["st"].reset()
        box["st"].apply(c, params)
        return box["st"].get_amplitudes()

    def energy():
        return box["st"].expectation(ham)

    def grad():
        return ctx.param_shift_grad(c, params, ham, C64)

    return box, [("alloc", alloc), ("apply", apply), ("energy", energy), ("grad", grad)]


def _run_all(ctx, c, params, ham):
    box, steps = _steps(ctx, c, params, ham)
    out, failed = {}, []
    for name, f in steps:
        try:
            out[name] = f()
        except SvError as e:
            assert e.code == SV_ENOMEM, e
            failed.append(name)
            out[name] = f()  # the same call again, past the injected fault
    if "st" in box:
        box["st"].free()
    return out, failed


def test_fault_injected_allocations_report_enomem_and_recover(sv, monkeypatch):
    import torch
    c, params, ham = _workload()
    monkeypatch.delenv("SV_FAULT_ALLOC", raising=False)
    with sv.Context(0) as ctx:
        clean, failed = _run_all(ctx, c, params, ham)
    assert not failed
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    hit = 0
    for k in range(1, 9):
        monkeypatch.setenv("SV_FAULT_ALLOC", str(k))
        ctx = sv.Context(0)
        try:
            out, failed = _run_all(ctx, c, params, ham)
        finally:
            ctx.close()
        assert len(failed) <= 1, failed
        hit += len(failed)
        assert np.array_equal(out["apply"], clean["apply"])
        assert out["energy"] == clean["energy"]
        assert out["grad"][0] == clean["grad"][0] and np.array_equal(out["grad"][1], clean["grad"][1])
    monkeypatch.delenv("SV_FAULT_ALLOC")
    assert hit >= 3, hit  # the state, plan / term buffers and batch buffers
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] >= free0 - (2 << 20)


def test_queue_request_meeting_a_failed_allocation_completes_with_enomem(sv, monkeypatch):
    c, params, ham = _workload()
    e_ref, g_ref = oracle.param_shift(c, params, ham)
    # allocation 1 of the queue is its energy pool; 2 is the first buffer of
    # its first tick
    monkeypatch.setenv("SV_FAULT_ALLOC", "2")
    ctx = sv.Context(0)
    monkeypatch.delenv("SV_FAULT_ALLOC")
    try:
        q = ctx.queue(1 << 30)
        t = q.submit(c, params, ham, True, C64)
        with pytest.raises(sv.SvError) as ei:
            q.wait(t, 60000)
        assert ei.value.code == SV_ENOMEM
        t = q.submit(c, params, ham, True, C64)
        e, g, _ = q.wait(t, 60000)
        assert abs(e - e_ref) <= 1e-5 and np.max(np.abs(g - g_ref)) <= 1e-5
        st = q.stats()
        assert st["failed"] == 1 and st["completed"] == 1
        q.close()
    finally:
        ctx.close()
