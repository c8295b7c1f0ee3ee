"""ctypes binding of the C ABI in include/sv.h (argument marshalling only).

Every computation runs in libsv.so's HIP kernels.  Importing this module
fails loudly if the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import weakref
from typing import List, Optional, Sequence, Tuple

import numpy as np

from .inputs import GATE_DTYPE, Circuit, PauliSum

_HERE = os.path.dirname(os.path.abspath(__file__))
# SV_LIBRARY names another build of the same library (the sanitizer build
# of the host code, for CPU checks); by default the in-tree libsv.so
LIB_PATH = os.environ.get("SV_LIBRARY") or os.path.join(_HERE, "libsv.so")

C64, C128 = 0, 1
FLAG_UNFUSED = 1
FLAG_SEQUENTIAL = 2

STATUS = {0: "SV_OK", -1: "SV_EINVAL", -2: "SV_ENOMEM", -3: "SV_EDEVICE",
          -4: "SV_EBUSY", -5: "SV_ENUMERIC", -6: "SV_ECANCELED",
          -7: "SV_ENODEV", -8: "SV_ETIMEDOUT"}


class SvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class _Circuit(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_params", ctypes.c_int32),
                ("gates", ctypes.c_void_p), ("n_gates", ctypes.c_size_t),
                ("mats", ctypes.c_void_p), ("n_mats", ctypes.c_size_t)]


class _PauliSum(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_terms", ctypes.c_size_t),
                ("coeffs", ctypes.c_void_p), ("paulis", ctypes.c_void_p)]


class _Config(ctypes.Structure):
    _fields_ = [("tile_bits_c64", ctypes.c_int32), ("tile_bits_c128", ctypes.c_int32),
                ("expect_bits_c64", ctypes.c_int32), ("expect_bits_c128", ctypes.c_int32),
                ("perm_bits_c64", ctypes.c_int32), ("perm_bits_c128", ctypes.c_int32),
                ("dense_fuse", ctypes.c_int32), ("graph_batch", ctypes.c_int32),
                ("tile_bits_layers_c64", ctypes.c_int32), ("tile_bits_layers_c128", ctypes.c_int32)]


class _PlanStats(ctypes.Structure):
    _fields_ = [("tile_passes", ctypes.c_int32), ("perm_passes", ctypes.c_int32),
                ("sweep_passes", ctypes.c_int32), ("stages", ctypes.c_int32), ("ops", ctypes.c_int32),
                ("tile_passes_by_engine", ctypes.c_int32 * 5), ("dense_blocks", ctypes.c_int32),
                ("diagonal_tables", ctypes.c_int32),
                ("min_pass_scale", ctypes.c_double), ("max_pass_scale", ctypes.c_double)]


class _Request(ctypes.Structure):
    _fields_ = [("want_grad", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("circuit", _Circuit), ("params", ctypes.c_void_p),
                ("n_params", ctypes.c_size_t), ("ham", _PauliSum)]


class _QStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in
                ("submitted", "completed", "failed", "cancelled", "launches",
                 "circuits_run", "peak_bytes")]


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load libsv.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build()")
        # PyTorch ships its own HIP runtime under the same soname.  Loading it
        # first lets libsv bind to that one runtime, so torch streams and
        # device pointers are valid handles for libsv too.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "sv_init": [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_Config)],
            "sv_shutdown": [_vp],
            "sv_set_stream": [_vp, _vp],
            "sv_synchronize": [_vp],
            "sv_alloc": [_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)],
            "sv_wrap": [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)],
            "sv_free": [_vp],
            "sv_reset": [_vp],
            "sv_state_info": [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                              ctypes.POINTER(_vp)],
            "sv_set_amplitudes": [_vp, _vp, ctypes.c_size_t],
            "sv_get_amplitudes": [_vp, _vp, ctypes.c_size_t],
            "sv_apply_circuit": [_vp, ctypes.POINTER(_Circuit), _dp, ctypes.c_size_t],
            "sv_apply_circuit_ex": [_vp, ctypes.POINTER(_Circuit), _dp, ctypes.c_size_t,
                                    ctypes.c_uint32],
            "sv_apply_circuit_noalloc": [_vp, ctypes.POINTER(_Circuit), _dp, ctypes.c_size_t],
            "sv_plan_info": [ctypes.POINTER(_Circuit), _dp, ctypes.c_size_t, ctypes.c_int,
                             ctypes.POINTER(_Config), ctypes.POINTER(_PlanStats)],
            "sv_psr_info": [ctypes.POINTER(_Circuit), _dp, ctypes.c_size_t, ctypes.POINTER(_PauliSum),
                            ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int32)],
            "sv_plan_dump": [ctypes.POINTER(_Circuit), _dp, ctypes.c_size_t, ctypes.c_int,
                             ctypes.POINTER(_Config), ctypes.c_char_p, ctypes.c_size_t,
                             ctypes.POINTER(ctypes.c_size_t)],
            "sv_qft": [_vp],
            "sv_qft_ex": [_vp, ctypes.c_uint32],
            "sv_norm2": [_vp, _dp],
            "sv_normalize": [_vp],
            "sv_expectation": [_vp, ctypes.POINTER(_PauliSum), _dp, _dp],
            "sv_param_shift_grad": [_vp, ctypes.c_int, ctypes.POINTER(_Circuit), _dp,
                                    ctypes.c_size_t, ctypes.POINTER(_PauliSum), _dp, _dp],
            "sv_param_shift_grad_ex": [_vp, ctypes.c_int, ctypes.POINTER(_Circuit), _dp,
                                       ctypes.c_size_t, ctypes.POINTER(_PauliSum),
                                       ctypes.c_uint32, _dp, _dp],
            "sv_batch_energies": [_vp, ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(_Circuit),
                                  ctypes.POINTER(_dp), ctypes.POINTER(_PauliSum), _dp],
            "sv_queue_create": [_vp, ctypes.c_size_t, ctypes.POINTER(_vp)],
            "sv_queue_submit": [_vp, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_uint64)],
            "sv_queue_wait": [_vp, ctypes.c_uint64, ctypes.c_int, _dp, _dp, ctypes.c_size_t],
            "sv_queue_wait_timed": [_vp, ctypes.c_uint64, ctypes.c_int, _dp, _dp,
                                    ctypes.c_size_t, _dp],
            "sv_queue_cancel": [_vp, ctypes.c_uint64],
            "sv_queue_set_tick_budget": [_vp, ctypes.c_double],
            "sv_queue_get_stats": [_vp, ctypes.POINTER(_QStats)],
            "sv_queue_destroy": [_vp],
            "sv_check_circuit": [ctypes.POINTER(_Circuit), _dp, ctypes.c_size_t],
            "sv_check_pauli_sum": [ctypes.POINTER(_PauliSum), ctypes.c_int],
            "sv_profile_enable": [_vp, ctypes.c_int],
            "sv_profile_get": [_vp, ctypes.c_char_p, _dp, ctypes.POINTER(ctypes.c_uint64), _dp],
            "sv_profile_reset": [_vp],
            "sv_autotune": [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_char_p, ctypes.POINTER(_Config)],
            "sv_graph_stats": [_vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)],
            "sv_vqe_adam": [_vp, ctypes.c_int, ctypes.POINTER(_Circuit), _dp, ctypes.c_size_t,
                            ctypes.POINTER(_PauliSum), ctypes.c_double, ctypes.c_int, ctypes.c_double, _dp,
                            ctypes.POINTER(ctypes.c_int)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.sv_last_error.restype = ctypes.c_char_p
        L.sv_last_error.argtypes = []
        L.sv_version.restype = ctypes.c_char_p
        L.sv_version.argtypes = []
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise SvError(rc, lib().sv_last_error().decode(errors="replace"))


def _dptr(a: Optional[np.ndarray]):
    if a is None or a.size == 0:
        return ctypes.cast(None, _dp)
    return a.ctypes.data_as(_dp)


class _CircArgs:
    """Keeps the numpy buffers of a Circuit alive while the C struct is used."""

    def __init__(self, circuit: Circuit, params=None):
        self.gates = np.ascontiguousarray(circuit.gates, dtype=GATE_DTYPE)
        self.mats = np.ascontiguousarray(circuit.mats, dtype=np.float64)
        self.params = np.ascontiguousarray(
            np.zeros(0) if params is None else params, dtype=np.float64)
        self.c = _Circuit(circuit.n, circuit.n_params,
                          self.gates.ctypes.data if self.gates.size else None,
                          self.gates.shape[0],
                          self.mats.ctypes.data if self.mats.size else None,
                          self.mats.shape[0])


class _HamArgs:
    def __init__(self, ham: PauliSum):
        self.coeffs = np.ascontiguousarray(ham.coeffs, dtype=np.float64)
        self.paulis = np.ascontiguousarray(ham.paulis, dtype=np.uint8)
        self.h = _PauliSum(ham.n, self.coeffs.shape[0],
                           self.coeffs.ctypes.data if self.coeffs.size else None,
                           self.paulis.ctypes.data if self.paulis.size else None)


def version() -> str:
    return lib().sv_version().decode()


def check_circuit(circuit: Circuit, params=None) -> None:
    a = _CircArgs(circuit, params)
    _check(lib().sv_check_circuit(ctypes.byref(a.c), _dptr(a.params), a.params.size))


def check_pauli_sum(ham: PauliSum, n: int) -> None:
    h = _HamArgs(ham)
    _check(lib().sv_check_pauli_sum(ctypes.byref(h.h), n))


def _config(**widths) -> "_Config":
    names = [k for k, _ in _Config._fields_]
    for k in widths:
        if k not in names:
            raise TypeError(f"unknown config field {k}")
    return _Config(*[int(widths.get(k, 0)) for k in names])


def plan_info(circuit: Circuit, params=None, dtype: int = C64, **widths) -> dict:
    """sv_plan_info: what the fused apply of this circuit would run (host
    only, no device): passes, stages, ops per engine."""
    a = _CircArgs(circuit, params)
    cfg = _config(**widths)
    out = _PlanStats()
    _check(lib().sv_plan_info(ctypes.byref(a.c), _dptr(a.params), a.params.size, dtype,
                              ctypes.byref(cfg), ctypes.byref(out)))
    d = {k: getattr(out, k) for k, _ in _PlanStats._fields_}
    d["tile_passes_by_engine"] = list(out.tile_passes_by_engine)
    return d


def psr_info(circuit: Circuit, params, ham: PauliSum) -> Tuple[int, np.ndarray]:
    """sv_psr_info: (circuits of the gradient batch, shifted circuits per
    parameter) -- host only."""
    a, h = _CircArgs(circuit, params), _HamArgs(ham)
    nc = ctypes.c_size_t()
    sh = np.zeros(max(a.params.size, 1), dtype=np.int32)
    _check(lib().sv_psr_info(ctypes.byref(a.c), _dptr(a.params), a.params.size, ctypes.byref(h.h),
                             ctypes.byref(nc), sh.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return nc.value, sh[:a.params.size].copy()


def plan_dump(circuit: Circuit, params=None, dtype: int = C64, **widths) -> str:
    """sv_plan_dump: text listing of the plan (host only)."""
    a = _CircArgs(circuit, params)
    cfg = _config(**widths)
    need = ctypes.c_size_t()
    _check(lib().sv_plan_dump(ctypes.byref(a.c), _dptr(a.params), a.params.size, dtype,
                              ctypes.byref(cfg), None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(need.value)
    _check(lib().sv_plan_dump(ctypes.byref(a.c), _dptr(a.params), a.params.size, dtype,
                              ctypes.byref(cfg), buf, need.value, None))
    return buf.value.decode()


def _np_dtype(dtype: int):
    return np.complex64 if dtype == C64 else np.complex128


class Context:
    def __init__(self, device: int = 0, tile_bits_c64: int = 0, tile_bits_c128: int = 0,
                 expect_bits_c64: int = 0, expect_bits_c128: int = 0,
                 perm_bits_c64: int = 0, perm_bits_c128: int = 0, dense_fuse: int = 0,
                 graph_batch: int = 0, tile_bits_layers_c64: int = 0, tile_bits_layers_c128: int = 0):
        cfg = _Config(tile_bits_c64, tile_bits_c128, expect_bits_c64, expect_bits_c128,
                      perm_bits_c64, perm_bits_c128, dense_fuse, graph_batch,
                      tile_bits_layers_c64, tile_bits_layers_c128)
        h = _vp()
        _check(lib().sv_init(ctypes.byref(h), device, ctypes.byref(cfg)))
        self.h = h
        # states and queues made on this context; close() releases those
        # still alive first (the library refuses to shut down under them)
        self._owned = weakref.WeakSet()

    def close(self):
        if self.h:
            for obj in list(self._owned):
                obj._release()
            _check(lib().sv_shutdown(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_stream(self, hip_stream_ptr: int = 0):
        _check(lib().sv_set_stream(self.h, hip_stream_ptr or None))

    def synchronize(self):
        _check(lib().sv_synchronize(self.h))

    def autotune(self, dtype: int, n_qubits: int, cache_path: Optional[str] = None) -> dict:
        """Time candidate tile widths for dtype at n_qubits and keep the
        fastest in this context; returns every width of the context."""
        cfg = _Config()
        _check(lib().sv_autotune(self.h, dtype, n_qubits,
                                 cache_path.encode() if cache_path else None, ctypes.byref(cfg)))
        return {k: getattr(cfg, k) for k, _ in _Config._fields_ if k != "graph_batch"}

    def graph_stats(self) -> Tuple[int, int]:
        """(hipGraph launches, instantiations) of this context's batches."""
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().sv_graph_stats(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def profile(self, on: bool = True):
        _check(lib().sv_profile_enable(self.h, 1 if on else 0))

    def profile_reset(self):
        _check(lib().sv_profile_reset(self.h))

    def profile_get(self, name: str) -> Tuple[float, int, float]:
        ms, n, b = ctypes.c_double(), ctypes.c_uint64(), ctypes.c_double()
        _check(lib().sv_profile_get(self.h, name.encode(), ctypes.byref(ms),
                                    ctypes.byref(n), ctypes.byref(b)))
        return ms.value, n.value, b.value

    def alloc(self, n: int, dtype: int = C64) -> "State":
        return State(self, n, dtype)

    def param_shift_grad(self, circuit: Circuit, params, ham: PauliSum,
                         dtype: int = C64, flags: int = 0) -> Tuple[float, np.ndarray]:
        a, h = _CircArgs(circuit, params), _HamArgs(ham)
        e = ctypes.c_double()
        g = np.zeros(max(a.params.size, 1))
        _check(lib().sv_param_shift_grad_ex(self.h, dtype, ctypes.byref(a.c), _dptr(a.params),
                                            a.params.size, ctypes.byref(h.h), flags,
                                            ctypes.byref(e), _dptr(g)))
        return e.value, g[:a.params.size].copy()

    def vqe_adam(self, circuit: Circuit, params, ham: PauliSum, dtype: int = C64, lr: float = 1e-2,
                 max_iters: int = 350, tol: float = 1e-7) -> Tuple[np.ndarray, np.ndarray]:
        """Adam on the energy with batched parameter-shift gradients; returns
        (parameters of the last evaluation, energies of every iteration)."""
        a, h = _CircArgs(circuit, params), _HamArgs(ham)
        theta = np.array(a.params, dtype=np.float64, copy=True)
        energies = np.zeros(max(max_iters, 1))
        it = ctypes.c_int()
        _check(lib().sv_vqe_adam(self.h, dtype, ctypes.byref(a.c), _dptr(theta), theta.size,
                                 ctypes.byref(h.h), lr, max_iters, tol, _dptr(energies), ctypes.byref(it)))
        return theta, energies[:it.value]

    def batch_energies(self, circuits: Sequence[Circuit], params: Sequence,
                       hams: Sequence[PauliSum], dtype: int = C64) -> np.ndarray:
        cas = [_CircArgs(c, p) for c, p in zip(circuits, params)]
        has = [_HamArgs(h) for h in hams]
        n = len(cas)
        carr = (_Circuit * max(n, 1))(*[a.c for a in cas])
        parr = (_dp * max(n, 1))(*[_dptr(a.params) for a in cas])
        harr = (_PauliSum * max(n, 1))(*[h.h for h in has])
        out = np.zeros(max(n, 1))
        _check(lib().sv_batch_energies(self.h, dtype, n, carr, parr, harr, _dptr(out)))
        return out[:n].copy()

    def queue(self, budget_bytes: int) -> "Queue":
        return Queue(self, budget_bytes)


class State:
    def __init__(self, ctx: Context, n: int, dtype: int = C64, _wrap_ptr: int = 0):
        self.ctx, self.n, self.dtype = ctx, n, dtype
        h = _vp()
        if not ctx.h:
            raise SvError(-1, "context is closed")
        if _wrap_ptr:
            _check(lib().sv_wrap(ctx.h, _wrap_ptr, n, dtype, ctypes.byref(h)))
        else:
            _check(lib().sv_alloc(ctx.h, n, dtype, ctypes.byref(h)))
        self.h = h
        ctx._owned.add(self)

    @staticmethod
    def from_torch(ctx: Context, tensor) -> "State":
        """Adopt a contiguous complex64/complex128 torch tensor of 2^n
        elements on the context's device as the state (torch keeps it)."""
        import torch
        assert tensor.is_contiguous() and tensor.dtype in (torch.complex64, torch.complex128)
        n = int(tensor.numel()).bit_length() - 1
        assert tensor.numel() == 1 << n
        dt = C64 if tensor.dtype == torch.complex64 else C128
        st = State(ctx, n, dt, _wrap_ptr=tensor.data_ptr())
        st._keep = tensor
        return st

    def free(self):
        if self.h:
            _check(lib().sv_free(self.h))
            self.h = None

    def _release(self):
        # the context is closing: free the handle now; later calls on this
        # object see a closed state
        self.free()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def reset(self):
        _check(lib().sv_reset(self.h))

    def set_amplitudes(self, psi: np.ndarray):
        a = np.ascontiguousarray(psi, dtype=_np_dtype(self.dtype))
        assert a.size == 1 << self.n
        _check(lib().sv_set_amplitudes(self.h, a.ctypes.data, a.size))

    def get_amplitudes(self) -> np.ndarray:
        a = np.empty(1 << self.n, dtype=_np_dtype(self.dtype))
        _check(lib().sv_get_amplitudes(self.h, a.ctypes.data, a.size))
        return a

    def apply(self, circuit: Circuit, params=None, flags: int = 0):
        a = _CircArgs(circuit, params)
        _check(lib().sv_apply_circuit_ex(self.h, ctypes.byref(a.c), _dptr(a.params),
                                         a.params.size, flags))

    def apply_noalloc(self, circuit: Circuit, params=None):
        """sv_apply_circuit_noalloc: the fused apply with its plan tables in
        the device's preallocated block (no device allocation)."""
        a = _CircArgs(circuit, params)
        _check(lib().sv_apply_circuit_noalloc(self.h, ctypes.byref(a.c), _dptr(a.params), a.params.size))

    def qft(self, flags: int = 0):
        _check(lib().sv_qft_ex(self.h, flags))

    def norm2(self) -> float:
        v = ctypes.c_double()
        _check(lib().sv_norm2(self.h, ctypes.byref(v)))
        return v.value

    def normalize(self):
        _check(lib().sv_normalize(self.h))

    def expectation(self, ham: PauliSum, terms: bool = False):
        h = _HamArgs(ham)
        e = ctypes.c_double()
        tv = np.zeros(max(ham.n_terms, 1))
        _check(lib().sv_expectation(self.h, ctypes.byref(h.h), ctypes.byref(e),
                                    _dptr(tv) if terms else ctypes.cast(None, _dp)))
        return (e.value, tv[:ham.n_terms].copy()) if terms else e.value


class Queue:
    def __init__(self, ctx: Context, budget_bytes: int):
        h = _vp()
        if not ctx.h:
            raise SvError(-1, "context is closed")
        _check(lib().sv_queue_create(ctx.h, budget_bytes, ctypes.byref(h)))
        self.h = h
        self._n_params = {}
        ctx._owned.add(self)

    def _release(self):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, circuit: Circuit, params, ham: PauliSum, want_grad: bool,
               dtype: int = C64) -> int:
        a, hh = _CircArgs(circuit, params), _HamArgs(ham)
        req = _Request(1 if want_grad else 0, dtype, a.c,
                       a.params.ctypes.data if a.params.size else None, a.params.size, hh.h)
        t = ctypes.c_uint64()
        _check(lib().sv_queue_submit(self.h, ctypes.byref(req), ctypes.byref(t)))
        self._n_params[t.value] = a.params.size if want_grad else 0
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        """-> (energy, gradient or None, latency seconds)."""
        npar = self._n_params.get(ticket, 0)
        e, lat = ctypes.c_double(), ctypes.c_double()
        g = np.zeros(max(npar, 1))
        rc = lib().sv_queue_wait_timed(self.h, ticket, timeout_ms, ctypes.byref(e), _dptr(g),
                                       g.size, ctypes.byref(lat))
        if rc != -8:
            self._n_params.pop(ticket, None)
        _check(rc)
        return e.value, (g[:npar].copy() if npar else None), lat.value

    def cancel(self, ticket: int):
        _check(lib().sv_queue_cancel(self.h, ticket))

    def set_tick_budget(self, amplitude_updates: float):
        """Bound the work of one scheduler tick (0 = no bound)."""
        _check(lib().sv_queue_set_tick_budget(self.h, float(amplitude_updates)))

    def stats(self) -> dict:
        s = _QStats()
        _check(lib().sv_queue_get_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in _QStats._fields_}

    def close(self):
        if self.h:
            _check(lib().sv_queue_destroy(self.h))
            self.h = None
