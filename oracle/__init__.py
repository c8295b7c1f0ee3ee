"""Python access to the FP64 CPU oracle (``liboracle.so``, built from
``sv_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may use it; the product library never does.  The oracle
shares no code with the GPU path; both read the same seeded inputs.

Every routine works on complex128 numpy vectors of length 2^n with qubit q at
index bit n-1-q (MSB-first).
"""
from __future__ import annotations

import ctypes
import os
from typing import Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.or_apply_gate.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _ip, _dp, _dp]
        L.or_apply_gate.restype = ctypes.c_int
        L.or_zero_state.argtypes = [_dp, ctypes.c_int]
        L.or_zero_state.restype = None
        circ = [ctypes.c_int, _ip, _ip, _ip, _dp, _ip, _dp, ctypes.c_int,
                _dp, ctypes.c_int]
        L.or_run_circuit.argtypes = [_dp, ctypes.c_int] + circ
        L.or_run_circuit.restype = ctypes.c_int
        L.or_qft.argtypes = [_dp, ctypes.c_int]
        L.or_qft.restype = None
        L.or_pauli_expectation.argtypes = [_dp, ctypes.c_int, ctypes.c_char_p, _dp, _dp]
        L.or_pauli_expectation.restype = ctypes.c_int
        L.or_energy.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _dp,
                                ctypes.c_char_p, _dp, _dp]
        L.or_energy.restype = ctypes.c_int
        ham = [ctypes.c_int, _dp, ctypes.c_char_p]
        L.or_circuit_energy.argtypes = [ctypes.c_int] + circ + ham + [_dp]
        L.or_circuit_energy.restype = ctypes.c_int
        L.or_param_shift.argtypes = [ctypes.c_int] + circ + ham + [_dp, _dp]
        L.or_param_shift.restype = ctypes.c_int
        L.or_param_shift_two_term.argtypes = [ctypes.c_int] + circ + ham + [_dp]
        L.or_param_shift_two_term.restype = ctypes.c_int
        L.or_norm2.argtypes = [_dp, ctypes.c_int]
        L.or_norm2.restype = ctypes.c_double
        _lib = L
    return _lib


def _d(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _i(a: np.ndarray):
    return a.ctypes.data_as(_ip)


def _state(psi: np.ndarray) -> np.ndarray:
    psi = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    n = int(psi.size).bit_length() - 1
    assert psi.size == 1 << n
    return psi


def _nq(psi: np.ndarray) -> int:
    return int(psi.size).bit_length() - 1


class _CircArgs:
    """Flat arrays of a Circuit in the oracle's calling convention."""

    def __init__(self, circuit, params):
        g = circuit.gates
        self.G = int(g.shape[0])
        self.kinds = np.ascontiguousarray(g["kind"], dtype=np.int32)
        self.q = np.ascontiguousarray(g["q"], dtype=np.int32).reshape(-1)
        self.p = np.ascontiguousarray(g["param_idx"], dtype=np.int32).reshape(-1)
        self.a = np.ascontiguousarray(g["angle"], dtype=np.float64).reshape(-1)
        self.mi = np.ascontiguousarray(g["mat_idx"], dtype=np.int32)
        self.mats = np.ascontiguousarray(circuit.mats, dtype=np.float64).reshape(-1)
        if self.mats.size == 0:
            self.mats = np.zeros(32)
        self.n_mats = int(circuit.mats.shape[0])
        prm = np.ascontiguousarray(
            params if params is not None else np.zeros(0), dtype=np.float64)
        self.n_params = int(prm.size)
        self.params = prm if prm.size else np.zeros(1)

    def args(self):
        return [self.G, _i(self.kinds), _i(self.q), _i(self.p), _d(self.a),
                _i(self.mi), _d(self.mats), self.n_mats, _d(self.params),
                self.n_params]


class _HamArgs:
    def __init__(self, ham):
        self.T = int(ham.n_terms)
        self.c = np.ascontiguousarray(ham.coeffs, dtype=np.float64)
        if self.c.size == 0:
            self.c = np.zeros(1)
        self.s = np.ascontiguousarray(ham.paulis, dtype=np.uint8).tobytes()

    def args(self):
        return [self.T, _d(self.c), self.s]


def zero_state(n: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().or_zero_state(_d(psi), n)
    return psi


def apply_gate(psi: np.ndarray, kind: int, qubits, angles=(), mat=None) -> np.ndarray:
    """Return a copy of psi with one gate applied."""
    psi = _state(psi)
    q = np.array(list(qubits) + [0] * (3 - len(qubits)), dtype=np.int32)
    a = np.array(list(angles) + [0.0] * (3 - len(angles)), dtype=np.float64)
    m = np.zeros(32)
    if mat is not None:
        v = np.asarray(mat, dtype=np.complex128).reshape(-1)
        m[0:2 * v.size:2] = v.real
        m[1:2 * v.size:2] = v.imag
    rc = lib().or_apply_gate(_d(psi), _nq(psi), int(kind), _i(q), _d(a), _d(m))
    if rc != 0:
        raise ValueError("oracle rejected gate")
    return psi


def run_circuit(circuit, params=None, psi=None) -> np.ndarray:
    """U_L ... U_1 psi (psi defaults to |0...0>); returns a new vector."""
    psi = zero_state(circuit.n) if psi is None else _state(psi)
    ca = _CircArgs(circuit, params)
    rc = lib().or_run_circuit(_d(psi), circuit.n, *ca.args())
    if rc != 0:
        raise ValueError("oracle rejected circuit")
    return psi


def qft(psi: np.ndarray) -> np.ndarray:
    psi = _state(psi)
    lib().or_qft(_d(psi), _nq(psi))
    return psi


def pauli_expectation(psi: np.ndarray, paulis: str) -> complex:
    psi = _state(psi)
    re, im = ctypes.c_double(), ctypes.c_double()
    rc = lib().or_pauli_expectation(_d(psi), _nq(psi), paulis.encode(),
                                    ctypes.byref(re), ctypes.byref(im))
    if rc != 0:
        raise ValueError("bad Pauli string")
    return complex(re.value, im.value)


def energy(psi: np.ndarray, ham) -> Tuple[float, float]:
    """(sum_t c_t Re<P_t>, max_t |Im <P_t>|)."""
    psi = _state(psi)
    ha = _HamArgs(ham)
    e, mi = ctypes.c_double(), ctypes.c_double()
    rc = lib().or_energy(_d(psi), _nq(psi), *ha.args(), ctypes.byref(e),
                         ctypes.byref(mi))
    if rc != 0:
        raise ValueError("bad Hamiltonian")
    return e.value, mi.value


def circuit_energy(circuit, params, ham) -> float:
    ca, ha = _CircArgs(circuit, params), _HamArgs(ham)
    e = ctypes.c_double()
    rc = lib().or_circuit_energy(circuit.n, *ca.args(), *ha.args(),
                                 ctypes.byref(e))
    if rc != 0:
        raise ValueError("oracle rejected input")
    return e.value


def param_shift(circuit, params, ham) -> Tuple[float, np.ndarray]:
    """(f(theta), gradient) by the parameter-shift rule."""
    ca, ha = _CircArgs(circuit, params), _HamArgs(ham)
    e = ctypes.c_double()
    g = np.zeros(max(ca.n_params, 1))
    rc = lib().or_param_shift(circuit.n, *ca.args(), *ha.args(),
                              ctypes.byref(e), _d(g))
    if rc != 0:
        raise ValueError("oracle rejected input")
    return e.value, g[:ca.n_params].copy()


def param_shift_two_term(circuit, params, ham) -> np.ndarray:
    """The paper's literal two-term loop over every parameter."""
    ca, ha = _CircArgs(circuit, params), _HamArgs(ham)
    g = np.zeros(max(ca.n_params, 1))
    rc = lib().or_param_shift_two_term(circuit.n, *ca.args(), *ha.args(), _d(g))
    if rc != 0:
        raise ValueError("oracle rejected input")
    return g[:ca.n_params].copy()


def adam_minimise(fg, theta0, lr=1e-2, max_iters=350, tol=1e-7,
                  beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma and Ba) on a function given as fg(theta) -> (f, grad):
    first and second moment estimates with decay beta1 / beta2, divided by
    1 - beta^t (bias correction), step -lr * m_hat / (sqrt(v_hat) + eps).
    The VQE loop of Sec. "Variational Quantum Eigensolver" uses lr = 1e-2,
    at most 350 iterations and tolerance 1e-7; the stopping rule read here:
    iteration t evaluates f_t at the current theta and stops when t equals
    max_iters or |f_t - f_{t-1}| < tol, else steps.  Returns (theta of the
    last evaluation, [f_1, ..., f_T])."""
    theta = np.array(theta0, dtype=np.float64, copy=True)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    fs = []
    for t in range(1, max_iters + 1):
        f, g = fg(theta)
        fs.append(f)
        if t == max_iters or (t > 1 and abs(f - fs[-2]) < tol):
            break
        m = beta1 * m + (1.0 - beta1) * g
        v = beta2 * v + (1.0 - beta2) * g * g
        m_hat = m / (1.0 - beta1 ** t)
        v_hat = v / (1.0 - beta2 ** t)
        theta = theta - lr * m_hat / (np.sqrt(v_hat) + eps)
    return theta, np.array(fs)


def vqe_adam(circuit, params, ham, lr=1e-2, max_iters=350, tol=1e-7):
    """VQE energy minimisation: Adam driven by parameter-shift gradients."""
    return adam_minimise(lambda th: param_shift(circuit, th, ham), params, lr, max_iters, tol)


def norm2(psi: np.ndarray) -> float:
    psi = _state(psi)
    return float(lib().or_norm2(_d(psi), _nq(psi)))
