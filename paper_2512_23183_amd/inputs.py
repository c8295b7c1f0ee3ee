"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the simulation method: it only lays out
gate lists (kinds, qubit operands, parameter indices, fixed angles), Pauli
strings with coefficients, parameter vectors and random input states.  Gate
matrices, phases, expectation values and gradients are computed separately
by the GPU path and by the oracle.

Gate records use the same field layout as the C ABI's ``sv_gate`` (56 bytes):
``kind, q[3], param_idx[3], mat_idx, angle[3]``.  Qubit q is index bit n-1-q
(MSB-first, as in the paper's direct state-vector CNOT algorithm).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Gate kinds (interface numbers, identical to ``sv_gate_kind`` in sv.h).
H, X, Y, Z = 0, 1, 2, 3
RX, RY, RZ, U3 = 4, 5, 6, 7
CNOT, CZ, CP, SWAP = 8, 9, 10, 11
CRX, CRY, CRZ, CCX = 12, 13, 14, 15
RXX, RYY, RZZ = 16, 17, 18
MAT1, MAT2 = 19, 20

KIND_NAMES = {
    H: "H", X: "X", Y: "Y", Z: "Z", RX: "RX", RY: "RY", RZ: "RZ", U3: "U3",
    CNOT: "CNOT", CZ: "CZ", CP: "CP", SWAP: "SWAP", CRX: "CRX", CRY: "CRY",
    CRZ: "CRZ", CCX: "CCX", RXX: "RXX", RYY: "RYY", RZZ: "RZZ",
    MAT1: "MAT1", MAT2: "MAT2",
}
ARITY = {H: 1, X: 1, Y: 1, Z: 1, RX: 1, RY: 1, RZ: 1, U3: 1, MAT1: 1,
         CNOT: 2, CZ: 2, CP: 2, SWAP: 2, CRX: 2, CRY: 2, CRZ: 2,
         RXX: 2, RYY: 2, RZZ: 2, MAT2: 2, CCX: 3}
N_ANGLES = {RX: 1, RY: 1, RZ: 1, CP: 1, CRX: 1, CRY: 1, CRZ: 1,
            RXX: 1, RYY: 1, RZZ: 1, U3: 3}

GATE_DTYPE = np.dtype([
    ("kind", np.int32), ("q", np.int32, (3,)), ("param_idx", np.int32, (3,)),
    ("mat_idx", np.int32), ("angle", np.float64, (3,)),
], align=True)
assert GATE_DTYPE.itemsize == 56


@dataclasses.dataclass
class Circuit:
    """A gate list over ``n`` qubits, optionally parameterised.

    ``gates`` is a structured array of GATE_DTYPE.  ``mats`` holds user
    matrices, one row of 32 doubles each (row-major (re, im); a 2x2 uses the
    first 8).  ``n_params`` is the length the parameter vector must have.
    """
    n: int
    gates: np.ndarray
    mats: np.ndarray
    n_params: int = 0

    @property
    def n_gates(self) -> int:
        return int(self.gates.shape[0])


class CircuitBuilder:
    """Append-only builder of gate records (no arithmetic)."""

    def __init__(self, n: int):
        self.n = n
        self._rows: List[tuple] = []
        self._mats: List[np.ndarray] = []
        self.n_params = 0

    def add(self, kind: int, qubits: Sequence[int],
            angles: Sequence[float] = (), params: Sequence[int] = ()):
        q = list(qubits) + [-1] * (3 - len(qubits))
        a = list(angles) + [0.0] * (3 - len(angles))
        p = list(params) + [-1] * (3 - len(params))
        for pi in p:
            if pi >= 0:
                self.n_params = max(self.n_params, pi + 1)
        self._rows.append((kind, q, p, -1, a))
        return self

    def add_matrix(self, qubits: Sequence[int], mat: np.ndarray):
        mat = np.asarray(mat, dtype=np.complex128)
        k = MAT1 if len(qubits) == 1 else MAT2
        flat = np.zeros(32)
        v = mat.reshape(-1)
        flat[0:2 * v.size:2] = v.real
        flat[1:2 * v.size:2] = v.imag
        self._mats.append(flat)
        q = list(qubits) + [-1] * (3 - len(qubits))
        self._rows.append((k, q, [-1, -1, -1], len(self._mats) - 1,
                           [0.0, 0.0, 0.0]))
        return self

    def build(self, n_params: Optional[int] = None) -> Circuit:
        gates = np.zeros(len(self._rows), dtype=GATE_DTYPE)
        for i, (k, q, p, mi, a) in enumerate(self._rows):
            gates[i]["kind"] = k
            gates[i]["q"] = q
            gates[i]["param_idx"] = p
            gates[i]["mat_idx"] = mi
            gates[i]["angle"] = a
        mats = (np.stack(self._mats) if self._mats
                else np.zeros((0, 32), dtype=np.float64))
        return Circuit(self.n, gates, np.ascontiguousarray(mats),
                       self.n_params if n_params is None else n_params)


@dataclasses.dataclass
class PauliSum:
    """H = sum_t coeffs[t] * P_t; ``paulis`` is uint8 [T, n] over b'IXYZ'."""
    n: int
    coeffs: np.ndarray
    paulis: np.ndarray

    @property
    def n_terms(self) -> int:
        return int(self.coeffs.shape[0])

    def strings(self) -> List[str]:
        return [bytes(r).decode() for r in self.paulis]

    @staticmethod
    def from_strings(n: int, terms: Sequence[Tuple[float, str]]) -> "PauliSum":
        coeffs = np.array([c for c, _ in terms], dtype=np.float64)
        rows = np.zeros((len(terms), n), dtype=np.uint8)
        for t, (_, s) in enumerate(terms):
            assert len(s) == n
            rows[t] = np.frombuffer(s.encode(), dtype=np.uint8)
        return PauliSum(n, coeffs, rows)


# ---------------------------------------------------------------------------
# Workload generators
# ---------------------------------------------------------------------------

def hea_circuit(n: int, layers: int) -> Circuit:
    """Hardware-efficient ansatz: per layer RY(theta) on every qubit, RZ(theta)
    on every qubit, then the CNOT ladder q_i -> q_{i+1} for i = 0..n-2 in
    increasing i.  Parameter of RY on qubit q in layer l is 2nl+q, of RZ is
    2nl+n+q, so 2n*layers parameters, each used once.
    """
    b = CircuitBuilder(n)
    for layer in range(layers):
        for q in range(n):
            b.add(RY, [q], params=[2 * n * layer + q])
        for q in range(n):
            b.add(RZ, [q], params=[2 * n * layer + n + q])
        for i in range(n - 1):
            b.add(CNOT, [i, i + 1])
    return b.build(2 * n * layers)


def hea_ry_circuit(n: int, layers: int) -> Circuit:
    """RY-only layers followed by the linear CNOT chain (n params per layer)."""
    b = CircuitBuilder(n)
    for layer in range(layers):
        for q in range(n):
            b.add(RY, [q], params=[n * layer + q])
        for i in range(n - 1):
            b.add(CNOT, [i, i + 1])
    return b.build(n * layers)


def uniform_params(count: int, seed: int) -> np.ndarray:
    """theta ~ U[0, 2 pi)^count from numpy's PCG64 generator."""
    return np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi, count)


def xyz_chain(n: int, jx: float = 1.0, jy: float = 0.8, jz: float = 0.6,
              h: float = 0.0, periodic: bool = False) -> PauliSum:
    """XYZ Heisenberg chain H = -sum_<ij>(Jx XX + Jy YY + Jz ZZ) - h sum Z.

    Bonds (i, i+1) for i = 0..n-2 (open chain) plus (n-1, 0) if periodic,
    listed bond by bond as XX, YY, ZZ; field terms are only added for h != 0.
    """
    terms = []
    bonds = [(i, i + 1) for i in range(n - 1)]
    if periodic and n > 2:
        bonds.append((n - 1, 0))
    for (i, j) in bonds:
        for p, jv in (("X", jx), ("Y", jy), ("Z", jz)):
            s = ["I"] * n
            s[i] = p
            s[j] = p
            terms.append((-jv, "".join(s)))
    if h != 0.0:
        for i in range(n):
            s = ["I"] * n
            s[i] = "Z"
            terms.append((-h, "".join(s)))
    return PauliSum.from_strings(n, terms)


def random_2local(n: int, n_terms: int, seed: int) -> PauliSum:
    """Random 2-local Pauli sum: each term picks an unordered pair of distinct
    qubits uniformly and an independent uniform Pauli in {X, Y, Z} for each;
    coefficients ~ N(0, 1).  Duplicated supports stay separate terms.
    """
    rng = np.random.default_rng(seed)
    rows = np.full((n_terms, n), ord("I"), dtype=np.uint8)
    letters = np.frombuffer(b"XYZ", dtype=np.uint8)
    for t in range(n_terms):
        a, b = rng.choice(n, size=2, replace=False)
        rows[t, a] = letters[rng.integers(3)]
        rows[t, b] = letters[rng.integers(3)]
    coeffs = rng.standard_normal(n_terms)
    return PauliSum(n, coeffs, rows)


def gaussian_state(n: int, seed: int) -> np.ndarray:
    """complex128 [2^n]: re, im i.i.d. N(0,1), scaled to unit norm in FP64."""
    rng = np.random.default_rng(seed)
    dim = 1 << n
    v = rng.standard_normal(dim) + 1j * rng.standard_normal(dim)
    return v / np.sqrt(np.vdot(v, v).real)


def deep_random_circuit(n: int, depth: int, seed: int) -> Circuit:
    """Per layer: U3(theta, phi, lambda) on every qubit with angles
    U[0, 2 pi)^3, then CZ on a fresh random perfect matching (qubits permuted
    by the layer's draw and paired (0,1), (2,3), ...).
    """
    rng = np.random.default_rng(seed)
    b = CircuitBuilder(n)
    for _ in range(depth):
        ang = rng.uniform(0.0, 2.0 * math.pi, size=(n, 3))
        for q in range(n):
            b.add(U3, [q], angles=list(ang[q]))
        perm = rng.permutation(n)
        for k in range(0, n - 1, 2):
            b.add(CZ, [int(perm[k]), int(perm[k + 1])])
    return b.build(0)


def xyz_field(t: float, amplitude: float = 2.0, omega: float = 1.0) -> float:
    """Longitudinal field h(t) = A sin(omega t) of Eq. "xyz_hamiltonian"."""
    return amplitude * math.sin(omega * t)


def trotter_xyz_circuit(n: int, steps: int, t_total: float, jx: float = 1.0, jy: float = 0.8,
                        jz: float = 0.6, amplitude: float = 2.0, omega: float = 1.0) -> Circuit:
    """First-order Trotter circuit (Eq. "trotter") for the open XYZ chain of
    Eq. "xyz_hamiltonian": X on every qubit (|1...1> from |0...0>), then per
    step j (t_j = j dt, dt = t_total / steps) the factor exp(-i H_k dt) of
    every term in the order bond (i, i+1) XX, YY, ZZ for i = 0..n-2, then
    the field on every qubit.  H's terms are -J P_i P_{i+1} and -h(t) Z_i,
    so exp(-i H_k dt) = R_PP(-2 J dt) and R_Z(-2 h(t_j) dt) with
    R_P(theta) = exp(-i theta P / 2).
    """
    dt = t_total / steps
    b = CircuitBuilder(n)
    for q in range(n):
        b.add(X, [q])
    for j in range(steps):
        h = xyz_field(j * dt, amplitude, omega)
        for i in range(n - 1):
            for kind, jv in ((RXX, jx), (RYY, jy), (RZZ, jz)):
                b.add(kind, [i, i + 1], angles=[-2.0 * jv * dt])
        for q in range(n):
            b.add(RZ, [q], angles=[-2.0 * h * dt])
    return b.build(0)


def app_d_circuit() -> Circuit:
    """Edge-case circuit of the paper's App. D (Fig. "edge_case_circuit"):
    RX(t0) q0, RY(t1) q1, RZ(t2) q0, CNOT(0 -> 1), CRY(t3) control 1 target 0.
    """
    b = CircuitBuilder(2)
    b.add(RX, [0], params=[0])
    b.add(RY, [1], params=[1])
    b.add(RZ, [0], params=[2])
    b.add(CNOT, [0, 1])
    b.add(CRY, [1, 0], params=[3])
    return b.build(4)


def app_d_observable() -> PauliSum:
    """<Z_0> on two qubits (App. D)."""
    return PauliSum.from_strings(2, [(1.0, "ZI")])


APP_D_CASES = {
    "normal": [0.5, 0.3, 0.2, 0.1],
    "large": [10.0, 5.0, 3.0, 2.0],
    "near_zero": [1e-8, 1e-7, 1e-6, 1e-5],
    "pi_half": [math.pi / 2] * 4,
    "pi": [math.pi] * 4,
}


def random_circuit(n: int, n_gates: int, seed: int,
                   kinds: Optional[Sequence[int]] = None,
                   n_params: int = 0) -> Circuit:
    """Random gate list over every kind (for parity tests).  Angles U[0,2pi);
    when n_params > 0, angled gates draw a parameter index with probability
    1/2 instead of a fixed angle.  MAT1/MAT2 get random unitaries (QR of a
    complex Gaussian matrix).
    """
    rng = np.random.default_rng(seed)
    allk = [k for k in (kinds if kinds is not None else range(21))
            if ARITY[k] <= n]
    b = CircuitBuilder(n)
    for _ in range(n_gates):
        k = int(allk[rng.integers(len(allk))])
        qs = [int(x) for x in rng.choice(n, size=ARITY[k], replace=False)]
        if k in (MAT1, MAT2):
            d = 2 if k == MAT1 else 4
            z = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
            qm, _ = np.linalg.qr(z)
            b.add_matrix(qs, qm)
            continue
        na = N_ANGLES.get(k, 0)
        ang = list(rng.uniform(0, 2 * math.pi, size=na))
        prm = []
        if n_params > 0 and na > 0:
            for _a in range(na):
                prm.append(int(rng.integers(n_params))
                           if rng.random() < 0.5 else -1)
        b.add(k, qs, angles=ang, params=prm)
    return b.build(max(n_params, b.n_params))


@dataclasses.dataclass
class Request:
    """One serving request: energy (grad=False) or full gradient."""
    rid: int
    arrival_s: float
    n: int
    depth: int
    grad: bool
    circuit: Circuit
    params: np.ndarray
    hamiltonian: PauliSum


def serving_requests(count: int, seed: int, rate_per_s: float,
                     n_range=(8, 24), depth_range=(2, 10),
                     terms_range=(20, 200)) -> List[Request]:
    """Poisson stream: exponential inter-arrival times at rate_per_s; qubit
    count, ansatz depth and term count uniform over their inclusive ranges;
    half energy-only, half gradient requests (independent fair draws); HEA
    RY/RZ + CNOT-ladder circuits; random 2-local Hamiltonians.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        # one Exp(1) draw per request whatever the rate, so the request list
        # is the same at every arrival rate (rate 0: all at t = 0)
        gap = rng.exponential(1.0)
        t += gap / rate_per_s if rate_per_s > 0 else 0.0
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        depth = int(rng.integers(depth_range[0], depth_range[1] + 1))
        nt = int(rng.integers(terms_range[0], terms_range[1] + 1))
        grad = bool(rng.integers(2))
        sub = int(rng.integers(2 ** 31))
        c = hea_circuit(n, depth)
        params = uniform_params(c.n_params, sub)
        ham = random_2local(n, nt, sub + 1)
        out.append(Request(rid, t, n, depth, grad, c, params, ham))
    return out
