"""Brute-force 2^n x 2^n operators for small n, built independently of the
oracle: rotations by matrix exponentials of their Pauli generators, controlled
gates from projectors, permutations from their action on basis states, and
qubit placement by Kronecker products (qubit 0 = leftmost factor = most
significant index bit).  Used only to pin the oracle on small inputs.
"""
import math

import numpy as np
import scipy.linalg as sla

from paper_2512_23183_amd import inputs as I

PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
ID = np.eye(2, dtype=complex)
P0 = np.array([[1, 0], [0, 0]], dtype=complex)
P1 = np.array([[0, 0], [0, 1]], dtype=complex)
# Hadamard as printed in App. C.
HAD = np.array([[1, 1], [1, -1]], dtype=complex) / math.sqrt(2.0)
PAULI = {"I": ID, "X": PX, "Y": PY, "Z": PZ}


def place(ops: dict, n: int) -> np.ndarray:
    """Kronecker product with ops[q] on qubit q and identity elsewhere."""
    m = np.eye(1, dtype=complex)
    for q in range(n):
        m = np.kron(m, ops.get(q, ID))
    return m


def rot(P, theta):
    return sla.expm(-0.5j * theta * P)


def u3(theta, phi, lam):
    # OpenQASM 2: U3 = e^{i(phi+lam)/2} RZ(phi) RY(theta) RZ(lam)
    return np.exp(0.5j * (phi + lam)) * rot(PZ, phi) @ rot(PY, theta) @ rot(PZ, lam)


def controlled(c, t, U, n):
    return place({c: P0}, n) + place({c: P1, t: U}, n)


def gate_operator(n, kind, q, ang, mat=None) -> np.ndarray:
    if kind == I.H:
        return place({q[0]: HAD}, n)
    if kind in (I.X, I.Y, I.Z):
        return place({q[0]: [PX, PY, PZ][kind - I.X]}, n)
    if kind in (I.RX, I.RY, I.RZ):
        return place({q[0]: rot([PX, PY, PZ][kind - I.RX], ang[0])}, n)
    if kind == I.U3:
        return place({q[0]: u3(*ang[:3])}, n)
    if kind == I.CNOT:
        return controlled(q[0], q[1], PX, n)
    if kind in (I.CRX, I.CRY, I.CRZ):
        return controlled(q[0], q[1], rot([PX, PY, PZ][kind - I.CRX], ang[0]), n)
    if kind == I.CZ:
        return np.eye(1 << n) - 2 * place({q[0]: P1, q[1]: P1}, n)
    if kind == I.CP:
        return sla.expm(1j * ang[0] * place({q[0]: P1, q[1]: P1}, n))
    if kind == I.CCX:
        both = place({q[0]: P1, q[1]: P1}, n)
        return np.eye(1 << n) - both + place({q[0]: P1, q[1]: P1, q[2]: PX}, n)
    if kind == I.SWAP:
        dim = 1 << n
        m = np.zeros((dim, dim), dtype=complex)
        for x in range(dim):
            bits = [(x >> (n - 1 - k)) & 1 for k in range(n)]
            bits[q[0]], bits[q[1]] = bits[q[1]], bits[q[0]]
            y = sum(b << (n - 1 - k) for k, b in enumerate(bits))
            m[y, x] = 1
        return m
    if kind in (I.RXX, I.RYY, I.RZZ):
        P = [PX, PY, PZ][kind - I.RXX]
        return sla.expm(-0.5j * ang[0] * place({q[0]: P, q[1]: P}, n))
    if kind == I.MAT1:
        return place({q[0]: np.asarray(mat).reshape(2, 2)}, n)
    if kind == I.MAT2:
        U = np.asarray(mat).reshape(4, 4)
        dim = 1 << n
        m = np.zeros((dim, dim), dtype=complex)
        for r in range(4):
            for c in range(4):
                er = np.zeros((2, 2), dtype=complex)
                ec = np.zeros((2, 2), dtype=complex)
                er[r >> 1, c >> 1] = 1
                ec[r & 1, c & 1] = 1
                m += U[r, c] * place({q[0]: er, q[1]: ec}, n)
        return m
    raise ValueError(kind)


def circuit_unitary(circ, params=None) -> np.ndarray:
    n = circ.n
    U = np.eye(1 << n, dtype=complex)
    for g in circ.gates:
        k = int(g["kind"])
        a = [float(g["angle"][j]) + (params[int(g["param_idx"][j])]
             if g["param_idx"][j] >= 0 else 0.0) for j in range(3)]
        mat = None
        if k in (I.MAT1, I.MAT2):
            flat = circ.mats[int(g["mat_idx"])]
            d = 4 if k == I.MAT1 else 16
            mat = flat[0:2 * d:2] + 1j * flat[1:2 * d:2]
        U = gate_operator(n, k, [int(x) for x in g["q"]], a, mat) @ U
    return U


def pauli_operator(s: str) -> np.ndarray:
    m = np.eye(1, dtype=complex)
    for ch in s:
        m = np.kron(m, PAULI[ch])
    return m


def hamiltonian_matrix(ham) -> np.ndarray:
    dim = 1 << ham.n
    Hm = np.zeros((dim, dim), dtype=complex)
    for c, s in zip(ham.coeffs, ham.strings()):
        Hm += c * pauli_operator(s)
    return Hm
