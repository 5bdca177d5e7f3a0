"""Brute-force 2^n x 2^n operators for small n (TEST INFRASTRUCTURE ONLY).

Every gate is built as an explicit Kronecker product in the order of Eq. 2
(Section 2.1): the leftmost factor acts on the highest qubit, so a one-qubit
gate U on qubit k is I^(n-k-1) (x) U (x) I^(k).  Controlled gates use the
projector form of Section 2.1 (|0><0| (x) I + |1><1| (x) U).  Gate matrices
are defined from their generators with a matrix exponential, independently
of the closed-form table in sv_oracle.c, so the two pin each other.

Used only for n <= 10.
"""
from __future__ import annotations

import math
from functools import reduce

import numpy as np
from scipy.linalg import expm

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)
PAULI = {"I": I2, "X": X, "Y": Y, "Z": Z}


def rot(gen: np.ndarray, theta: float) -> np.ndarray:
    """exp(-i theta gen / 2)."""
    return expm(-0.5j * theta * gen)


def phase(lam: float) -> np.ndarray:
    """diag(1, e^{i lam}) = exp(i lam (I - Z) / 2)."""
    return expm(0.5j * lam * (I2 - Z))


def gate_matrix(name: str, params=()) -> np.ndarray:
    """2x2 matrix of a one-qubit kind, or of the target part of a
    controlled kind, from generators."""
    p = list(params) + [0.0] * (3 - len(params))
    if name == "h":
        return (X + Z) / math.sqrt(2.0)
    if name in ("x", "cx"):
        return X.copy()
    if name == "y":
        return Y.copy()
    if name in ("z", "cz"):
        return Z.copy()
    if name == "s":
        return phase(math.pi / 2)
    if name == "sdg":
        return phase(-math.pi / 2)
    if name == "t":
        return phase(math.pi / 4)
    if name == "tdg":
        return phase(-math.pi / 4)
    if name == "rx":
        return rot(X, p[0])
    if name == "ry":
        return rot(Y, p[0])
    if name == "rz":
        return rot(Z, p[0])
    if name in ("p", "cp"):
        return phase(p[0])
    if name in ("u3", "cu"):
        th, ph, la = p
        return np.exp(0.5j * (ph + la)) * rot(Z, ph) @ rot(Y, th) @ rot(Z, la)
    raise ValueError(name)


def embed(n: int, ops: dict) -> np.ndarray:
    """Kronecker product over qubits n-1 ... 0 (Eq. 2 order); `ops` maps
    qubit -> 2x2 operator, identity elsewhere."""
    return reduce(np.kron, [ops.get(q, I2) for q in reversed(range(n))])


def gate_operator(n: int, name: str, qubits, params=(), matrix=None) -> np.ndarray:
    qubits = tuple(qubits)
    if name in ("cx", "cz", "cp", "cu"):
        c, t = qubits
        u = gate_matrix(name, params)
        return embed(n, {c: P0}) + embed(n, {c: P1, t: u})
    if name == "swap":
        a, b = qubits
        return 0.5 * (embed(n, {}) + embed(n, {a: X, b: X}) + embed(n, {a: Y, b: Y})
                      + embed(n, {a: Z, b: Z}))
    if name == "dense":
        k = len(qubits)
        d = 1 << k
        op = np.zeros((1 << n, 1 << n), dtype=np.complex128)
        for r in range(d):
            for c in range(d):
                if matrix[r, c] == 0:
                    continue
                ops = {}
                for j, q in enumerate(qubits):
                    e = np.zeros((2, 2), dtype=np.complex128)
                    e[(r >> j) & 1, (c >> j) & 1] = 1.0
                    ops[q] = e
                op += matrix[r, c] * embed(n, ops)
        return op
    (q,) = qubits
    return embed(n, {q: gate_matrix(name, params)})


def circuit_operator(circuit) -> np.ndarray:
    """U_G ... U_1 as one dense matrix."""
    n = circuit.n
    U = np.eye(1 << n, dtype=np.complex128)
    for g in circuit.gates:
        U = gate_operator(n, g.name, g.qubits, g.params, g.matrix) @ U
    return U


def pauli_operator(n: int, letters) -> np.ndarray:
    """Dense Pauli string from (qubit, letter) pairs."""
    return embed(n, {q: PAULI[a] for q, a in letters})


def pauli_from_masks(n: int, x: int, z: int) -> np.ndarray:
    letters = []
    for q in range(n):
        bx, bz = (x >> q) & 1, (z >> q) & 1
        if bx and bz:
            letters.append((q, "Y"))
        elif bx:
            letters.append((q, "X"))
        elif bz:
            letters.append((q, "Z"))
    return pauli_operator(n, letters)
