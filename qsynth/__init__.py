"""Seeded synthetic workloads: circuits and Pauli sums.

This module is shared by the oracle, the tests and the benchmark.  It holds
no simulation arithmetic: it only draws random numbers and lays gates out in
order.  A gate is (name, qubits, params[, matrix]); for controlled kinds the
control comes first.  Qubit q is bit q of the amplitude index.

Workload shapes follow the paper's circuit families (Section 4.1: QFT, QAOA
and a hardware-efficient ansatz of parameterised one-qubit layers with
staggered CNOTs, 20-30 qubits, hundreds to ~1.7k gates; Section 1: VQE with
UCC and hardware-efficient ansatze and Pauli-sum Hamiltonians).  The paper's
own circuit files are not available; these seeded generators stand in for
them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

ONE_QUBIT = ("h", "x", "y", "z", "s", "sdg", "t", "tdg", "rx", "ry", "rz", "u3", "p")
TWO_QUBIT = ("cx", "cz", "cp", "cu", "swap")
N_PARAMS = {"rx": 1, "ry": 1, "rz": 1, "p": 1, "cp": 1, "u3": 3, "cu": 3}


@dataclass
class Gate:
    name: str
    qubits: Tuple[int, ...]
    params: Tuple[float, ...] = ()
    matrix: Optional[np.ndarray] = None  # only for name == "dense"

    def __post_init__(self):
        self.qubits = tuple(int(q) for q in self.qubits)
        self.params = tuple(float(p) for p in self.params)


@dataclass
class Circuit:
    n: int
    gates: List[Gate] = field(default_factory=list)

    def add(self, name, qubits, params=(), matrix=None):
        self.gates.append(Gate(name, tuple(qubits), tuple(params), matrix))
        return self

    def __len__(self):
        return len(self.gates)

    def prefix(self, count: int) -> "Circuit":
        return Circuit(self.n, list(self.gates[:count]))


@dataclass
class PauliSum:
    """sum_k coeff[k] * P_k with P_k given by masks: x = X or Y positions,
    z = Z or Y positions."""
    n: int
    x: np.ndarray
    z: np.ndarray
    coeff: np.ndarray

    def __len__(self):
        return len(self.coeff)


# ------------------------------------------------------------ helpers
def _rng(*seed) -> np.random.Generator:
    return np.random.default_rng(list(seed) if len(seed) > 1 else seed[0])


def haar_u3_angles(rng: np.random.Generator):
    """U3 angles whose matrices are Haar distributed on SU(2) modulo phase:
    phi, lambda ~ U[0, 2pi), theta = arccos(1 - 2u) (density ~ sin theta)."""
    u = rng.random()
    theta = math.acos(1.0 - 2.0 * u)
    phi = rng.random() * 2 * math.pi
    lam = rng.random() * 2 * math.pi
    return theta, phi, lam


def random_disjoint_pairs(rng: np.random.Generator, n: int, count: int):
    """`count` disjoint qubit pairs from a random permutation; the first
    element of each pair is the control."""
    perm = rng.permutation(n)
    assert 2 * count <= n
    return [(int(perm[2 * i]), int(perm[2 * i + 1])) for i in range(count)]


def pauli_masks(letters: Sequence[Tuple[int, str]]) -> Tuple[int, int]:
    x = z = 0
    for q, a in letters:
        if a in ("X", "Y"):
            x |= 1 << q
        if a in ("Z", "Y"):
            z |= 1 << q
    return x, z


# ---------------------------------------------------------- workloads
def plain_random(n: int = 12, layers: int = 20, pairs: int = 6, seed: int = 1) -> Circuit:
    """Random circuit: per layer every qubit gets H or RZ(theta ~ U[0,2pi))
    with probability 1/2 each, then `pairs` CNOTs on random disjoint pairs."""
    rng = _rng(seed)
    c = Circuit(n)
    for _ in range(layers):
        for q in range(n):
            if rng.random() < 0.5:
                c.add("h", (q,))
            else:
                c.add("rz", (q,), (rng.random() * 2 * math.pi,))
        for a, b in random_disjoint_pairs(rng, n, pairs):
            c.add("cx", (a, b))
    return c


def brickwork(n: int = 28, depth: int = 40, seed: int = 2) -> Circuit:
    """Haar-random U3 on every qubit, then CNOTs on neighbour pairs that
    alternate between (0,1),(2,3),... and (1,2),(3,4),... layer by layer."""
    rng = _rng(seed)
    c = Circuit(n)
    for layer in range(depth):
        for q in range(n):
            c.add("u3", (q,), haar_u3_angles(rng))
        start = layer % 2
        for a in range(start, n - 1, 2):
            c.add("cx", (a, a + 1))
    return c


def pauli_exponential(c: Circuit, letters: Sequence[Tuple[int, str]], theta: float) -> None:
    """Append exp(-i theta P) for P = prod of letters (support ascending):
    basis change (X: H, Y: RX(pi/2)), CNOT ladder along the support, RZ(2 theta)
    on the last support qubit, reverse ladder, reverse basis change
    (X: H, Y: RX(-pi/2))."""
    letters = sorted(letters)
    sup = [q for q, _ in letters]
    for q, a in letters:
        if a == "X":
            c.add("h", (q,))
        elif a == "Y":
            c.add("rx", (q,), (math.pi / 2,))
    for i in range(len(sup) - 1):
        c.add("cx", (sup[i], sup[i + 1]))
    c.add("rz", (sup[-1],), (2.0 * theta,))
    for i in reversed(range(len(sup) - 1)):
        c.add("cx", (sup[i], sup[i + 1]))
    for q, a in letters:
        if a == "X":
            c.add("h", (q,))
        elif a == "Y":
            c.add("rx", (q,), (-math.pi / 2,))


def ucc(n: int = 30, n_exp: int = 2000, wmin: int = 4, wmax: int = 8,
        theta_sd: float = 0.1, seed: int = 3):
    """UCC-style ansatz: `n_exp` Pauli exponentials exp(-i theta P) with
    weight w ~ U{wmin..wmax}, support w distinct uniform qubits, letters
    uniform in {X, Y, Z}, theta ~ N(0, theta_sd).

    Returns (circuit, rotations) where rotations is a list of (x, z, theta)
    for the closed-form oracle."""
    rng = _rng(seed)
    c = Circuit(n)
    rots = []
    for _ in range(n_exp):
        w = int(rng.integers(wmin, wmax + 1))
        sup = sorted(int(q) for q in rng.choice(n, size=w, replace=False))
        letters = [(q, "XYZ"[int(rng.integers(0, 3))]) for q in sup]
        theta = float(rng.normal(0.0, theta_sd))
        pauli_exponential(c, letters, theta)
        x, z = pauli_masks(letters)
        rots.append((x, z, theta))
    return c, rots


def hea(n: int, layers: int = 8, seed=(4, 0)) -> Circuit:
    """Hardware-efficient ansatz: per layer RY(theta) and RZ(theta) on every
    qubit (theta ~ U[0,2pi)), then a CZ ring (i, i+1 mod n)."""
    rng = _rng(*seed) if isinstance(seed, tuple) else _rng(seed)
    c = Circuit(n)
    for _ in range(layers):
        for q in range(n):
            c.add("ry", (q,), (rng.random() * 2 * math.pi,))
        for q in range(n):
            c.add("rz", (q,), (rng.random() * 2 * math.pi,))
        for q in range(n):
            c.add("cz", (q, (q + 1) % n))
    return c


def hea_rxyz(n: int, layers: int = 5, seed=(8, 0)) -> Circuit:
    """The paper's HEA shape: per layer RX, RY, RZ (theta ~ U[0,2pi)) on every
    qubit, then staggered CNOTs (0,1),(2,3),... on even layers and
    (1,2),(3,4),... on odd layers."""
    rng = _rng(*seed) if isinstance(seed, tuple) else _rng(seed)
    c = Circuit(n)
    for layer in range(layers):
        for name in ("rx", "ry", "rz"):
            for q in range(n):
                c.add(name, (q,), (rng.random() * 2 * math.pi,))
        for q in range(layer % 2, n - 1, 2):
            c.add("cx", (q, q + 1))
    return c


def random_regular_edges(rng: np.random.Generator, n: int, degree: int = 3):
    """Edges of a random `degree`-regular simple graph on n vertices (n*degree
    even), by the configuration model with restarts."""
    assert (n * degree) % 2 == 0 and degree < n
    while True:
        stubs = rng.permutation(np.repeat(np.arange(n), degree))
        pairs = stubs.reshape(-1, 2)
        edges = {tuple(sorted((int(a), int(b)))) for a, b in pairs}
        if all(a != b for a, b in pairs) and len(edges) == len(pairs):
            return sorted(edges)


def qaoa_maxcut(n: int, p: int = 3, seed=(9, 0)) -> Circuit:
    """QAOA for MaxCut on a random 3-regular graph: H on every qubit, then p
    rounds of exp(-i gamma Z_a Z_b) per edge (CNOT, RZ(2 gamma), CNOT) and
    RX(2 beta) on every qubit; gamma, beta ~ U[0, pi)."""
    rng = _rng(*seed) if isinstance(seed, tuple) else _rng(seed)
    edges = random_regular_edges(rng, n, 3 if n % 2 == 0 else 2)
    c = Circuit(n)
    for q in range(n):
        c.add("h", (q,))
    for _ in range(p):
        gamma, beta = rng.random() * math.pi, rng.random() * math.pi
        for a, b in edges:
            c.add("cx", (a, b))
            c.add("rz", (b,), (2 * gamma,))
            c.add("cx", (a, b))
        for q in range(n):
            c.add("rx", (q,), (2 * beta,))
    return c


def random_pauli_sum(n: int, n_terms: int = 200, seed=(5, 0)) -> PauliSum:
    """Per term and qubit a letter uniform in {I, X, Y, Z}; coeff ~ N(0, 1)."""
    rng = _rng(*seed) if isinstance(seed, tuple) else _rng(seed)
    xs = np.zeros(n_terms, dtype=np.uint64)
    zs = np.zeros(n_terms, dtype=np.uint64)
    for k in range(n_terms):
        letters = [(q, "IXYZ"[int(rng.integers(0, 4))]) for q in range(n)]
        x, z = pauli_masks([(q, a) for q, a in letters if a != "I"])
        xs[k], zs[k] = x, z
    coeff = rng.normal(0.0, 1.0, size=n_terms)
    return PauliSum(n, xs, zs, coeff)


def hea_batch(n_states: int = 256, nmin: int = 12, nmax: int = 22, layers: int = 8,
              n_terms: int = 200, seed: int = 4):
    """Batch of HEA states with qubit counts uniform in nmin..nmax and one
    random Pauli-sum Hamiltonian per state."""
    rng = _rng(seed)
    ns = [int(v) for v in rng.integers(nmin, nmax + 1, size=n_states)]
    circuits = [hea(n, layers, seed=(seed, i)) for i, n in enumerate(ns)]
    hams = [random_pauli_sum(n, n_terms, seed=(seed + 1000, i)) for i, n in enumerate(ns)]
    return circuits, hams


def random_u3_cnot(n: int = 33, depth: int = 30, seed: int = 5) -> Circuit:
    """Per layer Haar U3 on every qubit plus floor(n/2) CNOTs on random
    disjoint pairs."""
    rng = _rng(seed)
    c = Circuit(n)
    for _ in range(depth):
        for q in range(n):
            c.add("u3", (q,), haar_u3_angles(rng))
        for a, b in random_disjoint_pairs(rng, n, n // 2):
            c.add("cx", (a, b))
    return c


def random_circuit(n: int, n_gates: int, seed: int = 0, kinds=None, max_dense: int = 0) -> Circuit:
    """Random mix of every gate kind (property and parity tests)."""
    rng = _rng(seed)
    kinds = list(kinds) if kinds is not None else list(ONE_QUBIT + TWO_QUBIT)
    if max_dense:
        kinds.append("dense")
    c = Circuit(n)
    for _ in range(n_gates):
        name = kinds[int(rng.integers(0, len(kinds)))]
        if name == "dense":
            k = int(rng.integers(1, min(max_dense, n) + 1))
            qs = [int(q) for q in rng.choice(n, size=k, replace=False)]
            a = rng.normal(size=(1 << k, 1 << k)) + 1j * rng.normal(size=(1 << k, 1 << k))
            q_, r_ = np.linalg.qr(a)
            c.add("dense", qs, (), q_ * (np.diag(r_) / np.abs(np.diag(r_))))
            continue
        if name in TWO_QUBIT and n < 2:
            name = "h"
        if name in TWO_QUBIT:
            qs = [int(q) for q in rng.choice(n, size=2, replace=False)]
        else:
            qs = [int(rng.integers(0, n))]
        params = tuple(rng.random() * 2 * math.pi for _ in range(N_PARAMS.get(name, 0)))
        c.add(name, qs, params)
    return c


# -------------------------------------------------- closed-form circuits
def ghz(n: int) -> Circuit:
    c = Circuit(n).add("h", (0,))
    for q in range(n - 1):
        c.add("cx", (q, q + 1))
    return c


def qft(n: int, swaps: bool = True) -> Circuit:
    """Quantum Fourier transform (most significant qubit first, controlled
    phases pi / 2^(j-k), then the reversing swap network)."""
    c = Circuit(n)
    for j in reversed(range(n)):
        c.add("h", (j,))
        for k in reversed(range(j)):
            c.add("cp", (k, j), (math.pi / (1 << (j - k)),))
    if swaps:
        for i in range(n // 2):
            c.add("swap", (i, n - 1 - i))
    return c


_SELF_INVERSE = {"h", "x", "y", "z", "cx", "cz", "swap"}
_SWAP_INV = {"s": "sdg", "sdg": "s", "t": "tdg", "tdg": "t"}


def inverse(c: Circuit) -> Circuit:
    """C^dagger: gates reversed, each replaced by its inverse."""
    out = Circuit(c.n)
    for g in reversed(c.gates):
        if g.name in _SELF_INVERSE:
            out.add(g.name, g.qubits)
        elif g.name in _SWAP_INV:
            out.add(_SWAP_INV[g.name], g.qubits)
        elif g.name in ("rx", "ry", "rz", "p", "cp"):
            out.add(g.name, g.qubits, (-g.params[0],))
        elif g.name in ("u3", "cu"):
            th, ph, la = g.params
            out.add(g.name, g.qubits, (-th, -la, -ph))
        elif g.name == "dense":
            out.add("dense", g.qubits, (), np.conj(g.matrix).T.copy())
        else:
            raise ValueError(g.name)
    return out


def random_state(n: int, seed: int = 0, dtype=np.complex128) -> np.ndarray:
    """Normalised random state with Gaussian real and imaginary parts."""
    rng = _rng(seed)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    v /= np.sqrt(np.vdot(v, v).real)
    return v.astype(dtype)
