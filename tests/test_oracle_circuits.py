"""Whole-circuit pins of the oracle: closed forms (GHZ, QFT), inverse
circuits, norm preservation and classical special cases."""
import math

import numpy as np
import pytest

import qsynth


@pytest.mark.parametrize("n", [1, 2, 5, 12])
def test_ghz(oracle, n):
    psi = oracle.run(qsynth.ghz(n))
    ref = np.zeros(1 << n, dtype=complex)
    ref[0] = ref[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(psi - ref)) < 1e-15


@pytest.mark.parametrize("n,x", [(3, 5), (6, 0), (6, 37), (10, 777)])
def test_qft_of_basis_state(oracle, n, x):
    """QFT|x> = 2^{-n/2} sum_y exp(2 pi i x y / 2^n) |y>."""
    N = 1 << n
    psi = oracle.run(qsynth.qft(n), oracle.basis_state(n, x))
    y = np.arange(N)
    ref = np.exp(2j * math.pi * x * y / N) / math.sqrt(N)
    assert np.max(np.abs(psi - ref)) < 1e-12


def test_qft_without_swaps_is_bit_reversed(oracle):
    n, x = 7, 93
    N = 1 << n
    psi = oracle.run(qsynth.qft(n, swaps=False), oracle.basis_state(n, x))
    rev = np.array([int(format(i, f"0{n}b")[::-1], 2) for i in range(N)])
    ref = np.exp(2j * math.pi * x * np.arange(N) / N) / math.sqrt(N)
    assert np.max(np.abs(psi[rev] - ref)) < 1e-12


@pytest.mark.parametrize("seed,n", [(0, 10), (1, 12), (2, 14)])
def test_inverse_circuit_returns_zero_state(oracle, seed, n):
    c = qsynth.random_circuit(n, 150, seed=seed, max_dense=3)
    psi = oracle.run(c)
    psi = oracle.run(qsynth.inverse(c), psi)
    ref = oracle.zero_state(n)
    assert np.max(np.abs(psi - ref)) < 1e-12


def test_norm_preserved(oracle):
    n = 14
    psi = oracle.run(qsynth.brickwork(n, depth=6, seed=3))
    assert abs(math.sqrt(oracle.norm2(psi, n)) - 1.0) < 1e-13
    psi = oracle.run(qsynth.plain_random(12, 20, 6, seed=1))
    assert abs(math.sqrt(oracle.norm2(psi, 12)) - 1.0) < 1e-13


def test_zero_angles_are_identity(oracle):
    n = 8
    c = qsynth.Circuit(n)
    for q in range(n):
        c.add("rx", (q,), (0.0,)).add("ry", (q,), (0.0,)).add("rz", (q,), (0.0,))
        c.add("u3", (q,), (0.0, 0.0, 0.0)).add("cp", (q, (q + 3) % n), (0.0,))
    psi0 = qsynth.random_state(n, seed=4)
    psi = oracle.run(c, psi0.copy())
    assert np.max(np.abs(psi - psi0)) < 1e-15


def test_cnot_circuit_is_bit_permutation(oracle):
    """CNOT/X/SWAP-only circuits map basis states to basis states by the
    classical reversible function, computed here on the integer index."""
    n = 9
    rng = np.random.default_rng(8)
    c = qsynth.Circuit(n)
    for _ in range(60):
        kind = ["cx", "x", "swap"][int(rng.integers(0, 3))]
        if kind == "x":
            c.add("x", (int(rng.integers(0, n)),))
        else:
            a, b = (int(v) for v in rng.choice(n, size=2, replace=False))
            c.add(kind, (a, b))

    def classical(i):
        for g in c.gates:
            if g.name == "x":
                i ^= 1 << g.qubits[0]
            elif g.name == "cx":
                a, b = g.qubits
                if (i >> a) & 1:
                    i ^= 1 << b
            else:
                a, b = g.qubits
                ba, bb = (i >> a) & 1, (i >> b) & 1
                if ba != bb:
                    i ^= (1 << a) | (1 << b)
        return i

    for x in rng.integers(0, 1 << n, size=12):
        psi = oracle.run(c, oracle.basis_state(n, int(x)))
        assert abs(psi[classical(int(x))] - 1.0) < 1e-15
        assert abs(oracle.norm2(psi, n) - 1.0) < 1e-15


def test_rz_only_phases(oracle):
    """Product of RZ gates is diagonal: phase exp(-i/2 sum_q theta_q (-1)^{b_q})."""
    n = 8
    rng = np.random.default_rng(9)
    thetas = rng.random(n) * 2 * math.pi
    c = qsynth.Circuit(n)
    for q in range(n):
        c.add("rz", (q,), (thetas[q],))
    psi0 = qsynth.random_state(n, seed=10)
    psi = oracle.run(c, psi0.copy())
    idx = np.arange(1 << n)
    ph = np.zeros(1 << n)
    for q in range(n):
        ph += -0.5 * thetas[q] * (1 - 2 * ((idx >> q) & 1))
    assert np.max(np.abs(psi - np.exp(1j * ph) * psi0)) < 1e-14


def test_qaoa_state_is_invariant_under_global_flip(oracle):
    """QAOA for MaxCut starts from |+>^n and uses ZZ costs and an RX mixer,
    all of which commute with X on every qubit, so psi[k] = psi[~k]."""
    n = 10
    c = qsynth.qaoa_maxcut(n, p=2, seed=(3, 1))
    psi = oracle.run(c)
    full = (1 << n) - 1
    idx = np.arange(1 << n)
    assert np.max(np.abs(psi - psi[idx ^ full])) <= 1e-12
    assert abs(np.vdot(psi, psi).real - 1) <= 1e-12


def test_qaoa_graph_is_three_regular():
    rng = np.random.default_rng(4)
    edges = qsynth.random_regular_edges(rng, 12, 3)
    deg = np.zeros(12, dtype=int)
    for a, b in edges:
        assert a != b
        deg[a] += 1
        deg[b] += 1
    assert len(set(edges)) == len(edges) == 18 and np.all(deg == 3)


def test_hea_rxyz_shape_and_norm(oracle):
    n, layers = 9, 5
    c = qsynth.hea_rxyz(n, layers, seed=(2, 2))
    ncx = sum(len(range(l % 2, n - 1, 2)) for l in range(layers))
    assert len(c) == layers * 3 * n + ncx
    psi = oracle.run(c)
    assert abs(np.vdot(psi, psi).real - 1) <= 1e-12
