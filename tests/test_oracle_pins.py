"""Pins of the FP64 oracle against what the paper and the mathematics fix
(gate definitions, Eq. 2-4 and 6, Algorithms 1-4, the Kronecker fusion
entries and the operation-count model of Section 3.4)."""
import math
import os

import numpy as np
import pytest

import qsynth
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ONE_Q = ["h", "x", "y", "z", "s", "sdg", "t", "tdg", "rx", "ry", "rz", "u3", "p"]


def _params(rng, name):
    return tuple(rng.random() * 4 * math.pi - 2 * math.pi for _ in range(qsynth.N_PARAMS.get(name, 0)))


@pytest.mark.parametrize("name", ONE_Q + ["cx", "cz", "cp", "cu"])
def test_gate_table_matches_generators(oracle, name):
    rng = np.random.default_rng(7)
    for _ in range(5):
        p = _params(rng, name)
        got = oracle.gate_2x2(name, p)
        ref = brute.gate_matrix(name, p)
        assert np.max(np.abs(got - ref)) < 1e-14
        assert np.max(np.abs(got.conj().T @ got - np.eye(2))) < 1e-14


def test_textbook_identities(oracle):
    H = oracle.gate_2x2("h")
    assert np.allclose(H, np.array([[1, 1], [1, -1]]) / math.sqrt(2), atol=1e-15)
    X, Z = oracle.gate_2x2("x"), oracle.gate_2x2("z")
    assert np.allclose(H @ X @ H, Z, atol=1e-15)
    S, T = oracle.gate_2x2("s"), oracle.gate_2x2("t")
    assert np.allclose(S @ S, Z, atol=1e-15)
    assert np.allclose(T @ T, S, atol=1e-15)
    # RX(pi/2)^dagger Z RX(pi/2) = Y: the Y-basis change of the UCC compiler.
    R = oracle.gate_2x2("rx", (math.pi / 2,))
    assert np.allclose(R.conj().T @ Z @ R, oracle.gate_2x2("y"), atol=1e-15)
    # U3 special cases: U3(theta, 0, 0) = RY(theta); U3(0, 0, lam) = P(lam).
    assert np.allclose(oracle.gate_2x2("u3", (0.7, 0, 0)), oracle.gate_2x2("ry", (0.7,)), atol=1e-15)
    assert np.allclose(oracle.gate_2x2("u3", (0, 0, 0.3)), oracle.gate_2x2("p", (0.3,)), atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_single_qubit_vs_kronecker(oracle, n):
    """Algorithm 1 on every target equals the Eq. 2 Kronecker operator."""
    rng = np.random.default_rng(n)
    for k in range(n):
        for name in ("h", "u3", "rz", "y"):
            p = _params(rng, name)
            psi = qsynth.random_state(n, seed=100 * n + k)
            ref = brute.gate_operator(n, name, (k,), p) @ psi
            oracle.apply_gate(psi, n, name, (k,), p)
            assert np.max(np.abs(psi - ref)) < 1e-13


@pytest.mark.parametrize("n", [2, 3, 5, 6])
def test_controlled_vs_projector_form(oracle, n):
    """Algorithm 2 equals |0><0| (x) I + |1><1| (x) U for every (c, t),
    including c > t."""
    rng = np.random.default_rng(10 + n)
    for c in range(n):
        for t in range(n):
            if c == t:
                continue
            for name in ("cx", "cz", "cp", "cu"):
                p = _params(rng, name)
                psi = qsynth.random_state(n, seed=c * 31 + t)
                ref = brute.gate_operator(n, name, (c, t), p) @ psi
                oracle.apply_gate(psi, n, name, (c, t), p)
                assert np.max(np.abs(psi - ref)) < 1e-13


def test_controlled_touches_only_control_half(oracle):
    """Eq. 4: amplitudes with the control bit 0 are unchanged."""
    n, c, t = 6, 4, 1
    psi = qsynth.random_state(n, seed=3)
    before = psi.copy()
    oracle.apply_gate(psi, n, "cu", (c, t), (0.3, 1.1, -0.4))
    idx = np.arange(1 << n)
    assert np.array_equal(psi[(idx >> c) & 1 == 0], before[(idx >> c) & 1 == 0])
    assert not np.allclose(psi[(idx >> c) & 1 == 1], before[(idx >> c) & 1 == 1])


def test_swap_and_dense_vs_kronecker(oracle):
    rng = np.random.default_rng(5)
    n = 5
    for a in range(n):
        for b in range(n):
            if a == b:
                continue
            psi = qsynth.random_state(n, seed=a * 7 + b)
            ref = brute.gate_operator(n, "swap", (a, b)) @ psi
            oracle.apply_gate(psi, n, "swap", (a, b))
            assert np.max(np.abs(psi - ref)) < 1e-13
    for k in (1, 2, 3):
        for trial in range(4):
            qs = [int(q) for q in rng.choice(n, size=k, replace=False)]  # unsorted on purpose
            a = rng.normal(size=(1 << k, 1 << k)) + 1j * rng.normal(size=(1 << k, 1 << k))
            U, _ = np.linalg.qr(a)
            psi = qsynth.random_state(n, seed=trial)
            ref = brute.gate_operator(n, "dense", qs, (), U) @ psi
            oracle.apply_dense(psi, n, qs, U)
            assert np.max(np.abs(psi - ref)) < 1e-13


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_circuits_vs_brute(oracle, seed):
    n = 6
    c = qsynth.random_circuit(n, 60, seed=seed, max_dense=3)
    ref = brute.circuit_operator(c) @ oracle.zero_state(n)
    got = oracle.run(c)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_pair_index_sets(oracle):
    """The pairs a gate couples (Eq. 3, Eq. 4) against two other descriptions
    of the same set: a brute-force scan of all indices by their bits, and the
    grouped traversal of Section 2.2, where the index space is cut into
    groups of 2^(t+1) whose first half holds the lower members (for a control
    c < t, each half is cut again into runs of 2^c with the control bit in the
    odd runs).  The grouped form is written here as a reshape of the index
    array: group, half, run, parity of the run, position in the run."""
    n = 7
    idx = np.arange(1 << n)
    for t in range(n):
        got = oracle.pair_lows(n, t)
        assert len(got) == 1 << (n - 1)
        assert np.array_equal(got, idx[(idx >> t) & 1 == 0])
        grouped = idx.reshape(-1, 2, 1 << t)[:, 0, :].ravel()
        assert np.array_equal(got, grouped)
    for c in range(n):
        for t in range(n):
            if c == t:
                continue
            got = oracle.pair_lows(n, t, (c,))
            assert len(got) == 1 << (n - 2)
            assert np.array_equal(got, idx[((idx >> t) & 1 == 0) & ((idx >> c) & 1 == 1)])
            if c < t:
                grouped = idx.reshape(-1, 2, 1 << (t - c - 1), 2, 1 << c)[:, 0, :, 1, :].ravel()
                assert np.array_equal(got, grouped)
    # two controls: both bits set
    got = oracle.pair_lows(n, 3, (0, 5))
    assert np.array_equal(got, idx[((idx >> 3) & 1 == 0) & ((idx & 0b100001) == 0b100001)])


def test_kronecker_fusion_printed_entries(oracle):
    """M = M2 (x) M1 entries as printed in Section 3.4 (fixture), and the
    fused 4x4 applied with local bit 0 <-> t1 (lower qubit) equals M1 on t1
    followed by M2 on t2 (Eq. 6 ordering of the four amplitudes)."""
    rng = np.random.default_rng(11)
    a = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    b = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    M = np.kron(b, a)
    with open(os.path.join(GOLDEN, "kron_entries.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 16
    for r, c, ai, bi in rows:
        expect = a[int(ai[0]), int(ai[1])] * b[int(bi[0]), int(bi[1])]
        assert abs(M[int(r), int(c)] - expect) < 1e-15
    n, t1, t2 = 6, 1, 4
    psi = qsynth.random_state(n, seed=12)
    ref = psi.copy()
    oracle.apply_dense(ref, n, [t1], a)
    oracle.apply_dense(ref, n, [t2], b)
    oracle.apply_dense(psi, n, [t1, t2], M)
    assert np.max(np.abs(psi - ref)) < 1e-14


def test_same_qubit_and_cu_merge(oracle):
    """Section 3.4: two gates on the same qubit fuse to M2 M1; two CU gates
    with the same control and target fuse to CU(U2 U1)."""
    n = 5
    m1 = oracle.gate_2x2("u3", (0.4, 1.0, 2.0))
    m2 = oracle.gate_2x2("u3", (1.3, -0.5, 0.2))
    psi = qsynth.random_state(n, seed=1)
    ref = psi.copy()
    oracle.apply_gate(ref, n, "u3", (2,), (0.4, 1.0, 2.0))
    oracle.apply_gate(ref, n, "u3", (2,), (1.3, -0.5, 0.2))
    oracle.apply_dense(psi, n, [2], m2 @ m1)
    assert np.max(np.abs(psi - ref)) < 1e-14
    psi = qsynth.random_state(n, seed=2)
    ref = psi.copy()
    oracle.apply_gate(ref, n, "cu", (3, 0), (0.4, 1.0, 2.0))
    oracle.apply_gate(ref, n, "cu", (3, 0), (1.3, -0.5, 0.2))
    cu = np.eye(4, dtype=complex)
    cu[np.ix_([1, 3], [1, 3])] = m2 @ m1  # local bit 0 <-> control (qubit 3 listed first)
    oracle.apply_dense(psi, n, [3, 0], cu)
    assert np.max(np.abs(psi - ref)) < 1e-14


def test_opcount_model(oracle):
    with open(os.path.join(GOLDEN, "opcount.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    for k, coef, off in rows:
        for n in (10, 20, 30):
            assert oracle.opcount(n, int(k)) == int(coef) * 2.0 ** (n - int(off))
    # the fused two-qubit gate is cheaper than two one-qubit gates (9 vs 10 per 2^n)
    assert oracle.opcount(20, 2) < 2 * oracle.opcount(20, 1)
