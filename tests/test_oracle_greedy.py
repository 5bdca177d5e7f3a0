"""Pins of the oracle-side contraction rule (Section 3.4 DAG + greedy
merge, fixed-width reading) and of the block-product plan checker."""
import numpy as np
import pytest

import qsynth
from oracle import greedy


def _hand_circuit():
    c = qsynth.Circuit(4)
    c.add("h", (0,)).add("h", (1,)).add("h", (2,))          # g0 g1 g2
    c.add("cx", (0, 1)).add("cx", (1, 2))                    # g3 g4
    c.add("h", (3,)).add("rz", (0,), (0.3,))                 # g5 g6
    c.add("cx", (2, 3)).add("h", (1,)).add("cx", (1, 3))     # g7 g8 g9
    return c


def test_hand_worked_assignment():
    """Worked by hand from the rule with k_max = 2:
    g0,g1 open B1{0,1}; g2 -> B2{2}; g3 (f=1) -> B1; g4 (f=2) -> B2{1,2};
    g5 -> B3{3} (B1, B2 full); g6 (f=1) -> B1; g7 (f=3) -> B3{2,3};
    g8 (f=2) -> B2; g9 (f=3, B3 would need 3 qubits) -> B4{1,3}."""
    blocks = greedy.greedy_fw(_hand_circuit().gates, 2)
    assert blocks == [[0, 1, 3, 6], [2, 4, 8], [5, 7], [9]]


def test_width_one_keeps_only_same_qubit_runs():
    c = _hand_circuit()
    blocks = greedy.greedy_fw(c.gates, 1)
    for b in blocks:
        qs = greedy.block_qubits(c.gates, b)
        assert len(qs) == 1 or (len(b) == 1 and len(c.gates[b[0]].qubits) == 2)


@pytest.mark.parametrize("k_max", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("seed", [0, 1])
def test_blocks_reproduce_circuit(oracle, k_max, seed):
    """Executing the block products in block order equals the circuit
    (gate-by-gate) to rounding, and every per-qubit order is kept."""
    n = 9
    c = qsynth.random_circuit(n, 120, seed=seed, max_dense=2)
    blocks = greedy.greedy_fw(c.gates, k_max)
    greedy.check_order(c.gates, blocks)
    for b in blocks:
        assert len(greedy.block_qubits(c.gates, b)) <= max(k_max, max(len(c.gates[i].qubits) for i in b))
    qls = [greedy.block_qubits(c.gates, b) for b in blocks]
    mats = [greedy.block_matrix(c.gates, b) for b in blocks]
    for U in mats:
        assert np.max(np.abs(U.conj().T @ U - np.eye(U.shape[0]))) < 1e-12
    psi0 = qsynth.random_state(n, seed=seed)
    ref = oracle.run(c, psi0.copy())
    got = greedy.apply_blocks(psi0.copy(), n, qls, mats)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_order_checker_catches_swapped_gates():
    """The checker must reject a plan that swaps two gates sharing a qubit."""
    c = _hand_circuit()
    bad = [[0, 1, 6, 3], [2, 4, 8], [5, 7], [9]]
    with pytest.raises(AssertionError):
        greedy.check_order(c.gates, bad)


def test_ucc_exponential_compresses():
    """A weight-8 Pauli exponential (about 30 gates) contracts into a few
    blocks at k_max = 5 (8 qubits need at least two 5-qubit blocks, and the
    ladder forces the middle block); the compression ratio
    (N_before - N_after)/N_before of Section 4.3 is then far above the paper's
    52-63 % averages."""
    c = qsynth.Circuit(8)
    qsynth.pauli_exponential(c, [(q, "XYZXYZXY"[q]) for q in range(8)], 0.3)
    blocks = greedy.greedy_fw(c.gates, 5)
    ratio = (len(c.gates) - len(blocks)) / len(c.gates)
    assert 2 <= len(blocks) <= 4 and ratio > 0.8


# ---- commutation-aware rule (beyond Section 3.4's DAG) -----------------------

def test_diagonal_qubits_of_known_gates():
    """Phase-type gates are diagonal on their qubit, CZ / CP on both, a
    controlled gate on its control only; H, SWAP and U3 on none."""
    c = qsynth.Circuit(4)
    c.add("rz", (0,), (0.4,)).add("t", (1,)).add("cx", (2, 3)).add("cz", (0, 3))
    c.add("cp", (1, 2), (0.7,)).add("h", (0,)).add("swap", (1, 2)).add("u3", (3,), (0.1, 0.2, 0.3))
    c.add("cu", (3, 0), (0.5, 0.1, 0.2))
    got = [greedy.diagonal_qubits(c.gates, i) for i in range(len(c.gates))]
    assert got == [{0}, {1}, {2}, {0, 3}, {1, 2}, set(), set(), set(), {3}]


def test_commute_hand_worked():
    """Worked by hand with k_max = 1 (paper rule in brackets):
    (a) RZ0, CX(0,1), H1, RZ0: the last RZ0 commutes with CX's control and
        with RZ0, so f = 0 and it joins B1 -> [[0,3],[1],[2]]  ([[0],[1],[2],[3]]);
    (b) H0, CX(0,1), RZ0: f = B1 (H0 is not diagonal), RZ0 joins B1 after H0
        -> [[0,2],[1]]  ([[0],[1],[2]]);
    (c) RZ1, CX(0,1), RZ1: CX acts on its target non-diagonally, f = B2 and B2
        is too wide -> [[0],[1],[2]] (same as the paper rule)."""
    a = qsynth.Circuit(2).add("rz", (0,), (0.3,)).add("cx", (0, 1)).add("h", (1,)).add("rz", (0,), (0.5,))
    assert greedy.greedy_commute(a.gates, 1) == [[0, 3], [1], [2]]
    assert greedy.greedy_fw(a.gates, 1) == [[0], [1], [2], [3]]
    b = qsynth.Circuit(2).add("h", (0,)).add("cx", (0, 1)).add("rz", (0,), (0.2,))
    assert greedy.greedy_commute(b.gates, 1) == [[0, 2], [1]]
    c = qsynth.Circuit(2).add("rz", (1,), (0.2,)).add("cx", (0, 1)).add("rz", (1,), (0.4,))
    assert greedy.greedy_commute(c.gates, 1) == [[0], [1], [2]] == greedy.greedy_fw(c.gates, 1)


@pytest.mark.parametrize("k_max", [1, 2, 3, 4])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_commute_blocks_reproduce_circuit(oracle, k_max, seed):
    """Block products in block order equal the circuit from a random state;
    only commuting gates swap; the rule does swap some pairs (the plain
    order check fails) on these phase-heavy circuits."""
    n = 8
    c = qsynth.random_circuit(n, 160, seed=seed, kinds=["cx", "cz", "rz", "t", "h", "cp", "rx", "s"])
    blocks = greedy.greedy_commute(c.gates, k_max)
    greedy.check_order_commute(c.gates, blocks)
    qls = [greedy.block_qubits(c.gates, b) for b in blocks]
    mats = [greedy.block_matrix(c.gates, b) for b in blocks]
    psi0 = qsynth.random_state(n, seed=seed)
    ref = oracle.run(c, psi0.copy())
    got = greedy.apply_blocks(psi0.copy(), n, qls, mats)
    assert np.max(np.abs(got - ref)) < 1e-12
    if k_max <= 2:
        with pytest.raises(AssertionError):
            greedy.check_order(c.gates, blocks)


def test_commute_checker_catches_non_commuting_swap():
    """Swapping RZ on a CNOT's target with that CNOT must be rejected; the
    same swap on its control is allowed."""
    c = qsynth.Circuit(2).add("cx", (0, 1)).add("rz", (1,), (0.3,)).add("rz", (0,), (0.2,))
    greedy.check_order_commute(c.gates, [[2], [0], [1]])
    with pytest.raises(AssertionError):
        greedy.check_order_commute(c.gates, [[1], [0], [2]])


def test_commute_contracts_further():
    """Commuting gates past each other gives fewer blocks than the paper's
    rule on 16-qubit QAOA (ZZ terms as CX-RZ-CX: RZ and the CX controls
    commute across terms; 42 against 50 blocks at k_max 3) and on a
    phase-heavy random circuit, and never more on either."""
    for c, ks in ((qsynth.qaoa_maxcut(16), (3, 4)),
                  (qsynth.random_circuit(10, 200, seed=1, kinds=["cx", "cz", "rz", "t", "h", "cp", "rx", "s"]),
                   (2, 3, 4, 5))):
        for k in (2, 3, 4, 5):
            a, b = len(greedy.greedy_commute(c.gates, k)), len(greedy.greedy_fw(c.gates, k))
            assert a <= b
            if k in ks:
                assert a < b, (k, a, b)
