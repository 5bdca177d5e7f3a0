"""Gate contraction rule and plan checker (TEST INFRASTRUCTURE ONLY).

Section 3.4 builds a DAG whose edges join gates that share a qubit (controls
count as operands), in program order, and then merges gates greedily; the
greedy rule itself is not spelled out.  The reading used here (fixed-width
greedy, "GREEDY-FW(k_max)"):

  walk the gates in program order; for gate g with qubit set Q_g let
  f = max over q in Q_g of last[q] (0 if none).  Put g into the lowest
  existing block j >= max(f, 1) with |Q_Bj u Q_g| <= k_max, else open a new
  block; then last[q] = j for q in Q_g.  A gate wider than k_max gets a block
  of its own.

Blocks after f share no qubit with g, so moving g in front of them only
reorders gates on disjoint qubits; executing blocks in index order therefore
gives the same state as the circuit (exact arithmetic).  Parity: pinned by
hand-worked assignments and by the block-product check below
(tests/test_oracle_greedy.py).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from . import apply_gate, apply_dense, zero_state


def greedy_fw(gates, k_max: int) -> List[List[int]]:
    """Block membership (lists of gate indices, program order inside each
    block) under GREEDY-FW(k_max)."""
    last = {}
    blocks: List[List[int]] = []
    qsets: List[set] = []
    for gi, g in enumerate(gates):
        Q = set(g.qubits)
        f = max((last.get(q, 0) for q in Q), default=0)
        j = None
        if len(Q) <= k_max:
            for cand in range(max(f, 1), len(blocks) + 1):
                if len(qsets[cand - 1] | Q) <= k_max:
                    j = cand
                    break
        if j is None:
            blocks.append([])
            qsets.append(set())
            j = len(blocks)
        blocks[j - 1].append(gi)
        qsets[j - 1] |= Q
        for q in Q:
            last[q] = j
    return blocks


def block_qubits(gates, members: Sequence[int]) -> Tuple[int, ...]:
    qs = set()
    for gi in members:
        qs |= set(gates[gi].qubits)
    return tuple(sorted(qs))


def block_matrix(gates, members: Sequence[int]) -> np.ndarray:
    """Product of the member gates (program order) on the block's own
    register: local bit j <-> j-th smallest qubit.  Column c is the image of
    basis state |c> under the member gates, each applied by the oracle's
    gate loops on a k-qubit register."""
    qs = block_qubits(gates, members)
    k = len(qs)
    loc = {q: j for j, q in enumerate(qs)}
    U = np.zeros((1 << k, 1 << k), dtype=np.complex128)
    for col in range(1 << k):
        v = zero_state(k)
        v[0] = 0.0
        v[col] = 1.0
        for gi in members:
            g = gates[gi]
            apply_gate(v, k, g.name, [loc[q] for q in g.qubits], g.params, g.matrix)
        U[:, col] = v
    return U


def check_order(gates, blocks: Sequence[Sequence[int]]) -> None:
    """Every pair of gates that share a qubit keeps its relative order
    under block-index execution (the DAG edges of Section 3.4); every gate
    appears exactly once."""
    where = {}
    for b, members in enumerate(blocks):
        for pos, gi in enumerate(members):
            assert gi not in where, f"gate {gi} in two blocks"
            where[gi] = (b, pos)
    assert sorted(where) == list(range(len(gates))), "gates missing from plan"
    last_on = {}
    for gi, g in enumerate(gates):
        for q in g.qubits:
            if q in last_on:
                prev = last_on[q]
                assert where[prev] < where[gi], f"order of gates {prev} and {gi} on qubit {q} broken"
            last_on[q] = gi


def diagonal_qubits(gates, gi: int) -> set:
    """Qubits on which gate gi acts diagonally: its matrix on its own qubits
    has no nonzero entry between basis states that differ in that qubit
    (it commutes with Z there; controls of controlled gates and every qubit
    of a phase or CZ gate are such qubits)."""
    U = block_matrix(gates, [gi])
    qs = block_qubits(gates, [gi])
    rows, cols = np.nonzero(U)
    return {q for j, q in enumerate(qs) if not np.any(((rows ^ cols) >> j) & 1)}


def greedy_commute(gates, k_max: int) -> List[List[int]]:
    """GREEDY-FW(k_max) with commutation (beyond Section 3.4's DAG, which
    orders every pair of gates sharing a qubit).

    Two gates that are both diagonal on every qubit they share commute: with
    S the shared qubits, each is a sum over basis states s of S of the
    projector |s><s| times an operator on its other qubits, and those other
    operators act on disjoint qubits.  So gate g need only follow the
    earlier gates that act non-diagonally on a qubit g is diagonal on, and
    every earlier gate on a qubit g acts on non-diagonally:

      f = max over q in Q_g of (last_nd[q] if g is diagonal on q else last[q]),

    g goes into the lowest existing block j >= max(f, 1) with
    |Q_Bj u Q_g| <= k_max, else into a new block; then last[q] and, where g
    is not diagonal on q, last_nd[q] become max(old, j).  Blocks in index
    order then put every pair of non-commuting gates in program order."""
    last, last_nd = {}, {}
    blocks: List[List[int]] = []
    qsets: List[set] = []
    for gi, g in enumerate(gates):
        Q = set(g.qubits)
        D = diagonal_qubits(gates, gi)
        f = max(((last_nd if q in D else last).get(q, 0) for q in Q), default=0)
        j = None
        if len(Q) <= k_max:
            for cand in range(max(f, 1), len(blocks) + 1):
                if len(qsets[cand - 1] | Q) <= k_max:
                    j = cand
                    break
        if j is None:
            blocks.append([])
            qsets.append(set())
            j = len(blocks)
        blocks[j - 1].append(gi)
        qsets[j - 1] |= Q
        for q in Q:
            last[q] = max(last.get(q, 0), j)
            if q not in D:
                last_nd[q] = max(last_nd.get(q, 0), j)
    return blocks


def check_order_commute(gates, blocks: Sequence[Sequence[int]]) -> None:
    """Like check_order, except that two gates may swap when both are
    diagonal on every qubit they share (they commute); every gate appears
    exactly once."""
    where = {}
    for b, members in enumerate(blocks):
        for pos, gi in enumerate(members):
            assert gi not in where, f"gate {gi} in two blocks"
            where[gi] = (b, pos)
    assert sorted(where) == list(range(len(gates))), "gates missing from plan"
    diag = [diagonal_qubits(gates, gi) for gi in range(len(gates))]
    on = {}
    for gi, g in enumerate(gates):
        for q in g.qubits:
            on.setdefault(q, []).append(gi)
    for q, seq in on.items():
        for i, a in enumerate(seq):
            for b in seq[i + 1:]:
                if where[a] > where[b]:
                    shared = set(gates[a].qubits) & set(gates[b].qubits)
                    assert all(s in diag[a] and s in diag[b] for s in shared), \
                        f"gates {a} and {b} swapped on qubit {q} without commuting"


def block_diagonal_qubits(U: np.ndarray, qubits, tol: float = 1e-14) -> set:
    """Qubits on which a block matrix (local bit j <-> qubits[j]) acts
    diagonally, entries below tol counting as zero (rounding residue of the
    product's exact zeros)."""
    rows, cols = np.nonzero(np.abs(U) > tol)
    return {q for j, q in enumerate(qubits) if not np.any(((rows ^ cols) >> j) & 1)}


def check_block_order_commute(gates, blocks: Sequence[Sequence[int]], qubit_lists, matrices) -> None:
    """Plan checker for plans whose blocks were reordered by commutation:
    every gate appears exactly once, and every pair of gates sharing a qubit
    whose program order the block order reverses either commutes itself (both
    gates diagonal on every qubit they share) or lies in two blocks that are
    both diagonal on every qubit the two blocks share."""
    where = {}
    for b, members in enumerate(blocks):
        for pos, gi in enumerate(members):
            assert gi not in where, f"gate {gi} in two blocks"
            where[gi] = (b, pos)
    assert sorted(where) == list(range(len(gates))), "gates missing from plan"
    gdiag = [diagonal_qubits(gates, gi) for gi in range(len(gates))]
    bdiag = [block_diagonal_qubits(U, qs) for qs, U in zip(qubit_lists, matrices)]
    on = {}
    for gi, g in enumerate(gates):
        for q in g.qubits:
            on.setdefault(q, []).append(gi)
    for q, seq in on.items():
        for i, a in enumerate(seq):
            for b in seq[i + 1:]:
                if where[a] < where[b]:
                    continue
                shared = set(gates[a].qubits) & set(gates[b].qubits)
                if all(s in gdiag[a] and s in gdiag[b] for s in shared):
                    continue
                ba, bb = where[a][0], where[b][0]
                bshared = set(qubit_lists[ba]) & set(qubit_lists[bb])
                assert all(s in bdiag[ba] and s in bdiag[bb] for s in bshared), \
                    f"gates {a} and {b} swapped on qubit {q} without commuting"


def apply_blocks(psi: np.ndarray, n: int, qubit_lists, matrices) -> np.ndarray:
    """Apply block matrices in order with the oracle's dense routine."""
    for qs, U in zip(qubit_lists, matrices):
        apply_dense(psi, n, list(qs), U)
    return psi
