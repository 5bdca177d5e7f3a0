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


def apply_blocks(psi: np.ndarray, n: int, qubit_lists, matrices) -> np.ndarray:
    """Apply block matrices in order with the oracle's dense routine."""
    for qs, U in zip(qubit_lists, matrices):
        apply_dense(psi, n, list(qs), U)
    return psi
