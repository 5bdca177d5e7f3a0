"""Host-side checks of the C-ABI library (no GPU needed): every declared
symbol is exported, argument errors come back as status codes, and the host
planner (Section 3.4 contraction) agrees with the oracle's rule and block
products."""
import os
import re

import numpy as np
import pytest

import qsynth
from oracle import greedy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def Q():
    from paper_2509_04955_amd import qsim

    qsim.lib()
    return qsim


def test_every_declared_symbol_is_exported(Q):
    with open(os.path.join(ROOT, "include", "qsim.h")) as f:
        text = f.read()
    declared = set(re.findall(r"^\s*(?:qs_status|const char \*|int)\s*(qs_\w+)\s*\(", text, re.M))
    assert len(declared) >= 30
    L = Q.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert declared <= set(Q.exported_symbols())


def test_gate_struct_layout(Q):
    import ctypes

    assert ctypes.sizeof(Q.qs_gate) == 80
    assert ctypes.sizeof(Q.qs_contract_opts) == 32


def _plan(Q, c, **kw):
    gl = Q.GateList(c)
    return Q.qs_contract(c.n, gl, Q.opts(**kw)), gl


@pytest.mark.parametrize("k_max", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_greedy_membership_matches_oracle(Q, k_max, seed):
    """Block membership is integer work: it must equal the oracle's rule
    exactly, block by block."""
    c = qsynth.random_circuit(11, 200, seed=seed)
    plan, _ = _plan(Q, c, k_max=k_max, tile_qubits=11)
    try:
        info = Q.qs_plan_info_get(plan)
        ref = greedy.greedy_fw(c.gates, k_max)
        assert info.n_blocks == len(ref)
        for b, members in enumerate(ref):
            qs, _, mem = Q.qs_plan_block(plan, b, with_matrix=False)
            assert mem == members
            assert qs == greedy.block_qubits(c.gates, members)
    finally:
        Q.qs_plan_destroy(plan)


@pytest.mark.parametrize("k_max", [2, 4, 5])
def test_block_products_match_oracle(Q, oracle, k_max):
    """FP64 block matrices agree with the oracle's own composition, and the
    blocks applied in order reproduce the circuit (plan checker)."""
    n = 10
    c = qsynth.random_circuit(n, 150, seed=7, max_dense=3)
    plan, _ = _plan(Q, c, k_max=k_max, tile_qubits=10)
    try:
        info = Q.qs_plan_info_get(plan)
        qls, mats, blocks = [], [], []
        for b in range(info.n_blocks):
            qs, U, mem = Q.qs_plan_block(plan, b)
            ref = greedy.block_matrix(c.gates, mem)
            assert np.max(np.abs(U - ref)) < 1e-13
            qls.append(qs)
            mats.append(U)
            blocks.append(mem)
        greedy.check_order(c.gates, blocks)
        psi0 = qsynth.random_state(n, seed=3)
        ref = oracle.run(c, psi0.copy())
        got = greedy.apply_blocks(psi0.copy(), n, qls, mats)
        assert np.max(np.abs(got - ref)) < 1e-12
    finally:
        Q.qs_plan_destroy(plan)


@pytest.mark.parametrize("k_max,t,c", [(2, 5, 1), (3, 6, 2), (4, 8, 3), (5, 9, 4)])
def test_pass_packing_reorders_blocks_validly(Q, oracle, k_max, t, c):
    """With tiles smaller than the register the packer pulls later blocks on
    other qubits into earlier passes: the blocks are the oracle's greedy
    blocks as sets, every pair of gates on a shared qubit keeps its order
    (the DAG edges of Section 3.4), and the blocks in plan order reproduce
    the circuit."""
    n = 12
    circ = qsynth.random_circuit(n, 300, seed=0, max_dense=2)
    plan, _ = _plan(Q, circ, k_max=k_max, tile_qubits=t, low_qubits=c)
    try:
        info = Q.qs_plan_info_get(plan)
        ref = greedy.greedy_fw(circ.gates, k_max)
        qls, mats, blocks = [], [], []
        for b in range(info.n_blocks):
            qs, U, mem = Q.qs_plan_block(plan, b)
            qls.append(qs)
            mats.append(U)
            blocks.append(mem)
        assert sorted(map(tuple, blocks)) == sorted(map(tuple, ref))
        assert blocks != ref, "expected the packer to move blocks at this tile size"
        greedy.check_order(circ.gates, blocks)
        psi0 = qsynth.random_state(n, seed=5)
        want = oracle.run(circ, psi0.copy())
        got = greedy.apply_blocks(psi0.copy(), n, qls, mats)
        assert np.max(np.abs(got - want)) < 1e-12
    finally:
        Q.qs_plan_destroy(plan)


@pytest.mark.parametrize("t,c", [(8, 3), (10, 6), (13, 6)])
def test_passes_cover_blocks(Q, t, c):
    circ, _ = qsynth.ucc(24, n_exp=40, seed=4)
    plan, _ = _plan(Q, circ, k_max=5, tile_qubits=t, low_qubits=c)
    try:
        info = Q.qs_plan_info_get(plan)
        nxt = 0
        for i in range(info.n_passes):
            tt, tile, fb, nb = Q.qs_plan_pass(plan, i)
            assert tt == t and len(tile) == t and list(tile) == sorted(set(tile))
            assert set(range(min(c, t - 5))) <= set(tile)
            assert fb == nxt and nb >= 1
            nxt += nb
            for b in range(fb, fb + nb):
                qs, _, _ = Q.qs_plan_block(plan, b, with_matrix=False)
                assert set(qs) <= set(tile)
        assert nxt == info.n_blocks
    finally:
        Q.qs_plan_destroy(plan)


@pytest.mark.parametrize("k_max,t", [(1, 6), (2, 6), (5, 6), (3, 4)])
def test_pass_tiles_hold_wide_gates(Q, k_max, t):
    """Gates wider than k_max (two-qubit gates at k_max = 1) are blocks of
    their own; every pass tile must still hold t qubits including qubit 0."""
    c = qsynth.random_circuit(12, 150, seed=k_max, max_dense=2)
    plan, _ = _plan(Q, c, k_max=k_max, tile_qubits=t)
    try:
        info = Q.qs_plan_info_get(plan)
        for i in range(info.n_passes):
            tt, tile, fb, nb = Q.qs_plan_pass(plan, i)
            assert len(tile) == t and 0 in tile
            for b in range(fb, fb + nb):
                assert set(Q.qs_plan_block(plan, b, with_matrix=False)[0]) <= set(tile)
    finally:
        Q.qs_plan_destroy(plan)


def test_block_wider_than_tile_rejected(Q):
    c = qsynth.random_circuit(14, 50, seed=1)
    with pytest.raises(Q.QsimError) as ei:
        _plan(Q, c, k_max=5, tile_qubits=5)
    assert ei.value.status == Q.QS_EINVAL


def test_strategy_none_is_one_block_per_gate(Q):
    c = qsynth.random_circuit(8, 50, seed=1)
    plan, _ = _plan(Q, c, strategy=Q.STRATEGY_NONE, tile_qubits=8)
    try:
        info = Q.qs_plan_info_get(plan)
        assert info.n_blocks == 50
        for b in range(50):
            assert Q.qs_plan_block(plan, b, with_matrix=False)[2] == [b]
    finally:
        Q.qs_plan_destroy(plan)


@pytest.mark.parametrize("bad", [
    ("h", (12,)), ("cx", (3, 3)), ("cx", (1,)), ("u3", (-1,)),
])
def test_invalid_gates_rejected(Q, bad):
    c = qsynth.Circuit(12).add("h", (0,)).add(bad[0], bad[1], (0.1, 0.2, 0.3)[: qsynth.N_PARAMS.get(bad[0], 0)])
    with pytest.raises(Q.QsimError) as ei:
        _plan(Q, c)
    assert ei.value.status == Q.QS_EINVAL
    assert "gate 1" in str(ei.value)


def test_bad_options_rejected(Q):
    c = qsynth.ghz(8)
    for kw in ({"k_max": 7}, {"tile_qubits": 15}, {"k_max": 6, "dtype": Q.QS_C128}):
        with pytest.raises(Q.QsimError):
            _plan(Q, c, **kw)


def test_compression_on_paper_style_circuit(Q):
    """HEA-like circuit (Section 4.1): greedy contraction removes most gates
    (the paper reports 52-63 % average compression)."""
    c = qsynth.hea(20, layers=5, seed=(9, 0))
    plan, _ = _plan(Q, c, k_max=5)
    try:
        info = Q.qs_plan_info_get(plan)
        ratio = (info.n_gates - info.n_blocks) / info.n_gates
        assert ratio > 0.5
        assert info.max_k <= 5
    finally:
        Q.qs_plan_destroy(plan)


def test_pass_features_on_host(Q):
    """Pass features are host-side: a CNOT/CZ-only circuit gives only
    monomial blocks; a dense-U3 circuit at k_max = 5 gives MFMA-width blocks."""
    from paper_2509_04955_amd import costmodel

    F = Q.lib().qs_costmodel_num_features()
    mono = qsynth.random_circuit(20, 80, seed=3, kinds=["cx", "cz", "rz"])
    plan, _ = _plan(Q, mono, k_max=3, tile_qubits=12)
    try:
        f = costmodel.pass_features(plan)
        assert f.shape == (Q.qs_plan_info_get(plan).n_passes, F)
        assert np.all(f[:, 10] > 0) and np.all(f[:, 5:10] == 0)   # only monomial blocks
        assert np.allclose(f[:, 0], 20 / 32) and np.allclose(f[:, 1], 12 / 16)
    finally:
        Q.qs_plan_destroy(plan)
    dense = qsynth.brickwork(20, 6, seed=1)
    plan, _ = _plan(Q, dense, k_max=5, tile_qubits=12)
    try:
        f = costmodel.pass_features(plan)
        assert np.sum(f[:, 8] + f[:, 9]) > 0   # k = 4, 5 dense blocks -> MFMA kind
    finally:
        Q.qs_plan_destroy(plan)


def _class_width(U):
    """log2 of the narrowest packing of U's nonzero pattern into equal
    classes: connected components of the row/column graph, first fit by
    decreasing size into 2^s-wide bins."""
    D = U.shape[0]
    nz = np.abs(U) > 1e-14
    comp = list(range(2 * D))

    def find(x):
        while comp[x] != x:
            x = comp[x]
        return x

    for r, col in zip(*np.nonzero(nz)):
        comp[find(r)] = find(D + col)
    sizes = {}
    for r in range(D):
        sizes[find(r)] = sizes.get(find(r), 0) + 1
    sizes = sorted(sizes.values(), reverse=True)
    s = int(np.ceil(np.log2(sizes[0])))
    while True:
        bins = [0] * (D >> s)
        ok = True
        for z in sizes:
            j = next((j for j, b in enumerate(bins) if b + z <= 1 << s), None)
            if j is None:
                ok = False
                break
            bins[j] += z
        if ok:
            return s
        s += 1


@pytest.mark.parametrize("k_max", [3, 4, 5])
def test_block_diagonal_classification(Q, k_max):
    """The planner marks a 3- or 4-qubit block permuted block-diagonal when
    its nonzero pattern packs into classes narrower than the block and wider
    than one; 4-qubit monomial blocks (classes of one) take the same path."""
    from paper_2509_04955_amd import costmodel

    c = qsynth.random_circuit(16, 400, seed=k_max, kinds=["cx", "cz", "rz", "t", "x", "h", "ry"])
    plan, _ = _plan(Q, c, k_max=k_max, tile_qubits=12)
    try:
        info = Q.qs_plan_info_get(plan)
        want = 0
        for b in range(info.n_blocks):
            qs, U, _ = Q.qs_plan_block(plan, b)
            s = _class_width(U)
            want += int(len(qs) in (3, 4) and 1 <= s < len(qs)) + int(len(qs) == 4 and s == 0)
        f = costmodel.pass_features(plan)
        assert want > 0
        assert round(float(f[:, 16].sum()) * 8) == want
    finally:
        Q.qs_plan_destroy(plan)


def test_learned_strategy_without_model_falls_back_to_greedy(Q):
    c = qsynth.random_circuit(12, 100, seed=2)
    a, _ = _plan(Q, c, k_max=4, tile_qubits=10)
    b, _ = _plan(Q, c, k_max=4, tile_qubits=10, strategy=Q.STRATEGY_LEARNED)
    try:
        ia, ib = Q.qs_plan_info_get(a), Q.qs_plan_info_get(b)
        assert ia.n_blocks == ib.n_blocks and ia.n_passes == ib.n_passes
        for i in range(ia.n_blocks):
            assert Q.qs_plan_block(a, i, False)[2] == Q.qs_plan_block(b, i, False)[2]
    finally:
        Q.qs_plan_destroy(a)
        Q.qs_plan_destroy(b)


def _pauli_matrix(qs, x, z, theta):
    """exp(-i theta P) on the qubits qs (local bit j <-> qs[j]) for the Pauli
    string with X part x and Z part z: cos(theta) I - i sin(theta) P with
    P|j> = i^|x&z| (-1)^|j&z| |j ^ x>."""
    D = 1 << len(qs)
    lx = sum(1 << j for j, q in enumerate(qs) if (x >> q) & 1)
    lz = sum(1 << j for j, q in enumerate(qs) if (z >> q) & 1)
    P = np.zeros((D, D), dtype=np.complex128)
    for j in range(D):
        P[j ^ lx, j] = (1j) ** bin(lx & lz).count("1") * (-1) ** bin(j & lz).count("1")
    return np.cos(theta) * np.eye(D) - 1j * np.sin(theta) * P


@pytest.mark.parametrize("n,t", [(12, 10), (16, 13), (20, 9)])
def test_pauli_strategy_recovers_the_rotations(Q, oracle, n, t):
    """The Pauli strategy contracts each exponential of a UCC circuit (basis
    changes, CNOT ladder, RZ, ladder and basis changes undone) into one block
    whose matrix is the rotation the generator drew, exp(-i theta P); blocks
    sharing a qubit run out of program order only when their strings commute,
    and the blocks in plan order reproduce the circuit (plan checker)."""
    c, rots = qsynth.ucc(n, n_exp=30, seed=n)
    plan, _ = _plan(Q, c, k_max=4, tile_qubits=t, low_qubits=1, strategy=Q.STRATEGY_PAULI)
    try:
        info = Q.qs_plan_info_get(plan)
        assert info.n_blocks == len(rots)
        qls, mats, mems = [], [], []
        for b in range(info.n_blocks):
            qs, U, mem = Q.qs_plan_block(plan, b)
            qls.append(qs)
            mats.append(U)
            mems.append(mem)
        rot_of = {}
        for e, b in enumerate(sorted(range(len(mems)), key=lambda b: mems[b][0])):
            x, z, theta = rots[e]
            assert np.max(np.abs(mats[b] - _pauli_matrix(qls[b], x, z, theta))) < 1e-13
            rot_of[b] = (x, z)
        swapped = 0
        for a in range(len(mems)):
            for b in range(a + 1, len(mems)):
                if set(qls[a]) & set(qls[b]) and mems[a][0] > mems[b][0]:
                    (xa, za), (xb, zb) = rot_of[a], rot_of[b]
                    assert (bin(xa & zb).count("1") + bin(za & xb).count("1")) % 2 == 0
                    swapped += 1
        psi0 = qsynth.random_state(n, seed=3)
        ref = oracle.run(c, psi0.copy())
        got = greedy.apply_blocks(psi0.copy(), n, qls, mats)
        assert np.max(np.abs(got - ref)) < 1e-12
    finally:
        Q.qs_plan_destroy(plan)


def test_pauli_strategy_on_mixed_circuits(Q, oracle):
    """Rotation windows inside other gates: a random circuit, a UCC segment and
    a brickwork segment back to back.  Windows are found only where a run
    multiplies to a rotation; everything else is contracted greedily, and the
    plan reproduces the circuit."""
    n = 10
    parts = [qsynth.random_circuit(n, 60, seed=1), qsynth.ucc(n, n_exp=8, seed=2)[0], qsynth.brickwork(n, 3, seed=3),
             qsynth.ucc(n, n_exp=5, seed=4)[0]]
    c = qsynth.Circuit(n, [g for p in parts for g in p.gates])
    plan, _ = _plan(Q, c, k_max=3, tile_qubits=9, strategy=Q.STRATEGY_PAULI)
    try:
        info = Q.qs_plan_info_get(plan)
        qls, mats, mems = [], [], []
        for b in range(info.n_blocks):
            qs, U, mem = Q.qs_plan_block(plan, b)
            qls.append(qs)
            mats.append(U)
            mems.append(mem)
        assert sum(1 for q in qls if len(q) > 3) >= 1   # at least one contracted rotation wider than k_max
        greedy.check_order(c.gates, mems)
        psi0 = qsynth.random_state(n, seed=4)
        ref = oracle.run(c, psi0.copy())
        got = greedy.apply_blocks(psi0.copy(), n, qls, mats)
        assert np.max(np.abs(got - ref)) < 1e-12
    finally:
        Q.qs_plan_destroy(plan)


def test_unknown_strategy_rejected(Q):
    with pytest.raises(Q.QsimError):
        _plan(Q, qsynth.ghz(6), strategy=7)


def test_pauli_strategy_without_windows_is_greedy(Q):
    """Circuits with no run equal to a rotation (random U3 + CNOT, QFT) get the
    greedy plan's blocks under the Pauli strategy."""
    for c in (qsynth.random_u3_cnot(12, 6, seed=3), qsynth.qft(10)):
        a, _ = _plan(Q, c, k_max=4, tile_qubits=9)
        b, _ = _plan(Q, c, k_max=4, tile_qubits=9, strategy=Q.STRATEGY_PAULI)
        try:
            na, nb = Q.qs_plan_info_get(a).n_blocks, Q.qs_plan_info_get(b).n_blocks
            assert na == nb
            ma = sorted(tuple(Q.qs_plan_block(a, i, False)[2]) for i in range(na))
            mb = sorted(tuple(Q.qs_plan_block(b, i, False)[2]) for i in range(nb))
            assert ma == mb
        finally:
            Q.qs_plan_destroy(a)
            Q.qs_plan_destroy(b)


@pytest.mark.parametrize("t", [9, 12, 14])
def test_pauli_plan_tiles_hold_x_supports(Q, t):
    """Every pass tile holds qubit 0 and the X part of each rotation block in
    it (the Z part may lie outside), and pass ranges cover the blocks."""
    n = 20
    c, rots = qsynth.ucc(n, n_exp=60, seed=t)
    plan, _ = _plan(Q, c, k_max=4, tile_qubits=t, low_qubits=2, strategy=Q.STRATEGY_PAULI)
    try:
        info = Q.qs_plan_info_get(plan)
        mems = [Q.qs_plan_block(plan, b, False)[2] for b in range(info.n_blocks)]
        start = sorted(range(len(mems)), key=lambda b: mems[b][0])
        xmask = {b: rots[e][0] for e, b in enumerate(start)}
        nxt = 0
        for i in range(info.n_passes):
            tt, tile, fb, nb = Q.qs_plan_pass(plan, i)
            assert fb == nxt and nb >= 1 and 0 in tile and len(tile) == t
            nxt += nb
            tmask = sum(1 << q for q in tile)
            for b in range(fb, fb + nb):
                assert xmask[b] & ~tmask == 0
        assert nxt == info.n_blocks
    finally:
        Q.qs_plan_destroy(plan)


# ---- commutation-aware contraction (the commute option) ----------------------

PHASE_HEAVY = ["cx", "cz", "rz", "t", "h", "cp", "rx", "s", "u3"]


@pytest.mark.parametrize("k_max", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_commute_membership_matches_oracle(Q, k_max, seed):
    """Block membership under the commute option equals the oracle's
    commutation-aware rule exactly (integer work)."""
    c = qsynth.random_circuit(11, 180, seed=seed, kinds=PHASE_HEAVY)
    plan, _ = _plan(Q, c, k_max=k_max, tile_qubits=10, commute=1)
    try:
        info = Q.qs_plan_info_get(plan)
        got = sorted(tuple(Q.qs_plan_block(plan, b, False)[2]) for b in range(info.n_blocks))
    finally:
        Q.qs_plan_destroy(plan)
    assert got == sorted(tuple(b) for b in greedy.greedy_commute(c.gates, k_max))


@pytest.mark.parametrize("family", ["qft", "qaoa", "phase"])
@pytest.mark.parametrize("k_max", [2, 3, 4])
def test_commute_plan_replays_exactly(Q, oracle, family, k_max):
    """Plan checker for commute plans (blocks also reordered by the pass
    packer where they commute): every reversed pair of gates commutes itself
    or sits in two blocks diagonal on every qubit they share, and the block
    matrices in plan order reproduce the oracle's state from a random state."""
    n = 11
    c = {"qft": lambda: qsynth.qft(n), "qaoa": lambda: qsynth.qaoa_maxcut(n),
         "phase": lambda: qsynth.random_circuit(n, 200, seed=k_max, kinds=PHASE_HEAVY)}[family]()
    plan, _ = _plan(Q, c, k_max=k_max, tile_qubits=8, low_qubits=2, commute=1)
    try:
        info = Q.qs_plan_info_get(plan)
        qls, mats, mems = [], [], []
        for b in range(info.n_blocks):
            qs, U, mem = Q.qs_plan_block(plan, b)
            qls.append(qs)
            mats.append(U)
            mems.append(mem)
    finally:
        Q.qs_plan_destroy(plan)
    greedy.check_block_order_commute(c.gates, mems, qls, mats)
    psi0 = qsynth.random_state(n, seed=3)
    ref = oracle.run(c, psi0.copy())
    got = greedy.apply_blocks(psi0.copy(), n, qls, mats)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_commute_needs_fewer_passes_on_qft(Q):
    """30-qubit QFT at t = 13: its controlled phases commute with each other,
    so the commute option packs them into fewer passes (20 against 25 at
    k_max 4, 27 against 34 at k_max 3)."""
    c = qsynth.qft(30)
    for k, want in ((3, (27, 34)), (4, (20, 25))):
        got = []
        for cm in (1, 0):
            plan, _ = _plan(Q, c, k_max=k, tile_qubits=13, low_qubits=4, commute=cm)
            got.append(int(Q.qs_plan_info_get(plan).n_passes))
            Q.qs_plan_destroy(plan)
        assert tuple(got) == want


def test_commute_flag_validated(Q):
    with pytest.raises(Q.QsimError):
        _plan(Q, qsynth.ghz(6), commute=2)


@pytest.mark.parametrize("strategy", ["greedy", "pauli", "none"])
def test_commute_with_every_strategy_replays_exactly(Q, oracle, strategy):
    """The commute option combined with the rotation contraction (rotation
    blocks and diagonal blocks passing each other in the packer) and with
    one block per gate: the plan still reproduces the circuit exactly."""
    n = 10
    parts = [qsynth.ucc(n, n_exp=6, seed=5)[0], qsynth.qaoa_maxcut(n), qsynth.qft(n)]
    c = qsynth.Circuit(n, [g for p in parts for g in p.gates])
    st = {"greedy": Q.STRATEGY_GREEDY, "pauli": Q.STRATEGY_PAULI, "none": Q.STRATEGY_NONE}[strategy]
    plan, _ = _plan(Q, c, k_max=3, tile_qubits=9, low_qubits=1, strategy=st, commute=1)
    try:
        info = Q.qs_plan_info_get(plan)
        qls, mats, mems = [], [], []
        for b in range(info.n_blocks):
            qs, U, mem = Q.qs_plan_block(plan, b)
            qls.append(qs)
            mats.append(U)
            mems.append(mem)
    finally:
        Q.qs_plan_destroy(plan)
    assert sorted(g for m in mems for g in m) == list(range(len(c.gates)))
    psi0 = qsynth.random_state(n, seed=6)
    ref = oracle.run(c, psi0.copy())
    got = greedy.apply_blocks(psi0.copy(), n, qls, mats)
    assert np.max(np.abs(got - ref)) < 1e-12
