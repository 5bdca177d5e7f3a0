"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Tolerances: complex128 paths max-abs <= 1e-12 (FP64 arithmetic, a few hundred
gates of unit-norm amplitudes).  complex64 paths: each amplitude update adds
a relative rounding error of about 2^-24 per gate or block; over the circuits
here (<= a few thousand gates) the accumulated error stays below 1e-5 in
max-abs and 1 - fidelity below 1e-6, which are the bounds written in the
tests (the headline requirement is fidelity >= 1 - 1e-5)."""
import math

import numpy as np
import pytest

import qsynth

pytestmark = pytest.mark.gpu

TOL128 = 1e-12
TOL64 = 1e-5


@pytest.fixture(scope="module")
def Q():
    import torch

    from paper_2509_04955_amd import qsim

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    qsim.lib()
    return qsim


def run_plain(Q, c, dtype, psi0=None):
    s = Q.State(c.n, dtype)
    if psi0 is not None:
        s.load(psi0)
    s.apply_gates(Q.GateList(c))
    out = s.amplitudes()
    s.close()
    return out


def run_plan(Q, c, dtype, psi0=None, **kw):
    kw.setdefault("dtype", dtype)
    gl = Q.GateList(c)
    plan = Q.qs_contract(c.n, gl, Q.opts(**kw))
    s = Q.State(c.n, dtype)
    if psi0 is not None:
        s.load(psi0)
    s.apply_plan(plan)
    out = s.amplitudes()
    nrm = s.norm()
    s.close()
    Q.qs_plan_destroy(plan)
    return out, nrm


def test_device_is_gfx950(Q):
    cu, lds, arch = Q.qs_device_query()
    assert arch.startswith("gfx950"), arch
    assert cu >= 1 and lds >= 65536


def test_plain_c128_random_12q(Q, oracle):
    """12-qubit random circuit, 20 layers of H/RZ plus 6 CNOTs, complex128,
    gate-by-gate: max-abs <= 1e-12 against the oracle."""
    c = qsynth.plain_random(12, 20, 6, seed=1)
    ref = oracle.run(c)
    got = run_plain(Q, c, Q.QS_C128)
    assert oracle.max_abs(ref, got) <= TOL128


@pytest.mark.parametrize("dtype,tol", [(0, TOL64), (1, TOL128)])
@pytest.mark.parametrize("n", [1, 2, 3, 7, 9])
def test_plain_every_kind_every_qubit(Q, oracle, dtype, tol, n):
    rng = np.random.default_rng(n)
    c = qsynth.Circuit(n)
    for q in range(n):
        for name in qsynth.ONE_QUBIT:
            c.add(name, (q,), tuple(rng.random() * 6 for _ in range(qsynth.N_PARAMS.get(name, 0))))
    if n >= 2:
        for a in range(n):
            for b in range(n):
                if a != b:
                    for name in qsynth.TWO_QUBIT:
                        c.add(name, (a, b), tuple(rng.random() * 6 for _ in range(qsynth.N_PARAMS.get(name, 0))))
    psi0 = qsynth.random_state(n, seed=n)
    ref = oracle.run(c, psi0.copy())
    got = run_plain(Q, c, dtype, psi0)
    assert oracle.max_abs(ref, got) <= tol * max(1, len(c) / 100)


@pytest.mark.parametrize("dtype,tol", [(0, TOL64), (1, TOL128)])
def test_plain_low_controls_18q(Q, oracle, dtype, tol):
    # controls 0..3 against every target: the whole-vector sweep of the
    # complex64 controlled kernels, over many workgroups and grid strides
    n = 18
    rng = np.random.default_rng(7)
    c = qsynth.Circuit(n)
    for ctl in range(4):
        for tgt in range(n):
            if tgt != ctl:
                for name in qsynth.TWO_QUBIT:
                    c.add(name, (ctl, tgt), tuple(rng.random() * 6 for _ in range(qsynth.N_PARAMS.get(name, 0))))
    psi0 = qsynth.random_state(n, seed=5)
    ref = oracle.run(c, psi0.copy())
    got = run_plain(Q, c, dtype, psi0)
    assert oracle.max_abs(ref, got) <= tol * max(1, len(c) / 100)


@pytest.mark.parametrize("dtype,tol", [(0, TOL64), (1, TOL128)])
def test_plain_dense_gates(Q, oracle, dtype, tol):
    n = 8
    c = qsynth.random_circuit(n, 40, seed=3, kinds=["h", "cx"], max_dense=5 if dtype == 1 else 6)
    psi0 = qsynth.random_state(n, seed=2)
    ref = oracle.run(c, psi0.copy())
    got = run_plain(Q, c, dtype, psi0)
    assert oracle.max_abs(ref, got) <= tol


@pytest.mark.parametrize("k_max", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("t", [6, 9, 10, 11, 12, 13])
def test_fused_c64_random(Q, oracle, k_max, t):
    """Fused tile passes, complex64: VALU blocks (k <= 3) and MFMA blocks
    (k = 4, 5) over several tiles and ragged pass boundaries; every tile size
    from a partial workgroup (t = 6) to 16 vectors per thread (t = 13)."""
    n = 14
    if k_max > t - 1:
        pytest.skip("block wider than tile")
    c = qsynth.random_circuit(n, 300, seed=10 + k_max, max_dense=2)
    psi0 = qsynth.random_state(n, seed=5)
    ref = oracle.run(c, psi0.copy())
    got, nrm = run_plan(Q, c, Q.QS_C64, psi0, k_max=k_max, tile_qubits=t)
    assert oracle.max_abs(ref, got) <= TOL64
    assert 1 - oracle.fidelity(ref, got) <= 1e-6
    assert abs(nrm - 1) <= 1e-6


@pytest.mark.parametrize("k_max", [1, 3, 5])
@pytest.mark.parametrize("t", [7, 8, 9, 10, 11, 12])
def test_fused_c128_random(Q, oracle, k_max, t):
    n = 13
    c = qsynth.random_circuit(n, 250, seed=20 + k_max, max_dense=2)
    psi0 = qsynth.random_state(n, seed=6)
    ref = oracle.run(c, psi0.copy())
    got, _ = run_plan(Q, c, Q.QS_C128, psi0, k_max=k_max, tile_qubits=t)
    assert oracle.max_abs(ref, got) <= TOL128


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("low", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("t", [11, 12, 13])
def test_fused_low_qubit_counts(Q, oracle, dtype, low, t):
    """Tiles with 1..5 fixed contiguous low qubits (shorter coalesced runs,
    more free high-qubit slots) give the same state."""
    if dtype == 1 and t > 12:
        pytest.skip("complex128 tiles stop at t = 12")
    n = 15
    c, _ = qsynth.ucc(n, 12, seed=50 + low)
    psi0 = qsynth.random_state(n, seed=9)
    ref = oracle.run(c, psi0.copy())
    got, _ = run_plan(Q, c, dtype, psi0, k_max=4, tile_qubits=t, low_qubits=low)
    assert oracle.max_abs(ref, got) <= (TOL64 if dtype == 0 else TOL128)


@pytest.mark.parametrize("n5,n3", [(1, 2), (0, 6), (3, 0), (2, 3)])
@pytest.mark.parametrize("t", [11, 12, 13, 14])
def test_fused_mfma_operands_staged_or_not(Q, oracle, n5, n3, t):
    """Passes whose MFMA operands fit the LDS left beside the tile (a dense
    5-qubit block is 12 KB in the three-product form, 16 KB embedded as in
    the 512-thread workgroups of 2^13 tiles; 3-qubit blocks 1 KB) stage them
    there and also run 3-qubit blocks on MFMA; passes over the budget (and
    every 2^14 tile) read them from the pool.  Both give the oracle's state."""
    n = 15
    rng = np.random.default_rng(100 * n5 + n3 + t)

    def unitary(k):
        a = rng.normal(size=(1 << k, 1 << k)) + 1j * rng.normal(size=(1 << k, 1 << k))
        return np.linalg.qr(a)[0]

    c = qsynth.Circuit(n)
    hi = list(range(6, n))
    for _ in range(2):
        for k, cnt in ((5, n5), (3, n3)):
            for _ in range(cnt):
                qs = sorted(int(x) for x in rng.choice(list(range(6)) + hi[: t - 6], size=k, replace=False))
                c.add("dense", qs, (), unitary(k))
    psi0 = qsynth.random_state(n, seed=11)
    ref = oracle.run(c, psi0.copy())
    got, nrm = run_plan(Q, c, Q.QS_C64, psi0, k_max=5, tile_qubits=t)
    assert oracle.max_abs(ref, got) <= TOL64
    assert 1 - oracle.fidelity(ref, got) <= 1e-6


@pytest.mark.parametrize("dtype,k,t", [(0, 6, 10), (0, 6, 12), (0, 6, 13), (0, 5, 12),
                                       (1, 4, 12), (1, 5, 9), (1, 5, 11), (1, 5, 12)])
def test_wide_dense_blocks_on_matrix_cores(Q, oracle, dtype, k, t):
    """Dense blocks wider than the LDS-staged forms: complex64 6-qubit blocks
    (128x128 real embedding, two M-tiles per wave) and complex128 4- and
    5-qubit blocks in passes whose operands are not staged run on the matrix
    cores in the wide kernel variant.  The pass features must count them as
    MFMA blocks and none as a wide vector-ALU block; the state must match
    the oracle."""
    from paper_2509_04955_amd import costmodel

    n = 15
    rng = np.random.default_rng(1000 * dtype + 10 * k + t)

    def unitary(m):
        a = rng.normal(size=(1 << m, 1 << m)) + 1j * rng.normal(size=(1 << m, 1 << m))
        return np.linalg.qr(a)[0]

    c = qsynth.Circuit(n)
    for _ in range(6):
        qs = sorted(int(x) for x in rng.choice(n, size=k, replace=False))
        c.add("dense", qs, (), unitary(k))
        qs = sorted(int(x) for x in rng.choice(n, size=2, replace=False))
        c.add("dense", qs, (), unitary(2))
    plan = Q.qs_contract(n, Q.GateList(c), Q.opts(k_max=k, tile_qubits=t, dtype=dtype))
    try:
        f = costmodel.pass_features(plan)
        assert f[:, 11].sum() == 0, "a dense block wider than 3 qubits ran on the vector ALU"
        assert f[:, 8 if k == 4 else 9].sum() > 0, "no MFMA block of this width"
    finally:
        Q.qs_plan_destroy(plan)
    psi0 = qsynth.random_state(n, seed=13)
    ref = oracle.run(c, psi0.copy())
    got, nrm = run_plan(Q, c, dtype, psi0, k_max=k, tile_qubits=t)
    assert oracle.max_abs(ref, got) <= (TOL64 if dtype == 0 else TOL128)
    assert 1 - oracle.fidelity(ref, got) <= (1e-6 if dtype == 0 else 1e-12)


@pytest.mark.parametrize("dtype", [0, 1])
def test_fused_k6_valu_and_wide_dense(Q, oracle, dtype):
    n = 12
    kmax = 6 if dtype == 0 else 5
    c = qsynth.random_circuit(n, 120, seed=31, max_dense=kmax)
    psi0 = qsynth.random_state(n, seed=7)
    ref = oracle.run(c, psi0.copy())
    got, _ = run_plan(Q, c, dtype, psi0, k_max=kmax, tile_qubits=12)
    assert oracle.max_abs(ref, got) <= (TOL64 if dtype == 0 else TOL128)


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("k_max", [1, 2, 3, 4, 5, 6])
def test_fused_monomial_blocks(Q, oracle, dtype, k_max):
    """Circuits of permutation and phase gates only (CNOT, CZ, SWAP, X, Z, S,
    T, RZ, CP): every fused block is monomial and takes the gather-and-phase
    path, up to the widest block (k = 6 complex64, 5 complex128)."""
    if dtype == 1 and k_max > 5:
        pytest.skip("complex128 blocks stop at k = 5")
    n = 13
    c = qsynth.random_circuit(n, 300, seed=40 + k_max,
                              kinds=["cx", "cz", "swap", "x", "z", "s", "t", "rz", "cp"])
    psi0 = qsynth.random_state(n, seed=8)
    ref = oracle.run(c, psi0.copy())
    got, _ = run_plan(Q, c, dtype, psi0, k_max=k_max, tile_qubits=12)
    assert oracle.max_abs(ref, got) <= (TOL64 if dtype == 0 else TOL128)


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("k_max", [3, 4])
@pytest.mark.parametrize("t", [9, 12, 13])
def test_fused_block_diagonal_blocks(Q, oracle, dtype, k_max, t):
    """Permutation and phase gates with a few Hadamards: most fused blocks
    split into independent 2- or 4-wide classes (permuted block-diagonal)
    and take the vector-ALU class path; fewer groups than lanes (t = 9) and
    several groups per lane (t = 13) are both covered."""
    from paper_2509_04955_amd import costmodel

    n = 14
    c = qsynth.random_circuit(n, 400, seed=60 + k_max + t,
                              kinds=["cx", "cx", "cz", "rz", "t", "s", "x", "h"])
    gl = Q.GateList(c)
    plan = Q.qs_contract(n, gl, Q.opts(k_max=k_max, tile_qubits=t, dtype=dtype))
    try:
        f = costmodel.pass_features(plan)
        assert f[:, 16].sum() > 0, "no permuted block-diagonal blocks in this plan"
    finally:
        Q.qs_plan_destroy(plan)
    psi0 = qsynth.random_state(n, seed=9)
    ref = oracle.run(c, psi0.copy())
    got, _ = run_plan(Q, c, dtype, psi0, k_max=k_max, tile_qubits=t)
    assert oracle.max_abs(ref, got) <= (TOL64 if dtype == 0 else TOL128)


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("n", [4, 5, 7])
def test_fused_block_diagonal_small_states(Q, oracle, dtype, n):
    """Class-path blocks when the tile is the whole state and a workgroup has
    fewer groups than lanes (down to one group)."""
    c = qsynth.random_circuit(n, 120, seed=70 + n, kinds=["cx", "cz", "rz", "t", "x", "h"])
    psi0 = qsynth.random_state(n, seed=12)
    ref = oracle.run(c, psi0.copy())
    for k_max in (3, 4):
        got, _ = run_plan(Q, c, dtype, psi0, k_max=min(k_max, n), tile_qubits=n)
        assert oracle.max_abs(ref, got) <= (TOL64 if dtype == 0 else TOL128)


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("t", [9, 12, 13, 14])
def test_pauli_strategy(Q, oracle, dtype, t):
    """Contracted Pauli rotations on the device: UCC exponentials mixed with
    Z-only strings (diagonal rotations, no tile qubit needed), rotations whose
    Z part lies outside the tile (per-tile sign) and a random segment that
    stays greedy, over several tile sizes."""
    if dtype == 1 and t > 13:
        pytest.skip("complex128 tiles stop at 2^13")
    n = 16
    rng = np.random.default_rng(t)
    c, _ = qsynth.ucc(n, n_exp=40, seed=30 + t)
    for _ in range(6):
        sup = sorted(int(q) for q in rng.choice(n, size=5, replace=False))
        qsynth.pauli_exponential(c, [(q, "Z") for q in sup], float(rng.normal(0, 0.5)))
    for g in qsynth.random_circuit(n, 40, seed=t).gates:
        c.gates.append(g)
    for _ in range(6):
        sup = sorted(int(q) for q in rng.choice(n, size=6, replace=False))
        qsynth.pauli_exponential(c, [(q, "XYZ"[int(rng.integers(0, 3))]) for q in sup], float(rng.normal(0, 0.5)))
    psi0 = qsynth.random_state(n, seed=13)
    ref = oracle.run(c, psi0.copy())
    got, _ = run_plan(Q, c, dtype, psi0, k_max=4, tile_qubits=t, strategy=Q.STRATEGY_PAULI)
    assert oracle.max_abs(ref, got) <= (TOL64 if dtype == 0 else TOL128)


@pytest.mark.parametrize("renorm", [0, 1])
def test_renorm_chain(Q, oracle, renorm):
    n = 16
    c = qsynth.brickwork(n, depth=10, seed=2)
    ref = oracle.run(c)
    got, nrm = run_plan(Q, c, Q.QS_C64, None, k_max=5, renorm=renorm)
    assert 1 - oracle.fidelity(ref, got) <= 1e-6
    assert abs(nrm - 1) <= (1e-12 if renorm else 1e-5)


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_tiny_states_fused(Q, oracle, n):
    c = qsynth.random_circuit(n, 30, seed=n, max_dense=min(n, 3))
    psi0 = qsynth.random_state(n, seed=n)
    ref = oracle.run(c, psi0.copy())
    for dtype, tol in ((0, TOL64), (1, TOL128)):
        got, _ = run_plan(Q, c, dtype, psi0, k_max=min(n, 3))
        assert oracle.max_abs(ref, got) <= tol


def test_strategy_none_and_greedy_agree(Q, oracle):
    n = 15
    c = qsynth.plain_random(n, 12, 7, seed=4)
    ref = oracle.run(c)
    a, _ = run_plan(Q, c, Q.QS_C128, None, strategy=Q.STRATEGY_NONE)
    b, _ = run_plan(Q, c, Q.QS_C128, None, strategy=Q.STRATEGY_GREEDY, k_max=4)
    assert oracle.max_abs(ref, a) <= TOL128
    assert oracle.max_abs(ref, b) <= TOL128


def test_ucc_against_closed_form(Q, oracle):
    """UCC-style ansatz (Pauli exponentials compiled to CNOT ladders) at 20
    qubits, complex64 fused, against the closed-form rotation oracle."""
    n = 20
    c, rots = qsynth.ucc(n, n_exp=60, seed=3)
    ref = oracle.zero_state(n)
    for x, z, th in rots:
        oracle.pauli_rotation(ref, n, x, z, th)
    got, nrm = run_plan(Q, c, Q.QS_C64, None, k_max=5)
    assert 1 - oracle.fidelity(ref, got) <= 1e-6
    assert oracle.max_abs(ref, got) <= TOL64
    got128, _ = run_plan(Q, c, Q.QS_C128, None, k_max=5)
    assert oracle.max_abs(ref, got128) <= TOL128


@pytest.mark.parametrize("dtype,tol", [(0, 1e-6), (1, 1e-12)])
def test_expectation(Q, oracle, dtype, tol):
    n = 14
    c = qsynth.hea(n, layers=3, seed=(1, 1))
    ham = qsynth.random_pauli_sum(n, 50, seed=(2, 2))
    ref_psi = oracle.run(c)
    ref_terms = np.array([oracle.expect_pauli(ref_psi, n, int(x), int(z)).real for x, z in zip(ham.x, ham.z)])
    ref_E = float(np.dot(ham.coeff, ref_terms))
    gl = Q.GateList(c)
    plan = Q.qs_contract(n, gl, Q.opts(dtype=dtype))
    s = Q.State(n, dtype)
    s.apply_plan(plan)
    E, terms = s.expect(ham, with_terms=True)
    s.close()
    Q.qs_plan_destroy(plan)
    assert np.max(np.abs(terms - ref_terms)) <= tol
    assert abs(E - ref_E) <= tol * 10


def test_expectation_special_cases(Q, oracle):
    n = 9
    s = Q.State(n, Q.QS_C128)
    s.set_basis(0)
    x = np.array([0, 1, 0b101, 0], dtype=np.uint64)
    z = np.array([0, 0, 0b101, 0b110], dtype=np.uint64)
    E, terms = Q.qs_expect_pauli_sum(s.handle, x, z, np.ones(4), with_terms=True)
    assert np.allclose(terms, [1, 0, 0, 1], atol=1e-15)
    s.close()


def test_errors_leave_state_unchanged(Q):
    n = 6
    s = Q.State(n, Q.QS_C128)
    s.set_basis(5)
    bad = qsynth.Circuit(n).add("h", (0,)).add("cx", (2, 2))
    with pytest.raises(Q.QsimError) as ei:
        s.apply_gates(Q.GateList(bad))
    assert ei.value.status == Q.QS_EINVAL
    amps = s.amplitudes()
    assert amps[5] == 1 and np.count_nonzero(amps) == 1
    other = Q.qs_contract(7, Q.GateList(qsynth.ghz(7)))
    with pytest.raises(Q.QsimError):
        Q.qs_apply_plan(s.handle, other)
    Q.qs_plan_destroy(other)
    with pytest.raises(Q.QsimError):
        Q.qs_state_set_basis(s.handle, 1 << n)
    s.close()
    with pytest.raises(Q.QsimError):
        Q.qs_state_create(0, 0, None, None)


def test_copy_kernel(Q):
    import torch

    a = torch.arange(1 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    Q.qs_copy(b.data_ptr(), a.data_ptr(), a.numel() * 4, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def _class_log_width(U, tol=1e-14):
    """log2 of the widest connected component of U's nonzero pattern (rows
    against columns): the class width of a permuted block-diagonal block."""
    D = U.shape[0]
    parent = list(range(2 * D))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for r in range(D):
        for c in range(D):
            if abs(U[r, c]) > tol:
                parent[find(r)] = find(D + c)
    sizes = {}
    for r in range(D):
        sizes[find(r)] = sizes.get(find(r), 0) + 1
    w = max(sizes.values())
    return int(np.ceil(np.log2(w))) if w > 1 else 0


@pytest.mark.parametrize("t", [11, 12, 13])
@pytest.mark.parametrize("family", ["ucc", "perm"])
def test_class_blocks_on_matrix_cores(Q, oracle, t, family):
    """Staged complex64 passes put 4-qubit blocks with classes of 8
    amplitudes on the matrix cores (16x16 real products of eight class
    members at a time), and those with classes of 2 and 4 too (16-block 4x4
    products with the class matrix broadcast from one lane quad); the plan
    must contain each class width in staged passes and the state must match
    the oracle."""
    from paper_2509_04955_amd import costmodel

    n = 16
    if family == "ucc":
        c, _ = qsynth.ucc(n, n_exp=40, seed=80 + t)
    else:
        c = qsynth.random_circuit(n, 400, seed=90 + t, kinds=["cx", "cx", "cz", "rz", "t", "s", "x", "h"])
    gl = Q.GateList(c)
    plan = Q.qs_contract(n, gl, Q.opts(k_max=4, tile_qubits=t, low_qubits=4))
    try:
        f = costmodel.pass_features(plan)
        info = Q.qs_plan_info_get(plan)
        hits = {1: 0, 2: 0, 3: 0}
        for p in range(info.n_passes):
            if f[p, 14] < 0.5:
                continue
            _, _, b0, nb = Q.qs_plan_pass(plan, p)
            for b in range(b0, b0 + nb):
                qs, U, _ = Q.qs_plan_block(plan, b)
                k = len(qs)
                s = _class_log_width(U)
                if k == 4 and s in hits:
                    hits[s] += 1
        if family == "ucc":   # CNOT ladders with basis changes: classes of 2, 4 and 8 in every tile size
            for s, h in hits.items():
                assert h > 0, f"no 4-qubit blocks with classes of {2 ** s} in staged passes"
    finally:
        Q.qs_plan_destroy(plan)
    psi0 = qsynth.random_state(n, seed=13)
    ref = oracle.run(c, psi0.copy())
    got, _ = run_plan(Q, c, 0, psi0, k_max=4, tile_qubits=t, low_qubits=4)
    assert oracle.max_abs(ref, got) <= TOL64
    assert 1 - oracle.fidelity(ref, got) <= 1e-6


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("k_max,t", [(5, 12), (5, 13), (6, 12), (6, 13)])
def test_wide_monomial_blocks_in_staged_passes(Q, oracle, dtype, k_max, t):
    """5- and 6-qubit monomial blocks (CNOT, CZ, SWAP, X and phase gates)
    in passes whose operands are staged in LDS read their per-lane records
    there; the plan must contain such blocks in staged passes and the state
    must match the oracle."""
    from paper_2509_04955_amd import costmodel

    if dtype == 1 and t > 12:
        pytest.skip("complex128 tiles stop at t = 12")
    if dtype == 1 and k_max > 5:
        pytest.skip("complex128 blocks stop at k = 5")
    n = 16
    c = qsynth.random_circuit(n, 500, seed=5, kinds=["cx", "cz", "rz", "t", "s", "x", "swap"])
    plan = Q.qs_contract(n, Q.GateList(c), Q.opts(k_max=k_max, tile_qubits=t, low_qubits=4, dtype=dtype))
    try:
        f = costmodel.pass_features(plan)
        info = Q.qs_plan_info_get(plan)
        hits = 0
        for p in range(info.n_passes):
            if f[p, 14] < 0.5:
                continue
            _, _, b0, nb = Q.qs_plan_pass(plan, p)
            for b in range(b0, b0 + nb):
                qs, U, _ = Q.qs_plan_block(plan, b)
                nz = np.abs(np.asarray(U)) > 1e-14
                if len(qs) >= 5 and (nz.sum(0) == 1).all():
                    hits += 1
        if dtype == 0:
            assert hits > 0, "no 5- or 6-qubit monomial blocks in staged passes"
    finally:
        Q.qs_plan_destroy(plan)
    psi0 = qsynth.random_state(n, seed=19)
    ref = oracle.run(c, psi0.copy())
    got, _ = run_plan(Q, c, dtype, psi0, k_max=k_max, tile_qubits=t, low_qubits=4)
    assert oracle.max_abs(ref, got) <= (TOL64 if dtype == 0 else TOL128)


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("t", [11, 12, 13])
def test_permutation_blocks(Q, oracle, dtype, t):
    """4-qubit blocks whose every nonzero entry is 1 (products of CNOT, X and
    SWAP) are applied as pure permutations (reads and permuted writes, no
    arithmetic); the plan must contain such blocks and the state must match
    the oracle exactly up to the state's own rounding."""
    if dtype == 1 and t > 12:
        pytest.skip("complex128 tiles stop at t = 12")
    n = 16
    c = qsynth.random_circuit(n, 500, seed=70 + t, kinds=["cx", "cx", "x", "swap"])
    plan = Q.qs_contract(n, Q.GateList(c), Q.opts(k_max=4, tile_qubits=t, low_qubits=4))
    try:
        info = Q.qs_plan_info_get(plan)
        perms = 0
        for b in range(info.n_blocks):
            qs, U, _ = Q.qs_plan_block(plan, b)
            U = np.asarray(U)
            nz = np.abs(U) > 1e-14
            if len(qs) == 4 and (nz.sum(0) == 1).all() and np.allclose(U[nz], 1.0):
                perms += 1
        assert perms > 0, "no 4-qubit permutation blocks in the plan"
    finally:
        Q.qs_plan_destroy(plan)
    psi0 = qsynth.random_state(n, seed=17)
    ref = oracle.run(c, psi0.copy())
    got, _ = run_plan(Q, c, dtype, psi0, k_max=4, tile_qubits=t, low_qubits=4)
    # a permutation moves amplitudes without arithmetic: the only error is the
    # complex64 rounding of the input state
    tol = 1e-7 if dtype == 0 else 1e-15
    assert oracle.max_abs(ref, got) <= tol


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("family", ["qft", "qaoa", "phase"])
@pytest.mark.parametrize("k_max,t", [(3, 12), (4, 13), (5, 12)])
def test_commute_plans_match_oracle(Q, oracle, dtype, family, k_max, t):
    """Plans contracted with the commute option (gates, and in the packer
    whole blocks, passing others they commute with) give the oracle's state:
    QFT (commuting controlled phases), QAOA and a phase-heavy random circuit
    at 18 qubits, both precisions."""
    if dtype == 1 and t > 12:
        pytest.skip("complex128 tiles stop at t = 12")
    n = 18
    c = {"qft": lambda: qsynth.qft(n), "qaoa": lambda: qsynth.qaoa_maxcut(n),
         "phase": lambda: qsynth.random_circuit(n, 400, seed=k_max,
                                                kinds=["cx", "cz", "rz", "t", "h", "cp", "rx", "s", "u3"])}[family]()
    psi0 = qsynth.random_state(n, seed=5)
    ref = oracle.run(c, psi0.copy())
    got, _ = run_plan(Q, c, dtype, psi0, k_max=k_max, tile_qubits=t, low_qubits=4, commute=1)
    assert oracle.max_abs(ref, got) <= (TOL64 if dtype == 0 else TOL128)
    assert 1 - oracle.fidelity(ref, got) <= (1e-6 if dtype == 0 else 1e-12)


def _every_qubit_layers(n):
    """Two layers of U3 on every qubit around a CNOT chain: layers with no
    free qubit for the segments."""
    c = qsynth.Circuit(n)
    for q in range(n):
        c.add("u3", (q,), (0.3 + q, 0.2, 0.1 * q))
    for q in range(n - 1):
        c.add("cx", (q, q + 1))
    for q in range(n):
        c.add("h", (q,))
    return c


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("family,n", [("random", 1), ("random", 2), ("random", 3), ("random", 5), ("random", 9),
                                      ("random", 14), ("hea", 12), ("qaoa", 12), ("brickwork", 16), ("allq", 11),
                                      ("random", 19)])
def test_smgp_matches_oracle(Q, oracle, dtype, family, n):
    """Staggered multi-gate launches (DAG layers of one- and controlled
    one-qubit gates over cyclically assigned state segments) give the
    oracle's state: random circuits with SWAP and dense two-qubit gates
    mixed in (those run one sweep each), HEA and QAOA layers, brickwork, and
    a layer touching every qubit (split into chunks that leave enough qubits
    for the segments), both precisions."""
    c = {"random": lambda: qsynth.random_circuit(n, 12 * n, seed=n, max_dense=2),
         "hea": lambda: qsynth.hea_rxyz(n),
         "qaoa": lambda: qsynth.qaoa_maxcut(n),
         "brickwork": lambda: qsynth.brickwork(n, 6, seed=n),
         "allq": lambda: _every_qubit_layers(n)}[family]()
    psi0 = qsynth.random_state(n, seed=4)
    ref = oracle.run(c, psi0.copy())
    s = Q.State(n, dtype)
    s.load(psi0)
    s.apply_gates_smgp(Q.GateList(c))
    got = s.amplitudes()
    s.close()
    assert oracle.max_abs(ref, got) <= (TOL64 if dtype == 0 else TOL128)
