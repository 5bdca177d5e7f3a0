"""Pauli-sum expectation on the GPU (one read of the state per group of terms)
against the oracle's plain sum over amplitudes, <psi|P|psi> =
sum_j conj(psi[j^x]) i^{|x&z|} (-1)^{|j&z|} psi[j] (Section 1: VQE energies).

The oracle evaluates the same stored amplitudes (complex64 states are rounded
to complex64 first).  Complex128: products and sums in FP64 on both sides, so
only the summation order differs: 1e-12.  Complex64: a pair's Re or Im of
conj(psi[j^x]) psi[j] is formed in FP32 (one product and one fused
multiply-add, relative error below 2^-23) and summed in FP64, so a term of a
unit state is off by at most 2^-23 sum_pairs |psi_j psi_{j^x}| <= 2^-24; the
bound used is 2^-22.

Cases: state sizes from one qubit (a coset smaller than a workgroup) through
several cosets per group (15..20 qubits); Hamiltonians whose terms are all
diagonal, all within the low tile bits, all above them, or repeated, which
group differently; more terms than one launch takes; a state with a pending
renormalisation; and the benchmark's 30-qubit state, where the energy of the
first exponentials is known in closed form from the <= 2^10 nonzero
amplitudes."""
import math

import numpy as np
import pytest

import qsynth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    import torch

    from paper_2509_04955_amd import qsim

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    qsim.lib()
    return qsim


def _stored(psi, dtype):
    return psi.astype(np.complex64).astype(np.complex128) if dtype == 0 else psi


def _ref_terms(oracle, psi, n, xs, zs):
    return np.array([oracle.expect_pauli(psi, n, int(x), int(z)).real for x, z in zip(xs, zs)])


TOL = {0: 2.0 ** -22, 1: 1e-12}


def _check(Q, oracle, n, dtype, xs, zs, seed=0):
    tol = TOL[dtype]
    psi = qsynth.random_state(n, seed=seed)
    s = Q.State(n, dtype)
    s.load(psi)
    coeff = np.random.default_rng(seed).normal(size=len(xs))
    E, terms = Q.qs_expect_pauli_sum(s.handle, np.asarray(xs, dtype=np.uint64), np.asarray(zs, dtype=np.uint64),
                                     coeff, with_terms=True)
    s.close()
    ref = _ref_terms(oracle, _stored(psi, dtype), n, xs, zs)
    ref = ref / oracle.norm2(_stored(psi, dtype), n)
    assert np.max(np.abs(terms - ref)) <= tol, np.max(np.abs(terms - ref))
    assert abs(E - float(np.dot(coeff, ref))) <= tol * max(1.0, float(np.sum(np.abs(coeff))))


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("n", [1, 2, 5, 8, 9, 10, 13, 14, 15, 17, 20])
def test_random_pauli_sums(Q, oracle, n, dtype):
    ham = qsynth.random_pauli_sum(n, 40, seed=(n, 3))
    _check(Q, oracle, n, dtype, ham.x, ham.z, seed=n)


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("kind", ["diagonal", "low_x", "high_x", "repeated", "single_x_bits"])
def test_term_structures(Q, oracle, kind, dtype):
    n = 18
    rng = np.random.default_rng(7)
    full = (1 << n) - 1
    m = 37
    if kind == "diagonal":        # every term in one span (rank 0): groups by the term limit only
        xs = np.zeros(m, dtype=np.uint64)
        zs = rng.integers(0, full, size=m, dtype=np.uint64)
    elif kind == "low_x":         # X parts inside the contiguous tile bits
        xs = rng.integers(1, 64, size=m, dtype=np.uint64)
        zs = rng.integers(0, full, size=m, dtype=np.uint64)
    elif kind == "high_x":        # X parts only above the tile bits
        xs = rng.integers(1, 1 << (n - 6), size=m, dtype=np.uint64) << np.uint64(6)
        zs = rng.integers(0, full, size=m, dtype=np.uint64)
    elif kind == "repeated":      # the same strings many times (dependent spans)
        base = qsynth.random_pauli_sum(n, 5, seed=(9, 9))
        xs = np.tile(base.x, 8)
        zs = np.tile(base.z, 8)
    else:                         # X on one qubit each, every position
        xs = np.array([1 << q for q in range(n)], dtype=np.uint64)
        zs = rng.integers(0, full, size=n, dtype=np.uint64)
    _check(Q, oracle, n, dtype, xs, zs, seed=11)


def test_more_terms_than_one_launch(Q, oracle):
    n = 11
    ham = qsynth.random_pauli_sum(n, 5000, seed=(4, 4))
    _check(Q, oracle, n, 1, ham.x, ham.z, seed=4)


@pytest.mark.parametrize("dtype,tol", [(0, 1e-6), (1, 1e-12)])
def test_pending_renormalisation(Q, oracle, dtype, tol):
    """After a plan with renormalisation the stored amplitudes carry a pending
    scale; the terms are normalised by the squared norm the same launch
    computes."""
    n = 16
    c = qsynth.hea(n, layers=3, seed=(1, 2))
    ham = qsynth.random_pauli_sum(n, 60, seed=(2, 3))
    ref_psi = oracle.run(c)
    ref = _ref_terms(oracle, ref_psi, n, ham.x, ham.z)
    plan = Q.qs_contract(n, Q.GateList(c), Q.opts(dtype=dtype))
    s = Q.State(n, dtype)
    s.apply_plan(plan)
    E, terms = s.expect(ham, with_terms=True)
    s.close()
    Q.qs_plan_destroy(plan)
    assert np.max(np.abs(terms - ref)) <= tol
    assert abs(E - float(np.dot(ham.coeff, ref))) <= tol * 20


def _sparse_energy(state, xs, zs):
    """<psi|P|psi> from the nonzero amplitudes {index: amplitude}."""
    out = []
    for x, z in zip(xs, zs):
        x, z = int(x), int(z)
        ph = (1j) ** (bin(x & z).count("1") % 4)
        v = 0j
        for j, a in state.items():
            b = state.get(j ^ x)
            if b is not None:
                v += np.conj(b) * ph * (-1 if bin(j & z).count("1") % 2 else 1) * a
        out.append(v.real)
    return np.array(out)


def test_energy_30q_closed_form(Q):
    """The benchmark's 30-qubit state after the first 10 exponentials (bench
    plan configuration) and a 200-term random Pauli sum: every term against
    the closed form."""
    from test_gpu_fullsize import sparse_rotations

    n = 30
    c, rots = qsynth.ucc(n, n_exp=10, seed=3)
    # terms that touch the state's support: strings built from the rotations'
    # own X parts (nonzero expectations) mixed with random ones (mostly zero)
    ham = qsynth.random_pauli_sum(n, 150, seed=(7, 0))
    xs = list(ham.x) + [int(x) for x, _, _ in rots] * 5
    zs = list(ham.z) + [int(z) ^ (1 << (3 * i % n)) for i, (_, z, _) in enumerate(rots * 5)]
    plan = Q.qs_contract(n, Q.GateList(c), Q.opts(k_max=4, tile_qubits=13, low_qubits=4))
    s = Q.State(n, Q.QS_C64)
    s.apply_plan(plan)
    E, terms = Q.qs_expect_pauli_sum(s.handle, np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64),
                                     np.ones(len(xs)), with_terms=True)
    s.close()
    Q.qs_plan_destroy(plan)
    ref = _sparse_energy(sparse_rotations(rots), xs, zs)
    assert np.max(np.abs(terms - ref)) <= 1e-6
    assert np.count_nonzero(np.abs(ref) > 1e-3) >= 10   # the check is not all zeros
    assert math.isfinite(E)
