"""GPU parity of the batched persistent path (one hipGraph launch): every
state's energy and amplitudes against the FP64 oracle, for uneven qubit
counts, repeated launches (determinism) and the autotuned plan choice."""
import numpy as np
import pytest

import qsynth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    import torch

    from paper_2509_04955_amd import qsim

    assert torch.cuda.is_available()
    qsim.lib()
    return qsim


def _oracle_energy(oracle, c, h):
    psi = oracle.run(c)
    return psi, oracle.expect_pauli_sum(psi, c.n, h.x, h.z, h.coeff)


@pytest.mark.parametrize("dtype,tol", [(0, 1e-6), (1, 1e-12)])
def test_batch_small_uneven(Q, oracle, dtype, tol):
    """24 HEA states with 3..15 qubits (several passes for the larger ones
    at a 10-qubit tile), 8 layers RY/RZ + CZ ring, 30-term Pauli sums."""
    circuits, hams = qsynth.hea_batch(24, 3, 15, layers=8, n_terms=30, seed=7)
    b = Q.Batch(circuits, hams, Q.opts(k_max=3, tile_qubits=10, dtype=dtype))
    E1 = b.run()
    E2 = b.run()
    assert np.array_equal(E1, E2), "repeated launches must agree bitwise"
    for i, (c, h) in enumerate(zip(circuits, hams)):
        psi, e = _oracle_energy(oracle, c, h)
        assert abs(E1[i] - e) <= tol * max(1, abs(e)), (i, c.n, E1[i], e)
        amps = b.amplitudes(i)
        assert oracle.max_abs(psi, amps) <= (1e-5 if dtype == 0 else 1e-12)
    b.close()


def test_batch_mixed_block_kinds(Q, oracle):
    """k_max = 5 (MFMA blocks) and monomial blocks together in one batch."""
    circuits = [qsynth.random_circuit(n, 120, seed=n, max_dense=2) for n in (6, 9, 12, 14, 16)]
    hams = [qsynth.random_pauli_sum(c.n, 12, seed=(3, c.n)) for c in circuits]
    b = Q.Batch(circuits, hams, Q.opts(k_max=5, tile_qubits=11))
    E = b.run()
    for i, (c, h) in enumerate(zip(circuits, hams)):
        psi, e = _oracle_energy(oracle, c, h)
        assert abs(E[i] - e) <= 1e-5
        assert 1 - oracle.fidelity(psi, b.amplitudes(i)) <= 1e-6
    b.close()


@pytest.mark.parametrize("dtype,tol", [(0, 1e-5), (1, 1e-12)])
def test_batch_pauli_rotation_plans(Q, oracle, dtype, tol):
    """UCC states of 10..16 qubits under the Pauli-rotation contraction in the
    batch kernel: rotation blocks, grouped rotations and their per-tile signs
    (Z parts outside the tile) go through the same block dispatch."""
    circuits = [qsynth.ucc(n, n_exp=25, seed=40 + n)[0] for n in (10, 12, 13, 16)]
    hams = [qsynth.random_pauli_sum(c.n, 16, seed=(5, c.n)) for c in circuits]
    b = Q.Batch(circuits, hams, Q.opts(k_max=4, tile_qubits=10, dtype=dtype, strategy=Q.STRATEGY_PAULI))
    E = b.run()
    for i, (c, h) in enumerate(zip(circuits, hams)):
        psi, e = _oracle_energy(oracle, c, h)
        assert abs(E[i] - e) <= tol * max(1, abs(e)), (i, c.n, E[i], e)
        assert oracle.max_abs(psi, b.amplitudes(i)) <= tol
    b.close()


def test_batch_autotuned(Q, oracle):
    """k_max = 0 asks the autotuner for every distinct qubit count."""
    circuits, hams = qsynth.hea_batch(10, 12, 17, layers=8, n_terms=20, seed=9)
    b = Q.Batch(circuits, hams, Q.opts(k_max=0, tile_qubits=0))
    E = b.run()
    for i, (c, h) in enumerate(zip(circuits, hams)):
        _, e = _oracle_energy(oracle, c, h)
        assert abs(E[i] - e) <= 1e-5
    b.close()


def test_autotune_returns_valid_choice(Q):
    c = qsynth.brickwork(16, depth=6, seed=1)
    gl = Q.GateList(c)
    best = Q.qs_autotune(16, Q.QS_C64, gl)
    assert 2 <= best.k_max <= 5 and 11 <= best.tile_qubits <= 13
    again = Q.qs_autotune(16, Q.QS_C64, gl)
    assert (again.k_max, again.tile_qubits) == (best.k_max, best.tile_qubits)


def test_batch_rejects_bad_input(Q):
    c = qsynth.hea(5, 1, seed=(1, 1))
    h = qsynth.random_pauli_sum(6, 3, seed=(1, 2))  # acts on qubit 5 of a 5-qubit state
    with pytest.raises(Q.QsimError):
        Q.Batch([c], [h], Q.opts(k_max=2, tile_qubits=5))
