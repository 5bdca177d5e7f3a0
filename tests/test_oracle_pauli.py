"""Pins of the oracle's Pauli expectation and closed-form Pauli rotation."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import qsynth
from oracle import brute


def _random_masks(rng, n):
    letters = [(q, "IXYZ"[int(rng.integers(0, 4))]) for q in range(n)]
    return qsynth.pauli_masks([(q, a) for q, a in letters if a != "I"])


def test_expectation_on_zero_state(oracle):
    n = 10
    psi = oracle.zero_state(n)
    rng = np.random.default_rng(1)
    for _ in range(50):
        x, z = _random_masks(rng, n)
        v = oracle.expect_pauli(psi, n, x, z)
        assert abs(v - (1.0 if x == 0 else 0.0)) < 1e-15


def test_expectation_on_product_state(oracle):
    """For a product state every Pauli string factorises into single-qubit
    Bloch components <X>, <Y>, <Z>."""
    n = 8
    rng = np.random.default_rng(2)
    c = qsynth.Circuit(n)
    for q in range(n):
        c.add("u3", (q,), qsynth.haar_u3_angles(rng))
    psi = oracle.run(c)
    bloch = []
    for q in range(n):
        u = oracle.gate_2x2("u3", c.gates[q].params)
        v = u @ np.array([1, 0], dtype=complex)
        bloch.append({a: (v.conj() @ brute.PAULI[a] @ v).real for a in "IXYZ"})
    for _ in range(40):
        letters = [(q, "IXYZ"[int(rng.integers(0, 4))]) for q in range(n)]
        x, z = qsynth.pauli_masks([(q, a) for q, a in letters if a != "I"])
        expect = np.prod([bloch[q][a] for q, a in letters])
        got = oracle.expect_pauli(psi, n, x, z)
        assert abs(got - expect) < 1e-13


@pytest.mark.parametrize("n", [1, 3, 6, 8])
def test_expectation_vs_dense_pauli(oracle, n):
    rng = np.random.default_rng(3 + n)
    psi = qsynth.random_state(n, seed=n)
    for _ in range(20):
        x, z = _random_masks(rng, n)
        P = brute.pauli_from_masks(n, x, z)
        ref = np.vdot(psi, P @ psi)
        got = oracle.expect_pauli(psi, n, x, z)
        assert abs(got - ref) < 1e-13
        assert abs(got.imag) < 1e-13 and -1 - 1e-13 <= got.real <= 1 + 1e-13


def test_expectation_sum(oracle):
    n = 7
    psi = qsynth.random_state(n, seed=5)
    H = qsynth.random_pauli_sum(n, 30, seed=(5, 1))
    dense = sum(c * brute.pauli_from_masks(n, int(x), int(z)) for x, z, c in zip(H.x, H.z, H.coeff))
    ref = np.vdot(psi, dense @ psi).real
    assert abs(oracle.expect_pauli_sum(psi, n, H.x, H.z, H.coeff) - ref) < 1e-12


@pytest.mark.parametrize("n", [2, 4, 6])
def test_pauli_rotation_vs_expm(oracle, n):
    rng = np.random.default_rng(20 + n)
    for _ in range(10):
        x, z = _random_masks(rng, n)
        theta = float(rng.normal())
        psi = qsynth.random_state(n, seed=int(rng.integers(0, 1000)))
        ref = expm(-1j * theta * brute.pauli_from_masks(n, x, z)) @ psi
        oracle.pauli_rotation(psi, n, x, z, theta)
        assert np.max(np.abs(psi - ref)) < 1e-13


@pytest.mark.parametrize("n,seed", [(8, 1), (12, 2)])
def test_compiled_exponentials_match_closed_form(oracle, n, seed):
    """The UCC compiler (basis change, CNOT ladder, RZ(2 theta), reverse)
    equals the closed-form rotation exp(-i theta P)."""
    c, rots = qsynth.ucc(n, n_exp=25, wmin=1, wmax=min(8, n), theta_sd=0.7, seed=seed)
    psi0 = qsynth.random_state(n, seed=seed)
    got = oracle.run(c, psi0.copy())
    ref = psi0.copy()
    for x, z, th in rots:
        oracle.pauli_rotation(ref, n, x, z, th)
    assert np.max(np.abs(got - ref)) < 1e-12
