"""Pins of the oracle's comparison metrics (fidelity and max-abs error), the
two numbers every parity test and the accuracy report rest on.  Each case has
a value fixed by hand, so a dropped square, a missing normalisation or a
conjugation on the wrong side fails here."""
import math

import numpy as np
import pytest

import qsynth


def test_fidelity_of_orthogonal_states_is_zero(oracle):
    a = np.array([1, 0, 0, 0], dtype=complex)
    b = np.array([0, 0, 1j, 0], dtype=complex)
    assert oracle.fidelity(a, b) == 0.0
    # |+> and |-> are orthogonal although they share support
    plus = np.array([1, 1], dtype=complex) / math.sqrt(2)
    minus = np.array([1, -1], dtype=complex) / math.sqrt(2)
    assert oracle.fidelity(plus, minus) < 1e-30


def test_fidelity_zero_against_plus_is_one_half(oracle):
    zero = np.array([1, 0], dtype=complex)
    plus = np.array([1, 1], dtype=complex) / math.sqrt(2)
    assert abs(oracle.fidelity(zero, plus) - 0.5) < 1e-15
    # |<0|+i>|^2 with |+i> = (|0> + i|1>)/sqrt2 is also 1/2; a missing
    # conjugate would make <+i|+i> = 0 and break the normalisation
    plus_i = np.array([1, 1j], dtype=complex) / math.sqrt(2)
    assert abs(oracle.fidelity(zero, plus_i) - 0.5) < 1e-15
    assert abs(oracle.fidelity(plus_i, plus_i) - 1.0) < 1e-15


def test_fidelity_hand_computed_overlap(oracle):
    # a = (1, 2i)/sqrt5, b = (3, 4)/5: <a|b> = (3 - 8i)/(5 sqrt5), |.|^2 = 73/125
    a = np.array([1, 2j], dtype=complex) / math.sqrt(5)
    b = np.array([3, 4], dtype=complex) / 5
    assert abs(oracle.fidelity(a, b) - 73 / 125) < 1e-15
    assert abs(oracle.fidelity(b, a) - 73 / 125) < 1e-15   # symmetric


@pytest.mark.parametrize("n", [3, 8])
def test_fidelity_phase_and_scale_invariance(oracle, n):
    psi = qsynth.random_state(n, seed=n)
    phi = qsynth.random_state(n, seed=n + 100)
    f = oracle.fidelity(psi, phi)
    assert 0.0 <= f <= 1.0
    assert abs(oracle.fidelity(psi, psi * np.exp(0.73j)) - 1.0) < 1e-14
    assert abs(oracle.fidelity(psi, 3.5 * psi) - 1.0) < 1e-14       # unnormalised input
    assert abs(oracle.fidelity(2.0 * psi, np.exp(-1.1j) * phi) - f) < 1e-14


def test_fidelity_detects_a_small_rotation(oracle):
    # cos^2(eps) for a state rotated by eps out of itself
    eps = 1e-3
    a = np.array([1, 0, 0, 0], dtype=complex)
    b = np.array([math.cos(eps), 0, 0, math.sin(eps)], dtype=complex)
    assert abs((1 - oracle.fidelity(a, b)) - math.sin(eps) ** 2) < 1e-15


def test_max_abs_hand_computed(oracle):
    a = np.array([1, 0, 0.5j, -1], dtype=complex)
    b = np.array([1, 0.1, 0.5j + 0.3 + 0.4j, -1], dtype=complex)
    assert abs(oracle.max_abs(a, b) - 0.5) < 1e-15     # |0.3 + 0.4i| = 0.5
    assert oracle.max_abs(a, a) == 0.0
    # no phase alignment: a global phase of pi gives twice the largest modulus
    assert abs(oracle.max_abs(a, -a) - 2.0) < 1e-15
    # symmetric, and complex modulus rather than a per-part maximum
    assert abs(oracle.max_abs(b, a) - 0.5) < 1e-15
    c = np.array([0.6 + 0.8j], dtype=complex)
    assert abs(oracle.max_abs(np.zeros(1, dtype=complex), c) - 1.0) < 1e-15
