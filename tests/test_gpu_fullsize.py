"""Parity at the benchmark's full size: 30-qubit states in the launch
configuration the bench times for the UCC workload (k_max 4, 2^13-amplitude
tiles with 4 fixed low qubits, 512-thread workgroups), checked on
outputs an oracle computes one amplitude at a time and on properties that
hold at any size.

* Pauli-rotation products: m rotations exp(-i theta P) applied to |0...0>
  leave at most 2^m nonzero amplitudes, each a closed form of Pauli algebra
  (P|k> = i^{|x&z|} (-1)^{|k&z|} |k xor x>); the helper that enumerates them
  is pinned against the oracle's dense closed form on CPU below.
* GHZ: amplitudes 1/sqrt 2 at |0...0> and |1...1>.
* QFT of a basis state: QFT|x> = 2^{-n/2} sum_y exp(2 pi i x y / 2^n) |y>,
  sampled amplitudes.
* A UCC prefix followed by its inverse returns |0...0>."""
import math

import numpy as np
import pytest

import qsynth

N = 30
BENCH = dict(k_max=4, tile_qubits=13, low_qubits=4)


def sparse_rotations(rots):
    """Exact state prod_r exp(-i theta_r P_r) |0...0> as {index: amplitude}:
    exp(-i t P) = cos t I - i sin t P."""
    state = {0: 1.0 + 0.0j}
    for x, z, th in rots:
        x, z = int(x), int(z)
        ph = (1j) ** (bin(x & z).count("1") % 4)
        c, s = math.cos(th), math.sin(th)
        out = {}
        for k, a in state.items():
            out[k] = out.get(k, 0j) + c * a
            sign = -1.0 if bin(k & z).count("1") % 2 else 1.0
            kk = k ^ x
            out[kk] = out.get(kk, 0j) + (-1j * s) * ph * sign * a
        state = out
    return state


def test_sparse_rotation_helper_matches_oracle(oracle):
    """CPU pin of the helper: the oracle's dense closed form at 12 qubits."""
    n = 12
    _, rots = qsynth.ucc(n, n_exp=9, seed=5)
    ref = oracle.zero_state(n)
    for x, z, th in rots:
        oracle.pauli_rotation(ref, n, x, z, th)
    sp = sparse_rotations(rots)
    dense = np.zeros(1 << n, dtype=np.complex128)
    for k, a in sp.items():
        dense[k] = a
    assert oracle.max_abs(ref, dense) <= 1e-13


@pytest.fixture(scope="module")
def Q():
    import torch

    from paper_2509_04955_amd import qsim

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    qsim.lib()
    return qsim


def run(Q, c, dtype, basis=0, **kw):
    plan = Q.qs_contract(c.n, Q.GateList(c), Q.opts(dtype=dtype, **kw))
    s = Q.State(c.n, dtype)
    s.set_basis(basis)
    s.apply_plan(plan)
    Q.qs_plan_destroy(plan)
    return s


def amps_at(Q, s, idx):
    return np.array([Q.qs_state_copy_out(s.handle, int(k), 1)[0] for k in idx])


@pytest.mark.gpu
@pytest.mark.parametrize("dtype,tol", [(0, 1e-5), (1, 1e-12)])
def test_ucc_prefix_30q_every_nonzero_amplitude(Q, dtype, tol):
    """The first 10 exponentials of the benchmark circuit (seed 3): every one of
    the <= 2^10 nonzero amplitudes against the closed form, and all of the
    norm on them."""
    c, rots = qsynth.ucc(N, n_exp=10, seed=3)
    kw = BENCH if dtype == 0 else dict(k_max=3, tile_qubits=11, low_qubits=4)
    s = run(Q, c, dtype, **kw)
    exact = sparse_rotations(rots)
    idx = sorted(exact)
    ref = np.array([exact[k] for k in idx])
    got = amps_at(Q, s, idx)
    assert np.max(np.abs(got - ref)) <= tol
    assert abs(np.sum(np.abs(got) ** 2) - 1.0) <= 10 * tol   # nothing anywhere else
    assert abs(s.norm() - 1.0) <= 10 * tol
    s.close()


@pytest.mark.gpu
def test_ghz_30q(Q):
    s = run(Q, qsynth.ghz(N), 0, **BENCH)
    got = amps_at(Q, s, [0, (1 << N) - 1])
    assert np.max(np.abs(got - 1 / math.sqrt(2))) <= 1e-6
    assert abs(s.norm() - 1.0) <= 1e-6
    s.close()


@pytest.mark.gpu
def test_qft_of_basis_state_30q(Q):
    x = 0x2345ABC
    s = run(Q, qsynth.qft(N), 0, basis=x, **BENCH)
    rng = np.random.default_rng(0)
    idx = np.concatenate([[0, 1, (1 << N) - 1], rng.integers(0, 1 << N, size=509)])
    got = amps_at(Q, s, idx)
    ang = 2 * np.pi * ((x * idx.astype(object)) % (1 << N)).astype(np.float64) / (1 << N)
    ref = np.exp(1j * ang) / math.sqrt(1 << N)
    assert np.max(np.abs(got - ref)) <= 1e-5 / math.sqrt(1 << N) * 30
    s.close()


@pytest.mark.gpu
def test_ucc_prefix_and_inverse_return_to_zero_30q(Q):
    c, _ = qsynth.ucc(N, n_exp=40, seed=3)
    both = qsynth.Circuit(N, list(c.gates) + list(qsynth.inverse(c).gates))
    s = run(Q, both, 0, **BENCH)
    a0 = amps_at(Q, s, [0])[0]
    assert 1 - abs(a0) ** 2 <= 1e-5
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("t", [12, 13, 14])
def test_large_tiles_30q(Q, t):
    """2^12-amplitude tiles (block operands staged in LDS), 2^13- and
    2^14-amplitude tiles (512- and 1024-thread workgroups, several tiles per
    workgroup at 30 qubits): the UCC prefix's nonzero amplitudes
    against the closed form, and sampled QFT amplitudes with dense 4- and
    5-qubit blocks."""
    c, rots = qsynth.ucc(N, n_exp=10, seed=3)
    s = run(Q, c, 0, k_max=4, tile_qubits=t, low_qubits=4)
    exact = sparse_rotations(rots)
    idx = sorted(exact)
    got = amps_at(Q, s, idx)
    assert np.max(np.abs(got - np.array([exact[k] for k in idx]))) <= 1e-5
    assert abs(s.norm() - 1.0) <= 1e-4
    s.close()
    x = 0x1F00D5
    s = run(Q, qsynth.qft(N), 0, basis=x, k_max=5, tile_qubits=t, low_qubits=4)
    rng = np.random.default_rng(1)
    idx = np.concatenate([[0, 1, (1 << N) - 1], rng.integers(0, 1 << N, size=253)])
    got = amps_at(Q, s, idx)
    ang = 2 * np.pi * ((x * idx.astype(object)) % (1 << N)).astype(np.float64) / (1 << N)
    ref = np.exp(1j * ang) / math.sqrt(1 << N)
    assert np.max(np.abs(got - ref)) <= 1e-5 / math.sqrt(1 << N) * 30
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("t", [13, 14])
def test_pauli_strategy_30q_every_nonzero_amplitude(Q, t):
    """Pauli-rotation contraction at full size: the first 12 exponentials of
    the benchmark circuit (at most 2^12 nonzero amplitudes), every nonzero
    amplitude against the closed form."""
    c, rots = qsynth.ucc(N, n_exp=12, seed=3)
    s = run(Q, c, 0, k_max=4, tile_qubits=t, low_qubits=4, strategy=Q.STRATEGY_PAULI)
    exact = sparse_rotations(rots)
    idx = sorted(exact)
    got = amps_at(Q, s, idx)
    assert np.max(np.abs(got - np.array([exact[k] for k in idx]))) <= 1e-5
    assert abs(s.norm() - 1.0) <= 1e-4
    s.close()
