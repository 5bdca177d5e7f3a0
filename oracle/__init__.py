"""FP64 CPU oracle for the state-vector hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU
library never calls it, and it imports nothing from the GPU library: the two
share only the seeded input generators in ``qsynth``.

What it computes is the plain definition of circuit simulation (paper,
Section 2.1, Eq. 1-4): the output state is U_G ... U_1 psi_in, each gate
applied to the whole amplitude array in program order (Eq. 3 and Eq. 4),
in complex128.  Gate contraction, tiling and passes of the fast path reach
the same result (up to rounding) faster, so this plain form is what the fast
path is compared with.

Parts:
  * ``sv_oracle.c`` (compiled with gcc): gate loops, dense k-qubit gates,
    norm, Pauli expectation, closed-form Pauli rotation, the pair index set
    of Eq. 3/4, the operation-count model.
  * ``brute.py``: 2^n x 2^n Kronecker matrices (n <= 10), gates defined from
    their generators with a matrix exponential.
  * ``greedy.py``: the fixed-width greedy contraction rule and the plan
    checker (block products applied with the dense routine).
  * ``mlp.py``: FP64 forward/backward of the cost-model MLP.

Parity status of every function is stated in its docstring.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Oracle-private kind codes (the order of the enum in sv_oracle.c).
KINDS = {
    "h": 0, "x": 1, "y": 2, "z": 3, "s": 4, "sdg": 5, "t": 6, "tdg": 7,
    "rx": 8, "ry": 9, "rz": 10, "u3": 11, "p": 12,
    "cx": 13, "cz": 14, "cp": 15, "cu": 16, "swap": 17, "dense": 18,
}


def build(force: bool = False) -> str:
    """Compile sv_oracle.c with gcc (OpenMP on) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-D_GNU_SOURCE",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        c_dp = ctypes.c_void_p
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_get_threads.restype = ctypes.c_int
        L.or_gate_2x2.argtypes = [ctypes.c_int, c_dp, c_dp]
        L.or_gate_2x2.restype = ctypes.c_int
        L.or_apply_1q.argtypes = [c_dp, ctypes.c_int, ctypes.c_int, c_dp]
        L.or_apply_controlled.argtypes = [c_dp, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, c_dp]
        L.or_apply_dense.argtypes = [c_dp, ctypes.c_int, c_dp, ctypes.c_int, c_dp]
        L.or_apply_dense.restype = ctypes.c_int
        L.or_apply_swap.argtypes = [c_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_apply_gate.argtypes = [c_dp, ctypes.c_int, ctypes.c_int, c_dp, ctypes.c_int, c_dp, c_dp]
        L.or_apply_gate.restype = ctypes.c_int
        L.or_norm2.argtypes = [c_dp, ctypes.c_int]
        L.or_norm2.restype = ctypes.c_double
        L.or_expect_pauli.argtypes = [c_dp, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.or_expect_pauli_sum.argtypes = [c_dp, ctypes.c_int, c_dp, c_dp, c_dp, ctypes.c_int]
        L.or_expect_pauli_sum.restype = ctypes.c_double
        L.or_pauli_rotation.argtypes = [c_dp, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double]
        L.or_pair_lows.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, c_dp, ctypes.c_int64]
        L.or_pair_lows.restype = ctypes.c_int64
        L.or_opcount.argtypes = [ctypes.c_int, ctypes.c_int]
        L.or_opcount.restype = ctypes.c_double
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


# ---------------------------------------------------------------- states
def zero_state(n: int) -> np.ndarray:
    """|0...0> (Eq. 1 with alpha_0 = 1)."""
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def basis_state(n: int, index: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[index] = 1.0
    return psi


# ----------------------------------------------------------------- gates
def gate_2x2(name: str, params=()) -> np.ndarray:
    """2x2 matrix of a one-qubit kind (or the target part of a controlled
    kind) from the oracle's own table.  Pinned by tests/test_oracle_pins.py
    against matrix exponentials of Pauli generators."""
    p = np.zeros(4, dtype=np.float64)
    p[: len(params)] = params
    m = np.zeros(4, dtype=np.complex128)
    if lib().or_gate_2x2(KINDS[name], _ptr(p), _ptr(m)) != 0:
        raise ValueError(f"no 2x2 matrix for kind {name!r}")
    return m.reshape(2, 2)


def apply_gate(psi: np.ndarray, n: int, name: str, qubits, params=(), matrix=None) -> None:
    """Apply one gate in place (the pair update of Eq. 3 for one-qubit kinds,
    Eq. 4 for controlled kinds with qubits = (control, target), the dense routine
    for 'dense' with local bit j <-> qubits[j])."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous and psi.size == 1 << n
    q = np.asarray(qubits, dtype=np.int32)
    p = np.zeros(4, dtype=np.float64)
    p[: len(params)] = params
    dense = None
    if matrix is not None:
        dense = np.ascontiguousarray(matrix, dtype=np.complex128)
    rc = lib().or_apply_gate(_ptr(psi), n, KINDS[name], _ptr(q), len(q), _ptr(p),
                             _ptr(dense) if dense is not None else None)
    if rc != 0:
        raise ValueError(f"oracle rejected gate {name} {tuple(qubits)}")


def apply_dense(psi: np.ndarray, n: int, qubits, matrix: np.ndarray) -> None:
    """Dense k-qubit gate, local bit j <-> qubits[j] (Eq. 6 generalised)."""
    q = np.asarray(qubits, dtype=np.int32)
    m = np.ascontiguousarray(matrix, dtype=np.complex128)
    assert m.shape == (1 << len(q), 1 << len(q))
    if lib().or_apply_dense(_ptr(psi), n, _ptr(q), len(q), _ptr(m)) != 0:
        raise ValueError("oracle rejected dense gate")


def run(circuit, psi: np.ndarray | None = None) -> np.ndarray:
    """Gate-by-gate FP64 simulation of a qsynth.Circuit (program order)."""
    n = circuit.n
    if psi is None:
        psi = zero_state(n)
    for g in circuit.gates:
        apply_gate(psi, n, g.name, g.qubits, g.params, g.matrix)
    return psi


def norm2(psi: np.ndarray, n: int) -> float:
    return float(lib().or_norm2(_ptr(psi), n))


def expect_pauli(psi: np.ndarray, n: int, x: int, z: int) -> complex:
    re, im = ctypes.c_double(), ctypes.c_double()
    lib().or_expect_pauli(_ptr(psi), n, int(x), int(z), ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def expect_pauli_sum(psi: np.ndarray, n: int, xs, zs, coeffs) -> float:
    x = np.ascontiguousarray(xs, dtype=np.uint64)
    z = np.ascontiguousarray(zs, dtype=np.uint64)
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    return float(lib().or_expect_pauli_sum(_ptr(psi), n, _ptr(x), _ptr(z), _ptr(c), len(c)))


def pauli_rotation(psi: np.ndarray, n: int, x: int, z: int, theta: float) -> None:
    """exp(-i theta P) psi in place, closed form (P^2 = I)."""
    lib().or_pauli_rotation(_ptr(psi), n, int(x), int(z), float(theta))


def pair_lows(n: int, t: int, controls=()) -> np.ndarray:
    """Lower members of the amplitude pairs a gate on target t couples
    (Eq. 3; with controls, Eq. 4): every i with bit t clear and all control
    bits set, in increasing order.  Pinned against brute-force set-builder
    enumeration and the grouped traversal of Section 2.2 in
    tests/test_oracle_pins.py."""
    cap = 1 << n
    out = np.zeros(cap, dtype=np.int64)
    cm = 0
    for c in controls:
        cm |= 1 << int(c)
    cnt = lib().or_pair_lows(n, t, cm, _ptr(out), cap)
    return out[: min(cnt, cap)].copy()


def opcount(n: int, k: int) -> float:
    """Operation count of a k-qubit matrix applied to an n-qubit state
    (Section 3.4: 10 * 2^(n-1) for k = 1, 36 * 2^(n-2) for k = 2)."""
    return float(lib().or_opcount(n, k))


def fidelity(ref: np.ndarray, got: np.ndarray) -> float:
    """|<ref|got>|^2 / (<ref|ref> <got|got>), accumulated in FP64: 1 for equal
    states up to a global phase and scale, 0 for orthogonal ones.  Pinned in
    tests/test_oracle_metrics.py (orthogonal states, |0> against |+>, phase
    and scale invariance, a hand-computed overlap)."""
    ref = np.asarray(ref, dtype=np.complex128)
    got = np.asarray(got, dtype=np.complex128)
    ov = np.vdot(ref, got)
    return float(abs(ov) ** 2 / (np.vdot(ref, ref).real * np.vdot(got, got).real))


def max_abs(ref: np.ndarray, got: np.ndarray) -> float:
    """max_i |got[i] - ref[i]| in FP64, no phase alignment or normalisation.
    Pinned in tests/test_oracle_metrics.py (hand-computed cases)."""
    return float(np.max(np.abs(np.asarray(ref, dtype=np.complex128) - np.asarray(got, dtype=np.complex128))))
