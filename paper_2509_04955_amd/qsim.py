"""Thin ctypes binding of libqsim (include/qsim.h).

Argument marshalling only: every function here forwards to the C entry point
of the same name and raises QsimError on a non-zero status.  PyTorch is used
by the convenience helpers for device memory and the current HIP stream.
There is no fallback: if libqsim.so is missing the import fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsim.so")

QS_OK, QS_EINVAL, QS_ENOMEM, QS_EDEVICE, QS_ERANGE, QS_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
QS_C64, QS_C128 = 0, 1
STRATEGY_NONE, STRATEGY_GREEDY, STRATEGY_LEARNED, STRATEGY_PAULI = 0, 1, 2, 3
PROF_PLAIN, PROF_TILE, PROF_REDUCE, PROF_EXPECT, PROF_COPY = range(5)

# qsynth gate names -> qs_kind
KIND = {
    "h": 0, "x": 1, "y": 2, "z": 3, "s": 4, "sdg": 5, "t": 6, "tdg": 7,
    "rx": 8, "ry": 9, "rz": 10, "u3": 11, "p": 12,
    "cx": 13, "cz": 14, "cp": 15, "cu": 16, "swap": 17, "dense": 18,
}


class QsimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"qsim status {status}: {msg}")
        self.status = status


class qs_gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nq", ctypes.c_int32), ("qubits", ctypes.c_int32 * 8),
                ("params", ctypes.c_double * 4), ("matrix", ctypes.c_void_p)]


class qs_contract_opts(ctypes.Structure):
    _fields_ = [("k_max", ctypes.c_int32), ("tile_qubits", ctypes.c_int32), ("low_qubits", ctypes.c_int32),
                ("strategy", ctypes.c_int32), ("renorm", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("commute", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class qs_plan_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("max_k", ctypes.c_int32), ("n_gates", ctypes.c_uint64),
                ("n_blocks", ctypes.c_uint64), ("n_passes", ctypes.c_uint64),
                ("blocks_by_k", ctypes.c_uint64 * 8), ("flops_per_amp", ctypes.c_double)]


class qs_profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64 * 5), ("ms", ctypes.c_double * 5),
                ("bytes", ctypes.c_double * 5), ("flops", ctypes.c_double * 5)]


assert ctypes.sizeof(qs_gate) == 80

_lib = None
_vp, _u64, _i32, _dbl = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
_SIGS = {
    "qs_last_error": ([], ctypes.c_char_p),
    "qs_version": ([], ctypes.c_char_p),
    "qs_device_query": ([_vp, _vp, ctypes.c_char_p, ctypes.c_size_t], _i32),
    "qs_state_create": ([_i32, _i32, _vp, _vp, _vp], _i32),
    "qs_state_destroy": ([_vp], _i32),
    "qs_state_data": ([_vp, _vp], _i32),
    "qs_state_set_basis": ([_vp, _u64], _i32),
    "qs_state_normalize": ([_vp], _i32),
    "qs_state_copy_out": ([_vp, _u64, _u64, _vp], _i32),
    "qs_state_copy_in": ([_vp, _u64, _u64, _vp], _i32),
    "qs_norm": ([_vp, _vp], _i32),
    "qs_apply_gates": ([_vp, _vp, ctypes.c_size_t], _i32),
    "qs_apply_gates_smgp": ([_vp, _vp, ctypes.c_size_t], _i32),
    "qs_contract": ([_i32, _vp, ctypes.c_size_t, _vp, _vp], _i32),
    "qs_plan_destroy": ([_vp], _i32),
    "qs_plan_info_get": ([_vp, _vp], _i32),
    "qs_plan_block": ([_vp, _u64, _vp, _vp, _vp, _vp, _u64, _vp], _i32),
    "qs_plan_pass": ([_vp, _u64, _vp, _vp, _vp, _vp], _i32),
    "qs_apply_plan": ([_vp, _vp], _i32),
    "qs_expect_pauli_sum": ([_vp, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp], _i32),
    "qs_expect_pauli_sum_noalloc": ([_vp, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp], _i32),
    "qs_batch_create": ([_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "qs_batch_destroy": ([_vp], _i32),
    "qs_batch_run": ([_vp, _vp], _i32),
    "qs_batch_state_copy_out": ([_vp, _i32, _vp], _i32),
    "qs_autotune": ([_i32, _i32, _vp, ctypes.c_size_t, _vp, _vp], _i32),
    "qs_costmodel_num_features": ([], _i32),
    "qs_costmodel_num_weights": ([], _i32),
    "qs_plan_pass_features": ([_vp, _vp, _u64], _i32),
    "qs_plan_time_passes": ([_vp, _i32, _i32, _vp], _i32),
    "qs_costmodel_train": ([_vp, _vp, _i32, _i32, _i32, ctypes.c_float, _u64, _vp, _vp], _i32),
    "qs_costmodel_set_weights": ([_vp], _i32),
    "qs_costmodel_get_weights": ([_vp], _i32),
    "qs_costmodel_predict": ([_vp, _i32, _vp], _i32),
    "qs_costmodel_grad": ([_vp, _vp, _vp, _i32, _vp, _vp], _i32),
    "qs_profile_enable": ([_i32], _i32),
    "qs_profile_collect": ([_vp], _i32),
    "qs_copy": ([_vp, _vp, _u64, _vp], _i32),
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2509_04955_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(status: int):
    if status != QS_OK:
        raise QsimError(status, lib().qs_last_error().decode())


def _p(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return ctypes.c_void_p(a.ctypes.data)
    return ctypes.byref(a)


# ------------------------------------------------------------ gate lists
class GateList:
    """A circuit marshalled into a contiguous qs_gate array (keeps dense
    matrices alive)."""

    def __init__(self, circuit):
        self.n = circuit.n
        gates = circuit.gates
        self.arr = (qs_gate * max(1, len(gates)))()
        self.count = len(gates)
        self._keep = []
        for i, g in enumerate(gates):
            e = self.arr[i]
            e.kind = KIND[g.name]
            e.nq = len(g.qubits)
            for j, q in enumerate(g.qubits):
                e.qubits[j] = q
            for j, v in enumerate(g.params):
                e.params[j] = v
            if g.matrix is not None:
                m = np.ascontiguousarray(np.asarray(g.matrix, dtype=np.complex128)).view(np.float64).copy()
                self._keep.append(m)
                e.matrix = m.ctypes.data
            else:
                e.matrix = None

    @property
    def ptr(self):
        return ctypes.cast(self.arr, ctypes.c_void_p)


def opts(k_max=0, tile_qubits=0, low_qubits=0, strategy=STRATEGY_GREEDY, renorm=1, dtype=QS_C64, commute=0):
    o = qs_contract_opts()
    o.k_max, o.tile_qubits, o.low_qubits = k_max, tile_qubits, low_qubits
    o.strategy, o.renorm, o.dtype, o.commute = strategy, renorm, dtype, commute
    return o


# ---------------------------------------------------------------- C names
def qs_version() -> str:
    return lib().qs_version().decode()


def qs_device_query():
    cu, lds = ctypes.c_int(), ctypes.c_int()
    arch = ctypes.create_string_buffer(64)
    _check(lib().qs_device_query(ctypes.byref(cu), ctypes.byref(lds), arch, 64))
    return cu.value, lds.value, arch.value.decode()


def qs_state_create(n: int, dtype: int, dev_ptr: int | None, stream: int | None):
    h = ctypes.c_void_p()
    _check(lib().qs_state_create(n, dtype, dev_ptr, stream, ctypes.byref(h)))
    return h


def qs_state_destroy(h):
    _check(lib().qs_state_destroy(h))


def qs_state_set_basis(h, index: int):
    _check(lib().qs_state_set_basis(h, index))


def qs_state_normalize(h):
    _check(lib().qs_state_normalize(h))


def qs_state_copy_out(h, offset: int, count: int) -> np.ndarray:
    out = np.empty(2 * count, dtype=np.float64)
    _check(lib().qs_state_copy_out(h, offset, count, _p(out)))
    return out.view(np.complex128)


def qs_state_copy_in(h, offset: int, values: np.ndarray):
    v = np.ascontiguousarray(values, dtype=np.complex128).view(np.float64)
    _check(lib().qs_state_copy_in(h, offset, len(v) // 2, _p(v)))


def qs_norm(h) -> float:
    v = ctypes.c_double()
    _check(lib().qs_norm(h, ctypes.byref(v)))
    return v.value


def qs_apply_gates(h, gl: GateList):
    _check(lib().qs_apply_gates(h, gl.ptr, gl.count))


def qs_apply_gates_smgp(h, gl: GateList):
    _check(lib().qs_apply_gates_smgp(h, gl.ptr, gl.count))


def qs_contract(n: int, gl: GateList, o: qs_contract_opts | None = None):
    p = ctypes.c_void_p()
    _check(lib().qs_contract(n, gl.ptr, gl.count, ctypes.byref(o) if o is not None else None, ctypes.byref(p)))
    return p


def qs_plan_destroy(p):
    _check(lib().qs_plan_destroy(p))


def qs_plan_info_get(p) -> qs_plan_info:
    info = qs_plan_info()
    _check(lib().qs_plan_info_get(p, ctypes.byref(info)))
    return info


def qs_plan_block(p, b: int, with_matrix: bool = True):
    k = ctypes.c_int()
    nm = ctypes.c_uint64()
    _check(lib().qs_plan_block(p, b, ctypes.byref(k), None, None, None, 0, ctypes.byref(nm)))
    qs = np.zeros(k.value, dtype=np.int32)
    mat = np.zeros(2 * (1 << (2 * k.value)), dtype=np.float64) if with_matrix else None
    mem = np.zeros(nm.value, dtype=np.uint64)
    _check(lib().qs_plan_block(p, b, ctypes.byref(k), _p(qs), _p(mat), _p(mem), nm.value, ctypes.byref(nm)))
    d = 1 << k.value
    U = mat.view(np.complex128).reshape(d, d) if with_matrix else None
    return tuple(int(q) for q in qs), U, [int(m) for m in mem]


def qs_plan_pass(p, i: int):
    t = ctypes.c_int()
    fb, nb = ctypes.c_uint64(), ctypes.c_uint64()
    tq = np.zeros(64, dtype=np.int32)
    _check(lib().qs_plan_pass(p, i, ctypes.byref(t), _p(tq), ctypes.byref(fb), ctypes.byref(nb)))
    return t.value, tuple(int(q) for q in tq[: t.value]), fb.value, nb.value


def qs_apply_plan(h, p):
    _check(lib().qs_apply_plan(h, p))


def qs_expect_pauli_sum(h, x, z, coeff, with_terms: bool = False):
    x = np.ascontiguousarray(x, dtype=np.uint64)
    z = np.ascontiguousarray(z, dtype=np.uint64)
    c = np.ascontiguousarray(coeff, dtype=np.float64)
    out = ctypes.c_double()
    terms = np.zeros(len(c), dtype=np.float64) if with_terms else None
    _check(lib().qs_expect_pauli_sum(h, _p(x), _p(z), _p(c), len(c), ctypes.byref(out), _p(terms)))
    return (out.value, terms) if with_terms else out.value


def qs_expect_pauli_sum_noalloc(h, x, z, coeff, with_terms: bool = False):
    x = np.ascontiguousarray(x, dtype=np.uint64)
    z = np.ascontiguousarray(z, dtype=np.uint64)
    c = np.ascontiguousarray(coeff, dtype=np.float64)
    out = ctypes.c_double()
    terms = np.zeros(len(c), dtype=np.float64) if with_terms else None
    _check(lib().qs_expect_pauli_sum_noalloc(h, _p(x), _p(z), _p(c), len(c), ctypes.byref(out), _p(terms)))
    return (out.value, terms) if with_terms else out.value


class Batch:
    """A batch of states run by one persistent kernel in a hipGraph
    (qs_batch_create / qs_batch_run)."""

    def __init__(self, circuits, hams, o: qs_contract_opts | None = None, stream: int | None = None):
        self.n = [c.n for c in circuits]
        count = len(circuits)
        self._gls = [GateList(c) for c in circuits]
        self._x = [np.ascontiguousarray(h.x, dtype=np.uint64) for h in hams]
        self._z = [np.ascontiguousarray(h.z, dtype=np.uint64) for h in hams]
        self._c = [np.ascontiguousarray(h.coeff, dtype=np.float64) for h in hams]
        nq = (ctypes.c_int * count)(*self.n)
        circ = (ctypes.c_void_p * count)(*[g.ptr.value for g in self._gls])
        ng = (ctypes.c_size_t * count)(*[g.count for g in self._gls])
        xs = (ctypes.c_void_p * count)(*[a.ctypes.data for a in self._x])
        zs = (ctypes.c_void_p * count)(*[a.ctypes.data for a in self._z])
        cs = (ctypes.c_void_p * count)(*[a.ctypes.data for a in self._c])
        nt = (ctypes.c_size_t * count)(*[len(a) for a in self._c])
        self.handle = ctypes.c_void_p()
        _check(lib().qs_batch_create(count, nq, circ, ng, xs, zs, cs, nt,
                                     ctypes.byref(o) if o is not None else None, stream, ctypes.byref(self.handle)))

    def run(self) -> np.ndarray:
        out = np.zeros(len(self.n), dtype=np.float64)
        _check(lib().qs_batch_run(self.handle, _p(out)))
        return out

    def amplitudes(self, i: int) -> np.ndarray:
        out = np.zeros(2 << self.n[i], dtype=np.float64)
        _check(lib().qs_batch_state_copy_out(self.handle, i, _p(out)))
        return out.view(np.complex128)

    def close(self):
        if self.handle:
            lib().qs_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def qs_autotune(n: int, dtype: int, gl: GateList, base: qs_contract_opts | None = None) -> qs_contract_opts:
    best = qs_contract_opts()
    _check(lib().qs_autotune(n, dtype, gl.ptr, gl.count, ctypes.byref(base) if base is not None else None,
                             ctypes.byref(best)))
    return best


def qs_profile_enable(on: bool):
    _check(lib().qs_profile_enable(1 if on else 0))


def qs_profile_collect() -> qs_profile:
    p = qs_profile()
    _check(lib().qs_profile_collect(ctypes.byref(p)))
    return p


def qs_copy(dst: int, src: int, nbytes: int, stream: int | None):
    _check(lib().qs_copy(dst, src, nbytes, stream))


# ------------------------------------------------------- torch helpers
class State:
    """A state whose amplitudes live in a torch tensor on the current HIP
    device; all work runs on the torch current stream."""

    def __init__(self, n: int, dtype: int = QS_C64, device: str = "cuda"):
        import torch

        self.n = n
        self.dtype = dtype
        tdt = torch.complex64 if dtype == QS_C64 else torch.complex128
        self.tensor = torch.empty(1 << n, dtype=tdt, device=device)
        stream = torch.cuda.current_stream().cuda_stream
        self.handle = qs_state_create(n, dtype, self.tensor.data_ptr(), stream)
        qs_state_set_basis(self.handle, 0)

    def close(self):
        if self.handle is not None:
            qs_state_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_basis(self, index: int = 0):
        qs_state_set_basis(self.handle, index)

    def load(self, values: np.ndarray):
        qs_state_copy_in(self.handle, 0, values)

    def amplitudes(self) -> np.ndarray:
        return qs_state_copy_out(self.handle, 0, 1 << self.n)

    def norm(self) -> float:
        return qs_norm(self.handle)

    def apply_gates(self, gl: GateList):
        qs_apply_gates(self.handle, gl)

    def apply_gates_smgp(self, gl: GateList):
        qs_apply_gates_smgp(self.handle, gl)

    def apply_plan(self, plan):
        qs_apply_plan(self.handle, plan)

    def expect(self, ham, with_terms=False):
        return qs_expect_pauli_sum(self.handle, ham.x, ham.z, ham.coeff, with_terms)
