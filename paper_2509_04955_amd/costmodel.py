"""Cost-model harness: measured pass timings -> MLP training on the device ->
learned contraction plans.

The data are the library's own kernel timings: for a set of circuits, every
pass of the fixed-width greedy plan at widths k = 1..kmax and tile sizes t is
timed on the device (qs_plan_time_passes, median of hipEvent-timed launches)
and described by the pass features (qs_plan_pass_features).  The MLP learns
log(microseconds) from the features with the library's forward/backward/Adam
kernels (qs_costmodel_train); qs_contract with STRATEGY_LEARNED then uses it
to pick the width per window.  All numerics run in libqsim.
"""
from __future__ import annotations

import ctypes
import itertools
import math

import numpy as np

from . import qsim as Q


def pass_features(plan) -> np.ndarray:
    info = Q.qs_plan_info_get(plan)
    F = Q.lib().qs_costmodel_num_features()
    out = np.zeros((int(info.n_passes), F), dtype=np.float32)
    Q._check(Q.lib().qs_plan_pass_features(plan, Q._p(out), out.shape[0]))
    return out


def time_passes(plan, dtype: int, reps: int = 3) -> np.ndarray:
    info = Q.qs_plan_info_get(plan)
    us = np.zeros(int(info.n_passes), dtype=np.float64)
    Q._check(Q.lib().qs_plan_time_passes(plan, dtype, reps, Q._p(us)))
    return us


def collect(circuits, dtype: int = Q.QS_C64, widths=(1, 2, 3, 4, 5, 6), tiles=(12, 13), reps: int = 3,
            max_passes: int = 64, lows=(0,), strategies=(Q.STRATEGY_GREEDY,)):
    """Timing dataset over circuits x strategies x widths x tiles x
    fixed-low-qubit counts (0 = the library default; the first `max_passes`
    passes of each plan are timed).  STRATEGY_PAULI adds the passes of
    rotation-contracted plans (rotation blocks beside greedy blocks of each
    width).  Returns (X, target, us)."""
    xs, ys = [], []
    for c in circuits:
        gl = Q.GateList(c)
        for strat, t, low, k in itertools.product(strategies, tiles, lows, widths):
            if dtype == Q.QS_C128 and k > 5:
                continue
            try:
                plan = Q.qs_contract(c.n, gl, Q.opts(k_max=k, tile_qubits=t, low_qubits=low, dtype=dtype,
                                                     strategy=strat))
            except Q.QsimError:
                continue
            try:
                feats = pass_features(plan)[:max_passes]
                # time a plan restricted to its first passes: prefix circuit
                us = time_passes(plan, dtype, reps)[: len(feats)]
            finally:
                Q.qs_plan_destroy(plan)
            xs.append(feats)
            ys.append(us)
    X = np.concatenate(xs).astype(np.float32)
    us = np.concatenate(ys)
    return X, target(us, X), us


def target(us: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Training target: log of the pass time scaled to 2^30 amplitudes
    (log(us) - (n - 30) ln 2, n = 32 * feature 0).  A pass streams the whole
    state, so this removes the size dependence the model would otherwise
    have to extrapolate; candidate passes of one plan share n, so the
    planner's choice is unchanged by the shift."""
    n = np.rint(X[:, 0] * 32.0)
    return (np.log(us) - (n - 30.0) * math.log(2.0)).astype(np.float32)


def refine(X: np.ndarray, y: np.ndarray, circuits, rounds: int = 2, reps: int = 3, epochs: int = 300,
           batch: int = 64, lr: float = 3e-3, seed: int = 1, dtype: int = Q.QS_C64, **plan_opts):
    """Train on the model's own choices: plan each circuit with the learned
    strategy under the active model, time every pass of that plan, add those
    rows to (X, y) and retrain; `rounds` times.  The passes the learned
    partition proposes are the ones the fixed-width sweep in collect() rarely
    contains.  Returns the grown (X, y) and the last training loss."""
    loss = None
    for r in range(rounds):
        xs, ys = [X], [y]
        for c in circuits:
            plan = Q.qs_contract(c.n, Q.GateList(c), Q.opts(strategy=Q.STRATEGY_LEARNED, dtype=dtype, **plan_opts))
            try:
                f = pass_features(plan)
                us = time_passes(plan, dtype, reps)
            finally:
                Q.qs_plan_destroy(plan)
            xs.append(f)
            ys.append(target(us, f))
        X = np.concatenate(xs).astype(np.float32)
        y = np.concatenate(ys).astype(np.float32)
        loss = train(X, y, epochs=epochs, batch=batch, lr=lr, seed=seed + r + 1)
    return X, y, loss


def train(X: np.ndarray, y: np.ndarray, epochs: int = 400, batch: int = 64, lr: float = 3e-3, seed: int = 1):
    """Train on the device; the trained model becomes the active one."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    loss = ctypes.c_float()
    Q._check(Q.lib().qs_costmodel_train(Q._p(X), Q._p(y), len(y), epochs, batch, ctypes.c_float(lr), seed, None,
                                        ctypes.byref(loss)))
    return float(loss.value)


def predict(X: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float32)
    out = np.zeros(len(X), dtype=np.float32)
    Q._check(Q.lib().qs_costmodel_predict(Q._p(X), len(X), Q._p(out)))
    return out


def get_weights() -> np.ndarray:
    w = np.zeros(Q.lib().qs_costmodel_num_weights(), dtype=np.float32)
    Q._check(Q.lib().qs_costmodel_get_weights(Q._p(w)))
    return w


def set_weights(w: np.ndarray | None):
    if w is None:
        Q._check(Q.lib().qs_costmodel_set_weights(None))
        return
    w = np.ascontiguousarray(w, dtype=np.float32)
    Q._check(Q.lib().qs_costmodel_set_weights(Q._p(w)))


def grad(w: np.ndarray, X: np.ndarray, y: np.ndarray):
    """One device forward+backward: (loss, gradient) for weights w."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    g = np.zeros_like(w)
    loss = ctypes.c_float()
    Q._check(Q.lib().qs_costmodel_grad(Q._p(w), Q._p(X), Q._p(y), len(y), Q._p(g), ctypes.byref(loss)))
    return float(loss.value), g


def unflatten(w: np.ndarray, F: int, H1: int = 64, H2: int = 64) -> dict:
    """Flat weight array -> named matrices (W1 H1xF, b1, W2 H2xH1, b2, W3 1xH2, b3)."""
    o = 0
    out = {}
    for name, shape in (("W1", (H1, F)), ("b1", (H1,)), ("W2", (H2, H1)), ("b2", (H2,)), ("W3", (1, H2)),
                        ("b3", (1,))):
        size = int(np.prod(shape))
        out[name] = np.asarray(w[o:o + size], dtype=np.float64).reshape(shape)
        o += size
    return out


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], dtype=np.float32).ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def measure_plan(state, plan, reps: int = 3) -> float:
    """Median wall time (ms) of applying a plan to a state, HIP events on the
    torch current stream."""
    import torch

    st = torch.cuda.current_stream()
    times = []
    state.apply_plan(plan)
    torch.cuda.synchronize()
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        state.apply_plan(plan)
        e1.record(st)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times))
