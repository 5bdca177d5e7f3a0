"""Cost-model MLP on the GPU: forward, backward and Adam kernels against the
FP64 reference (oracle/mlp.py), training on measured pass timings, and what
the learned contraction gains over the fixed-width greedy rule."""
import numpy as np
import pytest

import qsynth
from oracle import mlp as ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def CM():
    import torch

    from paper_2509_04955_amd import costmodel, qsim

    assert torch.cuda.is_available()
    qsim.lib()
    return costmodel


def _random_problem(F, B, seed):
    rng = np.random.default_rng(seed)
    p = ref.init(F, 64, 64, seed=seed)
    p["b1"] = rng.normal(0, 0.1, size=64)
    p["b2"] = rng.normal(0, 0.1, size=64)
    X = rng.normal(size=(B, F)).astype(np.float32).astype(np.float64)
    t = rng.normal(size=B).astype(np.float32).astype(np.float64)
    return p, X, t


def test_forward_and_gradient_match_fp64(CM):
    """FP32 device kernels vs the FP64 reference: predictions within 1e-4
    relative, gradients within 1e-3 relative to the largest entry of each
    weight matrix (FP32 accumulation over 96 samples)."""
    from paper_2509_04955_amd import qsim as Q

    F = Q.lib().qs_costmodel_num_features()
    p, X, t = _random_problem(F, 96, 3)
    w = CM.flatten(p)
    p32 = CM.unflatten(w, F)  # the FP32-rounded weights the device sees
    y_ref, cache = ref.forward(p32, X)
    g_ref = ref.backward(p32, cache, y_ref, t)
    loss_ref = float(np.mean((y_ref - t) ** 2))
    CM.set_weights(w)
    y = CM.predict(X.astype(np.float32))
    assert np.max(np.abs(y - y_ref)) <= 1e-4 * max(1.0, np.max(np.abs(y_ref)))
    loss, g = CM.grad(w, X.astype(np.float32), t.astype(np.float32))
    assert abs(loss - loss_ref) <= 1e-4 * max(1.0, loss_ref)
    gd = CM.unflatten(g, F)
    for name in ref.NAMES:
        scale = max(1e-6, np.max(np.abs(g_ref[name])))
        assert np.max(np.abs(gd[name] - g_ref[name])) <= 1e-3 * scale, name


def test_single_adam_step_matches_reference(CM):
    """One Adam step (batch = whole data set) on the device equals the FP64
    reference update to FP32 precision."""
    from paper_2509_04955_amd import qsim as Q
    import ctypes

    F = Q.lib().qs_costmodel_num_features()
    p, X, t = _random_problem(F, 64, 5)
    w0 = CM.flatten(p)
    p32 = CM.unflatten(w0, F)
    y, cache = ref.forward(p32, X)
    g = ref.backward(p32, cache, y, t)
    ref.adam_step(p32, g, {}, lr=1e-2)
    loss = ctypes.c_float()
    Xf = np.ascontiguousarray(X, dtype=np.float32)
    tf = np.ascontiguousarray(t, dtype=np.float32)
    Q._check(Q.lib().qs_costmodel_train(Q._p(Xf), Q._p(tf), 64, 1, 64, ctypes.c_float(1e-2), 0, Q._p(w0),
                                        ctypes.byref(loss)))
    got = CM.unflatten(CM.get_weights(), F)
    for name in ref.NAMES:
        assert np.max(np.abs(got[name] - p32[name])) <= 2e-5, name


def _blocks(Q, plan):
    info = Q.qs_plan_info_get(plan)
    qls, mats, mems = [], [], []
    for b in range(info.n_blocks):
        qs, U, mem = Q.qs_plan_block(plan, b)
        qls.append(qs)
        mats.append(U)
        mems.append(list(mem))
    return qls, mats, mems


def test_training_fits_measured_timings_and_learned_plan_is_exact_and_faster(CM, oracle):
    """Timings of the library's own passes at 22 qubits train the MLP.  The
    learned partition of a held-out UCC circuit must differ from the greedy
    plan it falls back to (k_max 5, the library default), replay exactly on
    the oracle (plan checker: blocks in plan order against the closed-form
    rotations, DAG order of gates on shared qubits), give the oracle's state on
    the GPU in both precisions, and run faster than that greedy plan."""
    from oracle import greedy as G
    from paper_2509_04955_amd import qsim as Q

    n = 22
    train_c = [qsynth.ucc(n, 30, seed=11)[0], qsynth.brickwork(n, 8, seed=12), qsynth.random_u3_cnot(n, 8, seed=13)]
    X, y, us = CM.collect(train_c, widths=(1, 2, 3, 4, 5, 6), tiles=(12,), reps=3, max_passes=24)
    assert len(y) >= 50 and np.all(us > 0)
    loss = CM.train(X, y, epochs=300, batch=32, lr=3e-3, seed=2)
    pred = CM.predict(X)
    corr = np.corrcoef(pred, y)[0, 1]
    assert loss < 0.5 and corr > 0.8, (loss, corr)
    c, rots = qsynth.ucc(n, 60, seed=21)
    gl = Q.GateList(c)
    greedy = Q.qs_contract(n, gl, Q.opts(k_max=5, tile_qubits=12))
    learned = Q.qs_contract(n, gl, Q.opts(k_max=5, tile_qubits=12, strategy=Q.STRATEGY_LEARNED))
    # the learned partition is not the greedy one
    _, _, mem_g = _blocks(Q, greedy)
    qls, mats, mem_l = _blocks(Q, learned)
    assert sorted(map(tuple, mem_l)) != sorted(map(tuple, mem_g)), "learned plan equals the greedy plan"
    # plan checker on the oracle side (FP64)
    G.check_order(c.gates, mem_l)
    ref = oracle.zero_state(n)
    for x, z, th in rots:
        oracle.pauli_rotation(ref, n, x, z, th)
    replay = G.apply_blocks(oracle.zero_state(n), n, qls, mats)
    assert oracle.max_abs(ref, replay) <= 1e-12
    s = Q.State(n, Q.QS_C64)
    t_g = CM.measure_plan(s, greedy)
    t_l = CM.measure_plan(s, learned)
    s.set_basis(0)
    s.apply_plan(learned)
    got = s.amplitudes()
    s.close()
    assert oracle.max_abs(ref, got) <= 1e-5
    assert 1 - oracle.fidelity(ref, got) <= 1e-6
    learned128 = Q.qs_contract(n, gl, Q.opts(k_max=5, tile_qubits=12, strategy=Q.STRATEGY_LEARNED, dtype=Q.QS_C128))
    s = Q.State(n, Q.QS_C128)
    s.set_basis(0)
    s.apply_plan(learned128)
    got128 = s.amplitudes()
    s.close()
    assert oracle.max_abs(ref, got128) <= 1e-12
    print(f"greedy k_max 5 {t_g:.3f} ms, learned {t_l:.3f} ms, gain {t_g / t_l:.3f}x")
    assert t_l < t_g
    for p in (greedy, learned, learned128):
        Q.qs_plan_destroy(p)
    CM.set_weights(None)
