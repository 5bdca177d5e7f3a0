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


def _check_plan_exact(Q, oracle, G, c, plan, n):
    """Plan checker on the oracle side (FP64): every gate in exactly one
    block, and the blocks' matrices applied in plan order to a random state
    give the oracle's state of the circuit.  (The plain DAG-order check does
    not apply: rotation blocks whose Pauli strings commute may overtake each
    other; the replay from a random state is what shows the plan exact.)"""
    qls, mats, mems = _blocks(Q, plan)
    flat = sorted(g for m in mems for g in m)
    assert flat == list(range(len(c.gates))), "gates missing from or repeated in the plan"
    psi0 = qsynth.random_state(n, seed=17)
    ref = oracle.run(c, psi0.copy())
    replay = G.apply_blocks(psi0.copy(), n, qls, mats)
    assert oracle.max_abs(ref, replay) <= 1e-12
    return mems


@pytest.fixture(scope="module")
def trained(CM):
    """The MLP trained on the library's own pass timings at 22 qubits: greedy
    plans of every width on a UCC, a brickwork and a random circuit, and the
    UCC circuit's rotation-contracted plans."""
    from paper_2509_04955_amd import qsim as Q

    n = 22
    ucc = qsynth.ucc(n, 30, seed=11)[0]
    train_c = [ucc, qsynth.brickwork(n, 8, seed=12), qsynth.random_u3_cnot(n, 8, seed=13)]
    X, y, us = CM.collect(train_c, widths=(1, 2, 3, 4, 5, 6), tiles=(12,), reps=3, max_passes=24)
    Xp, yp, usp = CM.collect([ucc], widths=(2, 3, 4), tiles=(12,), reps=3, max_passes=24,
                             strategies=(Q.STRATEGY_PAULI,))
    X, y, us = np.concatenate([X, Xp]), np.concatenate([y, yp]), np.concatenate([us, usp])
    assert len(y) >= 50 and np.all(us > 0)
    loss = CM.train(X, y, epochs=300, batch=32, lr=3e-3, seed=2)
    pred = CM.predict(X)
    corr = np.corrcoef(pred, y)[0, 1]
    assert loss < 0.5 and corr > 0.8, (loss, corr)
    w = CM.get_weights()
    yield w
    CM.set_weights(None)


def test_training_fits_measured_timings_and_learned_plan_is_exact_and_faster(CM, oracle, trained):
    """Timings of the library's own passes at 22 qubits train the MLP.  The
    learned partition of a held-out UCC circuit must differ from the greedy
    plan it falls back to (k_max 5, the library default), give the oracle's
    state on the GPU in both precisions, and run faster than that greedy
    plan; a 16-qubit learned plan replays exactly on the oracle (plan
    checker: every gate once, blocks in plan order against the oracle from a
    random state)."""
    from oracle import greedy as G
    from paper_2509_04955_amd import qsim as Q

    CM.set_weights(trained)
    n = 22
    c, rots = qsynth.ucc(n, 60, seed=21)
    gl = Q.GateList(c)
    greedy = Q.qs_contract(n, gl, Q.opts(k_max=5, tile_qubits=12))
    learned = Q.qs_contract(n, gl, Q.opts(k_max=5, tile_qubits=12, strategy=Q.STRATEGY_LEARNED))
    # the learned partition is not the greedy one
    _, _, mem_g = _blocks(Q, greedy)
    _, _, mem_l = _blocks(Q, learned)
    assert sorted(map(tuple, mem_l)) != sorted(map(tuple, mem_g)), "learned plan equals the greedy plan"
    # host replay of a learned plan (16 qubits: the FP64 replay of 8-qubit
    # rotation blocks at 22 qubits would take minutes)
    c16 = qsynth.ucc(16, 40, seed=22)[0]
    p16 = Q.qs_contract(16, Q.GateList(c16), Q.opts(k_max=5, tile_qubits=12, strategy=Q.STRATEGY_LEARNED))
    try:
        _check_plan_exact(Q, oracle, G, c16, p16, 16)
    finally:
        Q.qs_plan_destroy(p16)
    ref = oracle.zero_state(n)
    for x, z, th in rots:
        oracle.pauli_rotation(ref, n, x, z, th)
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


def test_learned_beats_autotuned_greedy_on_rotation_circuits(CM, trained):
    """On a 26-qubit UCC circuit the learned partition, in the tile shape and
    width the autotuner picked for the greedy rule, may contract runs of
    windows as Pauli rotations where the model predicts a gain: it must beat
    that autotuned greedy plan by at least 5 % (median of 5 timings each; the
    gap is far above the run-to-run spread of these timings) and give the
    greedy plan's state (fidelity 1 - 1e-6; both plans are checked against
    the oracle in the other tests)."""
    from paper_2509_04955_amd import qsim as Q

    CM.set_weights(trained)
    n = 26
    c = qsynth.ucc(n, 120, seed=23)[0]
    gl = Q.GateList(c)
    best = Q.qs_autotune(n, Q.QS_C64, gl, Q.opts(strategy=Q.STRATEGY_GREEDY, renorm=1))
    kw = dict(k_max=best.k_max, tile_qubits=best.tile_qubits, low_qubits=best.low_qubits)
    greedy = Q.qs_contract(n, gl, Q.opts(**kw))
    learned = Q.qs_contract(n, gl, Q.opts(strategy=Q.STRATEGY_LEARNED, **kw))
    s = Q.State(n, Q.QS_C64)
    tg = [CM.measure_plan(s, greedy) for _ in range(5)]
    tl = [CM.measure_plan(s, learned) for _ in range(5)]
    s.set_basis(0)
    s.apply_plan(greedy)
    a = s.amplitudes()
    s.set_basis(0)
    s.apply_plan(learned)
    b = s.amplitudes()
    s.close()
    ig, il = Q.qs_plan_info_get(greedy), Q.qs_plan_info_get(learned)
    Q.qs_plan_destroy(greedy)
    Q.qs_plan_destroy(learned)
    f = abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)
    assert 1 - f <= 1e-6
    mg, ml = float(np.median(tg)), float(np.median(tl))
    print(f"autotuned greedy (k_max {best.k_max}, t {best.tile_qubits}, low {best.low_qubits}): "
          f"{mg:.3f} ms [{min(tg):.3f}, {max(tg):.3f}], {ig.n_passes} passes; learned {ml:.3f} ms "
          f"[{min(tl):.3f}, {max(tl):.3f}], {il.n_passes} passes; gain {mg / ml:.2f}x")
    assert ml <= 0.95 * mg
