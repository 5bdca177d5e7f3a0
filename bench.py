"""Benchmark: 30-qubit UCC-style ansatz, complex64, fused tile passes vs
plain gate-by-gate on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Workload (seeded, synthetic): 2000 Pauli exponentials exp(-i theta P), P of
weight 4..8 on random qubits with random X/Y/Z letters, theta ~ N(0, 0.1),
each compiled to basis changes + CNOT ladder + RZ (about 38k gates), applied
to |0...0> of 30 qubits in complex64 (8 GiB).  One step = reset the state
and run the whole contracted circuit (every tile pass with its FP64
renormalisation); the contraction plan (host) is built once before timing and
its time is reported separately.

Prints one JSON line.  `value` is the bandwidth of the fused circuit by the
algorithmic bytes of the method that ran: each tile pass reads and writes the
state once (2S, S = state bytes), plus the reset of the state to |0...0> at
the start of a step (one write, S), divided by the circuit time.  `gate_by_gate_equivalent` states what the plain
gate-by-gate method would have to stream for the same circuit (per gate 2S for
a general or diagonal 1-qubit gate, S for a phase gate, CNOT-type or SWAP,
S/2 for CZ-type) and that volume over the fused time: a speed measure, not an
HBM rate.  `roofline` is the tile kernel against the HBM (or MFMA) peak, and
`accuracy` runs the circuit's inverse after the timed steps (exact result
|0...0>) and states the round trip's error.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
import types

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
MFMA_FP32_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix
VALU_FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector
METRIC = "circuit wall time + effective HBM GB/s at 30q fp32; fused vs gate-by-gate"


# bytes one gate costs the gate-by-gate method (multiples of the state size),
# following which plain kernel the library launches for it
PLAIN_BYTES = {"z": 1.0, "s": 1.0, "sdg": 1.0, "t": 1.0, "tdg": 1.0, "p": 1.0, "cx": 1.0, "cu": 1.0,
               "swap": 1.0, "cz": 0.5, "cp": 0.5}


def plain_bytes(circ, S):
    return sum(PLAIN_BYTES.get(g.name, 2.0) for g in circ.gates) * S


def measured_traffic(n_qubits):
    """HBM bytes per tile-pass launch from the committed rocprofv3 counter
    summary (FETCH_SIZE x 2 + WRITE_SIZE x 1, copy-kernel calibrated), or None
    when the tile-kernel sources changed since the counters were taken or the
    workload is not the profiled 30-qubit one."""
    import hashlib
    import re

    path = os.path.join(ROOT, "profiles", "hbm_traffic_counters_ucc30.md")
    if n_qubits != 30 or not os.path.exists(path):
        return None
    text = open(path).read()
    m_t = re.search(r"^traffic_bytes_per_launch:\s*(\d+)", text, re.M)
    m_f = re.search(r"^kernel_source_fingerprint:\s*([0-9a-f]+)", text, re.M)
    if not m_t or not m_f:
        return None
    h = hashlib.sha256()
    for f in ("kernels_tile.hip", "tile_device.h", "internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2509_04955_amd", "csrc", f), "rb").read())
    return int(m_t.group(1)) if h.hexdigest()[:16] == m_f.group(1) else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--n-exp", type=int, default=2000)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--k-max", type=int, default=0, help="0 = autotune (with --tile)")
    ap.add_argument("--tile", type=int, default=0, help="0 = autotune (with --k-max)")
    ap.add_argument("--low", type=int, default=0, help="fixed low qubits per tile; 0 = autotuned / library default")
    ap.add_argument("--strategy", type=int, default=1)
    ap.add_argument("--pauli", type=int, default=1,
                    help="ucc mode with the greedy strategy: also time the Pauli-rotation contraction "
                         "(strategy 3, autotuned) and compare its final state with the greedy one")
    ap.add_argument("--plain-prefix", type=int, default=40,
                    help="Pauli exponentials timed gate-by-gate vs fused (0 = skip)")
    ap.add_argument("--cpu-gates", type=int, default=80,
                    help="gates of the circuit the FP64 oracle runs at full size (0 = skip)")
    ap.add_argument("--mode", default="ucc",
                    choices=["ucc", "copy", "batch", "learned", "brickwork", "plain12", "families"],
                    help="ucc: the benchmark line; copy: device copy of one state-sized buffer "
                         "(achievable streaming bandwidth and counter calibration); batch: 256 HEA states "
                         "in one graph launch; learned: cost-model plan vs greedy at --n qubits; "
                         "brickwork: 28-qubit brickwork, complex64 and complex128, plain vs fused; "
                         "plain12: 12-qubit random circuit, complex128, gate-by-gate vs the FP64 oracle; "
                         "families: the paper's circuit families (HEA, QAOA, QFT) at 20/25/30 qubits")
    ap.add_argument("--states", type=int, default=256)
    ap.add_argument("--circuit", default="random", choices=["random", "ucc"],
                    help="learned mode: the evaluated circuit (random U3 + CNOT depth 30, or the UCC workload "
                         "with --n-exp exponentials)")
    ap.add_argument("--train-n", type=int, default=28,
                    help="learned mode: the cost model is trained on passes at this and one fewer qubit")
    return ap.parse_args()


def copy_mode(a):
    """Streaming ceiling: copy S = 8 * 2^n bytes with the library's copy kernel."""
    import torch

    from paper_2509_04955_amd import qsim as Q

    S = 8 << a.n
    src = torch.ones(S // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    for _ in range(a.warmup):
        Q.qs_copy(dst.data_ptr(), src.data_ptr(), S, stream.cuda_stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(a.steps):
        Q.qs_copy(dst.data_ptr(), src.data_ptr(), S, stream.cuda_stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / a.steps
    print(json.dumps({"mode": "copy", "bytes_copied": S, "ms": round(ms, 4),
                      "gbs": round(2 * S / (ms * 1e-3) / 1e9, 1)}), flush=True)


def _timed(fn, reps=1):
    import torch

    stream = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def batch_mode(a):
    """256 hardware-efficient-ansatz states (12..22 qubits, 8 layers RY/RZ + CZ ring),
    a 200-term Pauli sum each, all in one hipGraph launch (autotuned plans)."""
    import numpy as np

    import qsynth
    from paper_2509_04955_amd import qsim as Q

    circuits, hams = qsynth.hea_batch(a.states, 12, 22, layers=8, n_terms=200, seed=4)
    t0 = time.perf_counter()
    b = Q.Batch(circuits, hams, Q.opts(k_max=0, tile_qubits=0))
    create_s = time.perf_counter() - t0
    E = b.run()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        E = b.run()
    ms = (time.perf_counter() - t0) / a.steps * 1e3
    amps = sum(1 << c.n for c in circuits)
    gbb = sum(plain_bytes(c, 8 << c.n) for c in circuits)
    out = {"mode": "batch", "states": a.states, "ms_per_batch": round(ms, 3),
           "states_per_s": round(a.states / (ms / 1e3), 1), "amplitudes": amps,
           "circuits_gate_by_gate_equivalent_gbs": round(gbb / (ms * 1e-3) / 1e9, 1),
           "note": "the circuits' gate-by-gate bytes / batch time (a speed measure); the states are MALL-resident "
                   "(cache-resident, not an HBM fraction)",
           "gates": sum(len(c) for c in circuits), "terms": sum(len(h) for h in hams),
           "create_s": round(create_s, 2), "energy_mean": float(np.mean(E))}
    # CPU baseline: the FP64 oracle on a sample of states (energy error of the GPU result)
    import oracle

    sample = list(range(0, a.states, max(1, a.states // 8)))[:8]
    t0 = time.perf_counter()
    errs = []
    for i in sample:
        psi = oracle.run(circuits[i])
        e = oracle.expect_pauli_sum(psi, circuits[i].n, hams[i].x, hams[i].z, hams[i].coeff)
        errs.append(abs(e - E[i]))
    cpu_s = time.perf_counter() - t0
    frac = sum(1 << circuits[i].n for i in sample) / amps
    out["cpu_baseline"] = {"value": round(len(sample) / cpu_s, 3), "unit": "states/s", "cores": oracle.get_threads(),
                           "kind": "oracle", "sample": f"{len(sample)} of {a.states} states ({frac:.3f} of the "
                           f"amplitudes), FP64 circuit + energy, {cpu_s:.1f} s"}
    out["max_energy_error_vs_fp64"] = float(max(errs))
    b.close()
    print(json.dumps(out), flush=True)


def learned_mode(a):
    """Cost model trained on the library's own pass timings (smaller states),
    then the learned plan vs the fixed-width greedy plan on an n-qubit random
    U3 + CNOT circuit (depth 30), complex64."""
    import numpy as np
    import torch

    import qsynth
    from paper_2509_04955_amd import costmodel as CM
    from paper_2509_04955_amd import qsim as Q

    def progress(msg):
        print(f"[learned] {msg}", file=sys.stderr, flush=True)

    n = a.n
    c = qsynth.random_u3_cnot(n, 30, seed=5) if a.circuit == "random" else qsynth.ucc(n, a.n_exp, seed=a.seed)[0]
    gl = Q.GateList(c)
    # the greedy reference gets its best fixed configuration, autotuned on the
    # circuit's first 400 gates; the cost model is trained and the learned
    # partition works inside the same tile shape
    t0 = time.perf_counter()
    best = Q.qs_autotune(n, Q.QS_C64, Q.GateList(c.prefix(400)), Q.opts(strategy=Q.STRATEGY_GREEDY, renorm=1))
    tune_s = time.perf_counter() - t0
    kw = dict(k_max=best.k_max, tile_qubits=best.tile_qubits, low_qubits=best.low_qubits)
    progress(f"autotuned greedy: k_max {best.k_max}, t {best.tile_qubits}, low {best.low_qubits} ({tune_s:.0f} s)")
    train = []
    for nt in sorted({min(n, a.train_n - 1), min(n, a.train_n)}):
        train += [(qsynth.random_u3_cnot(nt, 6, seed=31), False), (qsynth.ucc(nt, 30, seed=32)[0], True),
                  (qsynth.brickwork(nt, 6, seed=33), False), (qsynth.hea(nt, 3, seed=(34, 0)), False)]
    # circuits with Pauli rotations: the rotation strategy's own autotuned
    # configuration, whose tile size the training data then also cover
    bp = None
    tiles = (best.tile_qubits,)
    if a.circuit == "ucc":
        bp = Q.qs_autotune(n, Q.QS_C64, Q.GateList(c.prefix(400)), Q.opts(strategy=Q.STRATEGY_PAULI, renorm=1))
        tiles = tuple(sorted({best.tile_qubits, bp.tile_qubits}))
        progress(f"autotuned rotation strategy: k_max {bp.k_max}, t {bp.tile_qubits}, low {bp.low_qubits}")
    t0 = time.perf_counter()
    parts = []
    for i, (tc, rot) in enumerate(train):
        # circuits with Pauli rotations: also the passes of rotation-contracted plans
        strategies = (Q.STRATEGY_GREEDY, Q.STRATEGY_PAULI) if rot else (Q.STRATEGY_GREEDY,)
        parts.append(CM.collect([tc], widths=(1, 2, 3, 4, 5, 6), tiles=tiles,
                                lows=tuple(sorted({best.low_qubits, 6})), reps=3, max_passes=24,
                                strategies=strategies))
        progress(f"timed passes of training circuit {i + 1}/{len(train)} ({tc.n} qubits)")
    X = np.concatenate([p[0] for p in parts])
    y = np.concatenate([p[1] for p in parts])
    collect_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    loss = CM.train(X, y, epochs=300, batch=64, lr=3e-3, seed=1)
    train_s = time.perf_counter() - t0
    corr = float(np.corrcoef(CM.predict(X), y)[0, 1])
    progress(f"trained on {len(y)} passes: loss {loss:.4f}, corr {corr:.3f}")
    # two rounds on the model's own choices, on held-out circuits of the
    # benchmark family (seed 6, not the evaluated seed 5) at train_n + 2 qubits
    t0 = time.perf_counter()
    n_ref = min(n, a.train_n + 2)
    ref_circuits = ([qsynth.random_u3_cnot(n_ref, 30, seed=6)] if a.circuit == "random"
                    else [qsynth.ucc(n_ref, 100, seed=6)[0]])
    X, y, loss = CM.refine(X, y, ref_circuits, rounds=2, **kw)
    refine_s = time.perf_counter() - t0
    corr = float(np.corrcoef(CM.predict(X), y)[0, 1])
    progress(f"refined on the learned plans' own passes: {len(y)} rows, loss {loss:.4f}, corr {corr:.3f}")
    t0 = time.perf_counter()
    greedy = Q.qs_contract(n, gl, Q.opts(**kw))
    tg_plan = time.perf_counter() - t0
    t0 = time.perf_counter()
    learned = Q.qs_contract(n, gl, Q.opts(strategy=Q.STRATEGY_LEARNED, **kw))
    tl_plan = time.perf_counter() - t0
    # the library's default fixed-width greedy plan in the same tile shape
    kw5 = dict(kw, k_max=5)
    greedy5 = Q.qs_contract(n, gl, Q.opts(**kw5))
    learned5 = Q.qs_contract(n, gl, Q.opts(strategy=Q.STRATEGY_LEARNED, **kw5))
    ig, il = Q.qs_plan_info_get(greedy), Q.qs_plan_info_get(learned)
    progress(f"plans: greedy {ig.n_passes} passes, learned {il.n_passes} passes")
    st = Q.State(n, Q.QS_C64)
    ms_g5 = _timed(lambda: (st.set_basis(0), st.apply_plan(greedy5)))
    ms_l5 = _timed(lambda: (st.set_basis(0), st.apply_plan(learned5)))
    progress(f"k_max 5: greedy {ms_g5:.1f} ms, learned {ms_l5:.1f} ms")
    # five timings of each plan, interleaved; medians and spread
    runs_g, runs_l = [], []
    for _ in range(5):
        runs_g.append(_timed(lambda: (st.set_basis(0), st.apply_plan(greedy))))
        runs_l.append(_timed(lambda: (st.set_basis(0), st.apply_plan(learned))))
    ms_g, ms_l = float(np.median(runs_g)), float(np.median(runs_l))
    progress(f"greedy {ms_g:.1f} ms [{min(runs_g):.1f}, {max(runs_g):.1f}], "
             f"learned {ms_l:.1f} ms [{min(runs_l):.1f}, {max(runs_l):.1f}]")
    # beside it, the rotation strategy in its own autotuned configuration
    # (circuits with Pauli rotations only): what the learned plan is up against
    # when the rotation rule is applied to the whole circuit
    pauli = None
    if bp is not None:
        kwp = dict(k_max=bp.k_max, tile_qubits=bp.tile_qubits, low_qubits=bp.low_qubits)
        pp = Q.qs_contract(n, gl, Q.opts(strategy=Q.STRATEGY_PAULI, **kwp))
        lp = Q.qs_contract(n, gl, Q.opts(strategy=Q.STRATEGY_LEARNED, **kwp))
        runs_p, runs_lp = [], []
        for _ in range(5):
            runs_p.append(_timed(lambda: (st.set_basis(0), st.apply_plan(pp))))
            runs_lp.append(_timed(lambda: (st.set_basis(0), st.apply_plan(lp))))
        ms_p, ms_lp = float(np.median(runs_p)), float(np.median(runs_lp))
        pauli = {"config": kwp, "passes": int(Q.qs_plan_info_get(pp).n_passes), "ms": round(ms_p, 2),
                 "ms_range": [round(min(runs_p), 2), round(max(runs_p), 2)],
                 "learned_in_this_config": {"passes": int(Q.qs_plan_info_get(lp).n_passes), "ms": round(ms_lp, 2),
                                            "ms_range": [round(min(runs_lp), 2), round(max(runs_lp), 2)]},
                 "learned_gain_vs_it": round(ms_p / ms_lp, 3),
                 "note": "the rotation strategy and the learned partition, both in the rotation strategy's "
                         "autotuned configuration, medians of 5"}
        Q.qs_plan_destroy(pp)
        Q.qs_plan_destroy(lp)
        progress(f"rotation strategy (autotuned) {ms_p:.1f} ms, {pauli['passes']} passes; learned in that "
                 f"configuration {ms_lp:.1f} ms, {pauli['learned_in_this_config']['passes']} passes")
    # same state from both schedules: fidelity over all amplitudes, streamed
    # to the host in chunks of 2^26 (two device states, bounded host memory)
    st.set_basis(0)
    st.apply_plan(greedy)
    st2 = Q.State(n, Q.QS_C64)
    st2.set_basis(0)
    st2.apply_plan(learned)
    torch.cuda.synchronize()
    chunk = 1 << min(n, 26)
    dot, ng2, nl2 = 0j, 0.0, 0.0
    for off in range(0, 1 << n, chunk):
        ag = Q.qs_state_copy_out(st.handle, off, chunk)
        al = Q.qs_state_copy_out(st2.handle, off, chunk)
        dot += np.vdot(ag, al)
        ng2 += float(np.vdot(ag, ag).real)
        nl2 += float(np.vdot(al, al).real)
    fid = float(abs(dot) ** 2 / (ng2 * nl2))
    st2.close()
    del st2
    progress(f"fidelity learned vs greedy {fid:.9f}")
    # C followed by its inverse under the learned plan returns |0...0>; norm after renormalisation
    both = qsynth.Circuit(n, list(c.gates) + list(qsynth.inverse(c).gates))
    lb = Q.qs_contract(n, Q.GateList(both), Q.opts(strategy=Q.STRATEGY_LEARNED, **kw))
    st.set_basis(0)
    st.apply_plan(lb)
    a0 = complex(Q.qs_state_copy_out(st.handle, 0, 1)[0])
    norm_cc = st.norm()
    Q.qs_plan_destroy(lb)
    progress(f"C C^dagger |0>: |a0|^2 = {abs(a0) ** 2:.9f}, norm {norm_cc:.12f}")
    out = {"mode": "learned", "circuit": a.circuit, "n": n, "gates": len(c), "greedy_config": kw,
           "autotune_s": round(tune_s, 1),
           "train_rows": int(len(y)), "train_loss": loss, "refine_s": round(refine_s, 1),
           "train_corr": corr, "collect_s": round(collect_s, 1), "train_s": round(train_s, 2),
           "greedy": {"passes": int(ig.n_passes), "blocks": int(ig.n_blocks), "ms": round(ms_g, 2),
                      "ms_range": [round(min(runs_g), 2), round(max(runs_g), 2)], "plan_s": round(tg_plan, 2)},
           "learned": {"passes": int(il.n_passes), "blocks": int(il.n_blocks), "ms": round(ms_l, 2),
                       "ms_range": [round(min(runs_l), 2), round(max(runs_l), 2)], "plan_s": round(tl_plan, 2)},
           "gain": round(ms_g / ms_l, 3), "gain_note": "median of 5 timings each, vs the autotuned greedy plan",
           "rotation_strategy_autotuned": pauli, "fidelity_learned_vs_greedy": fid,
           "c_cdagger_zero_prob": abs(a0) ** 2, "norm_after_c_cdagger": norm_cc,
           "k_max5": {"greedy_ms": round(ms_g5, 2), "learned_ms": round(ms_l5, 2), "gain": round(ms_g5 / ms_l5, 3)}}
    Q.qs_plan_destroy(greedy5)
    Q.qs_plan_destroy(learned5)
    st.close()
    Q.qs_plan_destroy(greedy)
    Q.qs_plan_destroy(learned)
    print(json.dumps(out), flush=True)


def plain12_mode(a):
    """The plain method's configuration: 12-qubit random circuit (20 layers of
    H or RZ per qubit + 6 CNOTs), complex128 from |0...0>, gate by gate.
    GPU median of 5 runs; the FP64 oracle on 1 thread and on all threads."""
    import numpy as np

    import oracle
    import qsynth
    from paper_2509_04955_amd import qsim as Q

    n = 12
    c = qsynth.plain_random(n, 20, 6, seed=1)
    gl = Q.GateList(c)
    st = Q.State(n, Q.QS_C128)
    times = [_timed(lambda: (st.set_basis(0), st.apply_gates(gl))) for _ in range(5)]
    got = st.amplitudes()
    st.close()
    ref = oracle.run(c)
    cpu = {}
    threads = oracle.get_threads()
    for th in (1, threads):
        oracle.set_threads(th)
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            oracle.run(c)
            ts.append(time.perf_counter() - t0)
        cpu[str(th)] = round(float(np.median(ts)) * 1e3, 3)
    oracle.set_threads(threads)
    S = 16 << n
    ms = float(np.median(times))
    print(json.dumps({"mode": "plain12", "n": n, "gates": len(c), "gpu_ms_median5": round(ms, 3),
                      "gates_per_s": round(len(c) / (ms / 1e3), 1),
                      "effective_gbs": round(plain_bytes(c, S) / (ms * 1e-3) / 1e9, 2),
                      "max_abs_vs_fp64": float(np.max(np.abs(got - ref))),
                      "cpu_baseline": {"value": round(cpu[str(threads)], 3), "unit": "ms", "cores": threads,
                                       "kind": "oracle", "sample": "whole circuit, median of 3",
                                       "one_thread_ms": cpu["1"]}}), flush=True)


def families_mode(a):
    """The paper's circuit families at 20, 25 and 30 qubits, complex64: HEA
    (5 layers RX/RY/RZ + staggered CNOT), QAOA MaxCut (3-regular graph, p = 3)
    and QFT.  Gate-count compression of the contraction at k_max = 2 and at
    the autotuned width; time gate by gate (one sweep per gate), with every
    gate a block of its own streamed in the same tile passes (several gates
    per sweep, no contraction: the role of the paper's multi-gate ablation),
    fused, fused with Pauli-rotation contraction (strategy 3), and fused with
    commutation-aware contraction (the commute option, autotuned); and the
    literal staggered multi-gate form (DAG layers of gates over cyclically
    assigned state segments, qs_apply_gates_smgp), the paper's own ablation
    against gate by gate."""
    import qsynth
    from paper_2509_04955_amd import qsim as Q

    rows = []
    for n in (20, 25, 30):
        for name, c in (("hea", qsynth.hea_rxyz(n)), ("qaoa", qsynth.qaoa_maxcut(n)), ("qft", qsynth.qft(n))):
            gl = Q.GateList(c)
            p2 = Q.qs_contract(n, gl, Q.opts(k_max=2))
            b2 = int(Q.qs_plan_info_get(p2).n_blocks)
            Q.qs_plan_destroy(p2)
            best = Q.qs_autotune(n, Q.QS_C64, gl, Q.opts(strategy=Q.STRATEGY_GREEDY, renorm=1))
            plan = Q.qs_contract(n, gl, Q.opts(k_max=best.k_max, tile_qubits=best.tile_qubits,
                                               low_qubits=best.low_qubits))
            info = Q.qs_plan_info_get(plan)
            multi = Q.qs_contract(n, gl, Q.opts(k_max=best.k_max, tile_qubits=best.tile_qubits,
                                                low_qubits=best.low_qubits, strategy=Q.STRATEGY_NONE))
            minfo = Q.qs_plan_info_get(multi)
            # Pauli-rotation contraction in the same tile shape (QAOA's ZZ terms
            # become diagonal rotations that need no tile qubit)
            rot = Q.qs_contract(n, gl, Q.opts(k_max=best.k_max, tile_qubits=best.tile_qubits,
                                              low_qubits=best.low_qubits, strategy=Q.STRATEGY_PAULI))
            rinfo = Q.qs_plan_info_get(rot)
            # commutation-aware contraction (commute option), autotuned on its own
            best_c = Q.qs_autotune(n, Q.QS_C64, gl, Q.opts(strategy=Q.STRATEGY_GREEDY, renorm=1, commute=1))
            com = Q.qs_contract(n, gl, Q.opts(k_max=best_c.k_max, tile_qubits=best_c.tile_qubits,
                                              low_qubits=best_c.low_qubits, commute=1))
            cinfo = Q.qs_plan_info_get(com)
            st = Q.State(n, Q.QS_C64)
            ms_plain = _timed(lambda: (st.set_basis(0), st.apply_gates(gl)))
            ms_smgp = _timed(lambda: (st.set_basis(0), st.apply_gates_smgp(gl)))
            ms_multi = _timed(lambda: (st.set_basis(0), st.apply_plan(multi)))
            ms_fused = _timed(lambda: (st.set_basis(0), st.apply_plan(plan)))
            ms_rot = _timed(lambda: (st.set_basis(0), st.apply_plan(rot)))
            ms_com = _timed(lambda: (st.set_basis(0), st.apply_plan(com)))
            st.close()
            Q.qs_plan_destroy(plan)
            Q.qs_plan_destroy(multi)
            Q.qs_plan_destroy(rot)
            Q.qs_plan_destroy(com)
            S = 8 << n
            rows.append({"family": name, "n": n, "gates": len(c),
                         "compression_k2": round(1 - b2 / len(c), 4),
                         "k_max": best.k_max, "blocks": int(info.n_blocks),
                         "compression": round(1 - info.n_blocks / len(c), 4), "passes": int(info.n_passes),
                         "plain_ms": round(ms_plain, 2),
                         "smgp_ms": round(ms_smgp, 2), "smgp_speedup": round(ms_plain / ms_smgp, 2),
                         "multi_gate_ms": round(ms_multi, 2),
                         "multi_gate_passes": int(minfo.n_passes),
                         "multi_gate_speedup": round(ms_plain / ms_multi, 2), "fused_ms": round(ms_fused, 2),
                         "speedup": round(ms_plain / ms_fused, 2),
                         "rotation_passes": int(rinfo.n_passes), "rotation_ms": round(ms_rot, 2),
                         "rotation_speedup": round(ms_plain / ms_rot, 2),
                         "commute_k_max": best_c.k_max, "commute_blocks": int(cinfo.n_blocks),
                         "commute_passes": int(cinfo.n_passes), "commute_ms": round(ms_com, 2),
                         "commute_gain_vs_fused": round(ms_fused / ms_com, 3),
                         "fused_gate_by_gate_equivalent_gbs": round(plain_bytes(c, S) / (ms_fused * 1e-3) / 1e9, 1)})
            print(f"[families] {rows[-1]}", file=sys.stderr, flush=True)
    print(json.dumps({"mode": "families", "rows": rows}), flush=True)


def brickwork_mode(a):
    """28-qubit brickwork (Haar U3 on every qubit + alternating CNOT pairs,
    depth 40): complex64 and complex128, gate-by-gate vs fused (k_max 5 or
    below, tile shape autotuned per dtype; --k-max and --tile together fix
    the plan instead, e.g. k_max 5 to put every fused block on MFMA)."""
    import qsynth
    from paper_2509_04955_amd import qsim as Q

    import numpy as np

    n = min(a.n, 28)
    c = qsynth.brickwork(n, 40, seed=2)
    gl = Q.GateList(c)
    out = {"mode": "brickwork", "n": n, "gates": len(c)}
    fused_amps = {}
    for dt, name in ((Q.QS_C64, "c64"), (Q.QS_C128, "c128")):
        if a.k_max and a.tile:
            best = types.SimpleNamespace(k_max=a.k_max, tile_qubits=a.tile, low_qubits=a.low)
        else:
            best = Q.qs_autotune(n, dt, gl, Q.opts(strategy=Q.STRATEGY_GREEDY, renorm=1))
        print(f"[brickwork] {name}: plan k_max {best.k_max}, t {best.tile_qubits}, low {best.low_qubits}",
              file=sys.stderr, flush=True)
        st = Q.State(n, dt)
        plan = Q.qs_contract(n, gl, Q.opts(k_max=best.k_max, tile_qubits=best.tile_qubits,
                                           low_qubits=best.low_qubits, dtype=dt))
        info = Q.qs_plan_info_get(plan)
        ms_plain = _timed(lambda: (st.set_basis(0), st.apply_gates(gl)))
        ms_fused = _timed(lambda: (st.set_basis(0), st.apply_plan(plan)))
        S = (8 if dt == Q.QS_C64 else 16) * (1 << n)
        out[name] = {"plain_ms": round(ms_plain, 2), "fused_ms": round(ms_fused, 2),
                     "speedup": round(ms_plain / ms_fused, 2), "passes": int(info.n_passes),
                     "k_max": best.k_max, "tile_qubits": best.tile_qubits, "low_qubits": best.low_qubits,
                     "plain_effective_gbs": round(plain_bytes(c, S) / (ms_plain * 1e-3) / 1e9, 1),
                     "fused_gate_by_gate_equivalent_gbs": round(plain_bytes(c, S) / (ms_fused * 1e-3) / 1e9, 1),
                     "fused_streamed_gbs": round((info.n_passes * 2 + 1) * S / (ms_fused * 1e-3) / 1e9, 1)}
        st.set_basis(0)
        st.apply_plan(plan)
        fused_amps[name] = st.amplitudes()
        # round trip through the inverse circuit (exact result |0...0>)
        inv = Q.qs_contract(n, Q.GateList(qsynth.inverse(c)), Q.opts(k_max=best.k_max, tile_qubits=best.tile_qubits,
                                                                    low_qubits=best.low_qubits, dtype=dt))
        rt_inf, rt_max = roundtrip_error(Q, st, inv)
        Q.qs_plan_destroy(inv)
        out[name]["accuracy"] = {"check": "circuit then its inverse from |0...0> (exact result |0...0>)",
                                 "one_minus_fidelity": rt_inf, "max_abs": rt_max}
        st.close()
        Q.qs_plan_destroy(plan)
    # complex64 against the complex128 result (held to 1e-12 of the FP64 oracle by the parity tests)
    a64, a128 = fused_amps["c64"], fused_amps["c128"]
    out["c64_vs_c128"] = {"max_abs": float(np.max(np.abs(a64 - a128))),
                          "one_minus_fidelity": float(1 - abs(np.vdot(a128, a64)) ** 2
                                                      / (np.vdot(a64, a64).real * np.vdot(a128, a128).real))}
    del fused_amps, a64, a128
    # CPU baseline: the FP64 oracle on the circuit's first gates at full size, extrapolated
    import oracle

    psi = oracle.zero_state(n)
    t0 = time.perf_counter()
    k = 0
    while k < len(c) and time.perf_counter() - t0 < 15.0:
        g = c.gates[k]
        oracle.apply_gate(psi, n, g.name, g.qubits, g.params, g.matrix)
        k += 1
    cpu_s = time.perf_counter() - t0
    del psi
    out["cpu_baseline"] = {"value": round(cpu_s / k * len(c), 1), "unit": "s (extrapolated circuit time)",
                           "cores": oracle.get_threads(), "kind": "oracle",
                           "sample": f"first {k} of {len(c)} gates at n={n}, FP64 gate-by-gate ({cpu_s:.1f} s), "
                                     "extrapolated linearly"}
    print(json.dumps(out), flush=True)


def roundtrip_error(Q, st, plan_inv):
    """Apply the inverse circuit's plan to the state the timed steps left and
    compare with the exact result |0...0>: (1 - |<0|psi>|^2 / <psi|psi>,
    max_i |psi_i - delta_i0|) after the pending FP64 renormalisation is
    applied to the amplitudes."""
    import torch

    st.apply_plan(plan_inv)
    Q.qs_state_normalize(st.handle)
    torch.cuda.synchronize()
    t = st.tensor
    a0 = complex(t[0].item())
    nrm = st.norm()
    rest = float(t[1:].abs().max().item()) if t.numel() > 1 else 0.0
    return 1.0 - abs(a0) ** 2 / nrm, max(abs(a0 - 1.0), rest)


def pauli_contraction(a, Q, n, circ, gl, st_greedy, S, greedy_ms, stream):
    """Strategy 3: each run of gates equal to one Pauli rotation becomes one
    block; autotuned like the main line, timed over the same steps, and its
    final state compared with the greedy plan's (fidelity over all amplitudes,
    streamed to the host in chunks)."""
    import numpy as np
    import torch

    def progress(msg):
        print(f"[pauli] {msg}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    best = Q.qs_autotune(n, Q.QS_C64, gl, Q.opts(strategy=Q.STRATEGY_PAULI, renorm=1))
    tune_s = time.perf_counter() - t0
    progress(f"autotuned k_max {best.k_max}, t {best.tile_qubits}, low {best.low_qubits} ({tune_s:.0f} s)")
    t0 = time.perf_counter()
    plan = Q.qs_contract(n, gl, Q.opts(k_max=best.k_max, tile_qubits=best.tile_qubits, low_qubits=best.low_qubits,
                                       strategy=Q.STRATEGY_PAULI, renorm=1))
    plan_s = time.perf_counter() - t0
    info = Q.qs_plan_info_get(plan)
    st = Q.State(n, Q.QS_C64)

    def step():
        st.set_basis(0)
        st.apply_plan(plan)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    Q.qs_profile_enable(True)
    Q.qs_profile_collect()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(a.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / a.steps
    prof = Q.qs_profile_collect()
    Q.qs_profile_enable(False)
    progress(f"{ms:.1f} ms per circuit, {info.n_passes} passes")
    tl = prof.launches[Q.PROF_TILE]
    tile_ms = prof.ms[Q.PROF_TILE] / max(1, tl)
    chunk = 1 << min(n, 26)
    dot, n1, n2 = 0j, 0.0, 0.0
    for off in range(0, 1 << n, chunk):
        ag = Q.qs_state_copy_out(st_greedy.handle, off, chunk)
        ap = Q.qs_state_copy_out(st.handle, off, chunk)
        dot += np.vdot(ag, ap)
        n1 += float(np.vdot(ag, ag).real)
        n2 += float(np.vdot(ap, ap).real)
    fid = float(abs(dot) ** 2 / (n1 * n2))
    progress(f"fidelity vs greedy {fid:.12f}")
    import qsynth

    inv = Q.qs_contract(n, Q.GateList(qsynth.inverse(circ)),
                        Q.opts(k_max=best.k_max, tile_qubits=best.tile_qubits, low_qubits=best.low_qubits,
                               strategy=Q.STRATEGY_PAULI, renorm=1))
    rt_inf, rt_max = roundtrip_error(Q, st, inv)
    progress(f"circuit + inverse: 1 - F = {rt_inf:.3e}, max-abs {rt_max:.3e}")
    Q.qs_plan_destroy(inv)
    st.close()
    Q.qs_plan_destroy(plan)
    return {"strategy": Q.STRATEGY_PAULI, "k_max": best.k_max, "tile_qubits": best.tile_qubits,
            "low_qubits": best.low_qubits, "n_blocks": int(info.n_blocks), "n_passes": int(info.n_passes),
            "circuit_time_s": round(ms / 1e3, 4), "speedup_vs_greedy": round(greedy_ms / ms, 3),
            "streamed_gbs": round((info.n_passes * 2 * S + S) / (ms * 1e-3) / 1e9, 1),
            "gate_by_gate_equivalent_gbs": round(plain_bytes(circ, S) / (ms * 1e-3) / 1e9, 1),
            "accuracy": {"check": "circuit then its inverse from |0...0> (exact result |0...0>)",
                         "one_minus_fidelity": rt_inf, "max_abs": rt_max},
            "tile_pass_ms": round(tile_ms, 4), "tile_pass_frac_of_8tbs": round(2 * S / (tile_ms * 1e-3) / 8e12, 4),
            "plan_time_s": round(plan_s, 3), "autotune_s": round(tune_s, 2), "fidelity_vs_greedy": fid,
            "note": "runs of gates equal to one Pauli rotation contracted into one block each (beyond the "
                    "paper's fixed-width rule); value above is the paper's greedy contraction"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              "(the multi-GPU path is not part of this build)", file=sys.stderr)
        sys.exit(2)
    import torch

    # torch owns the device context; initialise it before any library call
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    torch.cuda.init()
    if a.mode != "ucc":
        {"copy": copy_mode, "batch": batch_mode, "learned": learned_mode, "brickwork": brickwork_mode,
         "plain12": plain12_mode, "families": families_mode}[a.mode](a)
        return
    import numpy as np

    import qsynth
    from paper_2509_04955_amd import qsim as Q

    n = a.n
    circ, rots = qsynth.ucc(n, n_exp=a.n_exp, seed=a.seed)
    gl = Q.GateList(circ)
    tune_s = 0.0
    if a.k_max == 0 or a.tile == 0:
        # autotuner: times candidate (k_max, t, low qubits) plans on the circuit's first gates
        t0 = time.perf_counter()
        best = Q.qs_autotune(n, Q.QS_C64, gl, Q.opts(strategy=a.strategy, renorm=1))
        tune_s = time.perf_counter() - t0
        a.k_max, a.tile, a.low = best.k_max, best.tile_qubits, best.low_qubits
    t0 = time.perf_counter()
    plan = Q.qs_contract(n, gl, Q.opts(k_max=a.k_max, tile_qubits=a.tile, low_qubits=a.low, strategy=a.strategy,
                                       renorm=1))
    plan_s = time.perf_counter() - t0
    info = Q.qs_plan_info_get(plan)
    S = 8.0 * (1 << n)

    st = Q.State(n, Q.QS_C64)
    stream = torch.cuda.current_stream()

    def step():
        st.set_basis(0)
        st.apply_plan(plan)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    Q.qs_profile_enable(True)
    Q.qs_profile_collect()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(a.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    prof = Q.qs_profile_collect()
    Q.qs_profile_enable(False)
    ms_step = total_ms / a.steps
    # algorithmic bytes of one step: the reset of the state (S) and 2S per tile pass
    alg_bytes = info.n_passes * 2 * S + S
    value = alg_bytes / (ms_step * 1e-3) / 1e9
    gbg_bytes = plain_bytes(circ, S)
    nrm = st.norm()

    # dominant kernel: tile pass (per-launch averages from HIP events)
    tl = prof.launches[Q.PROF_TILE]
    tile_ms = prof.ms[Q.PROF_TILE] / max(1, tl)
    tile_bytes = prof.bytes[Q.PROF_TILE] / max(1, tl)
    tile_flops = prof.flops[Q.PROF_TILE] / max(1, tl)
    t_hbm = tile_bytes / (HBM_PEAK_GBS * 1e9)
    t_mfma = tile_flops / (MFMA_FP32_PEAK_TFLOPS * 1e12)
    if t_mfma > t_hbm:
        roof = {"bound": "mfma", "achieved": tile_flops / (tile_ms * 1e-3) / 1e12, "peak": MFMA_FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": tile_bytes / (tile_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(n)
    roof["kernel"] = "k_tile_pass<float>"
    roof["avg_launch_ms"] = tile_ms
    roof["hbm_gbs"] = tile_bytes / (tile_ms * 1e-3) / 1e9
    roof["tflops"] = tile_flops / (tile_ms * 1e-3) / 1e12

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64 (fp32 amplitudes, fp32 MFMA/VALU, fp64 fusion and norms)",
        "data": "synthetic (seeded UCC-style Pauli-exponential circuit)",
        "config": {"workload": f"ucc n={n} n_exp={a.n_exp} seed={a.seed} complex64", "n_qubits": n,
                   "n_gates": int(info.n_gates), "n_blocks": int(info.n_blocks), "n_passes": int(info.n_passes),
                   "k_max": a.k_max, "tile_qubits": a.tile, "low_qubits": a.low, "strategy": a.strategy,
                   "flops_per_amp_dense_equiv": round(info.flops_per_amp / max(1, info.n_passes), 1)},
        "circuit_time_s": round(ms_step / 1e3, 4),
        "gates_per_s": round(info.n_gates / (ms_step / 1e3), 1),
        "gate_by_gate_equivalent": {
            "bytes_per_circuit": gbg_bytes,
            "rate_gbs": round(gbg_bytes / (ms_step * 1e-3) / 1e9, 1),
            "note": "bytes the gate-by-gate method must stream for this circuit / fused circuit time: a speed "
                    "measure (the plain method at the same rate would match the fused time), not an HBM rate"},
        "plan_time_s": round(plan_s, 3),
        "autotune_s": round(tune_s, 2),
        "norm_after": nrm,
        "roofline": roof,
    }

    # ---- energy of the final state: a 200-term Pauli sum (outside the step) ----
    ham = qsynth.random_pauli_sum(n, 200, seed=(7, 0))
    Q.qs_profile_enable(True)
    Q.qs_profile_collect()
    t0 = time.perf_counter()
    energy = st.expect(ham)
    energy_s = time.perf_counter() - t0
    pe = Q.qs_profile_collect()
    Q.qs_profile_enable(False)
    ex_ms = pe.ms[Q.PROF_EXPECT]
    out["energy"] = {"terms": len(ham), "value": energy, "call_ms": round(energy_s * 1e3, 2),
                     "kernel_ms": round(ex_ms, 2),
                     "kernel_gbs": round(pe.bytes[Q.PROF_EXPECT] / (ex_ms * 1e-3) / 1e9, 1) if ex_ms > 0 else None,
                     "state_reads": round(pe.bytes[Q.PROF_EXPECT] / S, 2),
                     "bytes": "one read of the state (S) per group of terms whose X parts above the tile bits "
                              "span at most 9 dimensions"}

    # ---- the same circuit with Pauli-rotation contraction (beside the paper's rule) ----
    if a.pauli and a.strategy == Q.STRATEGY_GREEDY:
        out["pauli_contraction"] = pauli_contraction(a, Q, n, circ, gl, st, S, ms_step, stream)

    # ---- accuracy: the inverse circuit after the timed steps returns |0...0> exactly ----
    inv = Q.qs_contract(n, Q.GateList(qsynth.inverse(circ)),
                        Q.opts(k_max=a.k_max, tile_qubits=a.tile, low_qubits=a.low, strategy=a.strategy, renorm=1))
    rt_inf, rt_max = roundtrip_error(Q, st, inv)
    Q.qs_plan_destroy(inv)
    out["accuracy"] = {"check": "circuit then its inverse from |0...0> in the same plan configuration; the exact "
                                "(FP64) result is |0...0>",
                       "one_minus_fidelity": rt_inf, "max_abs": rt_max,
                       "note": "whole-circuit error against the FP64 oracle at 22 qubits: tests/test_gpu_accuracy.py"}
    print(f"[accuracy] circuit + inverse: 1 - F = {rt_inf:.3e}, max-abs {rt_max:.3e}", file=sys.stderr, flush=True)

    # ---- fused vs gate-by-gate on a prefix of the same circuit ----
    if a.plain_prefix > 0:
        # the generator draws exponentials in order, so this is the circuit's prefix
        pre_gates, _ = qsynth.ucc(n, n_exp=a.plain_prefix, seed=a.seed)
        gl2 = Q.GateList(pre_gates)
        plan2 = Q.qs_contract(n, gl2, Q.opts(k_max=a.k_max, tile_qubits=a.tile, low_qubits=a.low,
                                             strategy=a.strategy, renorm=1))
        info2 = Q.qs_plan_info_get(plan2)
        Q.qs_profile_enable(True)
        Q.qs_profile_collect()
        st.set_basis(0)
        st.apply_gates(gl2)  # warm
        torch.cuda.synchronize()
        Q.qs_profile_collect()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        st.apply_gates(gl2)
        e1.record(stream)
        torch.cuda.synchronize()
        plain_ms = e0.elapsed_time(e1)
        pp = Q.qs_profile_collect()
        st.apply_plan(plan2)
        torch.cuda.synchronize()
        e0.record(stream)
        st.apply_plan(plan2)
        e1.record(stream)
        torch.cuda.synchronize()
        fused_ms = e0.elapsed_time(e1)
        Q.qs_profile_enable(False)
        Q.qs_plan_destroy(plan2)
        out["plain_vs_fused"] = {
            "prefix_exponentials": a.plain_prefix, "gates": int(info2.n_gates), "passes": int(info2.n_passes),
            "plain_ms": round(plain_ms, 3), "fused_ms": round(fused_ms, 3),
            "speedup": round(plain_ms / fused_ms, 3),
            "plain_gates_per_s": round(info2.n_gates / (plain_ms / 1e3), 1),
            "plain_effective_gbs": round(pp.bytes[Q.PROF_PLAIN] / (pp.ms[Q.PROF_PLAIN] * 1e-3) / 1e9, 1)
            if pp.ms[Q.PROF_PLAIN] > 0 else None,
            "fused_gate_by_gate_equivalent_gbs": round(plain_bytes(pre_gates, S) / (fused_ms * 1e-3) / 1e9, 1),
            # the byte table above against the library's own count for the prefix
            "plain_bytes_table_vs_library": round(plain_bytes(pre_gates, S) / max(1.0, pp.bytes[Q.PROF_PLAIN]), 6),
            "plain_extrapolated_circuit_s": round(plain_ms / 1e3 * info.n_gates / info2.n_gates, 2),
        }
    st.close()
    Q.qs_plan_destroy(plan)
    del st
    torch.cuda.empty_cache()

    # ---- CPU baseline: the FP64 oracle on a bounded sample ----
    if a.cpu_gates > 0:
        import oracle

        threads = oracle.get_threads()
        gates = circ.gates[: a.cpu_gates]
        psi = oracle.zero_state(n)
        t0 = time.perf_counter()
        for g in gates:
            oracle.apply_gate(psi, n, g.name, g.qubits, g.params, g.matrix)
        cpu_s = time.perf_counter() - t0
        del psi
        per_gate = cpu_s / len(gates)
        cpu_circuit_s = per_gate * info.n_gates
        out["cpu_baseline"] = {
            "value": round(plain_bytes(circ, 2 * S) / cpu_circuit_s / 1e9, 4), "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {len(gates)} gates of the same circuit at n={n}, FP64 gate-by-gate "
                      f"({cpu_s:.1f} s); extrapolated linearly to {info.n_gates} gates = {cpu_circuit_s:.0f} s; "
                      "value = the algorithmic bytes of the method the oracle runs (gate by gate on a complex128 "
                      "state) / extrapolated oracle time",
            "circuit_time_s_extrapolated": round(cpu_circuit_s, 1),
            "gates_per_s": round(1.0 / per_gate, 3),
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
