// Learned gate-contraction partition.
//
// Section 3.4 contracts gates greedily; this library's greedy rule uses one
// fixed width k_max for the whole circuit.  The learned strategy keeps the
// greedy rule but chooses its width per window of the circuit with a cost
// model trained on measured pass times:
//   1. plan the circuit with the fixed-width greedy rule (width k_max) and
//      take each of its passes as a window (the set of gates in that pass);
//   2. re-contract the gates of every run of 1..3 consecutive windows, in
//      program order, with each width k = 1 .. kcap and pack the blocks into
//      passes (a run can come out with fewer passes than windows);
//   3. predict every candidate pass's time with the MLP (device inference)
//      and cover the windows with the cheapest sequence of runs (dynamic
//      programme); anything but the greedy width on a single window must
//      beat it by a margin, so greedy stays where the model sees no clear gain.
// Windows are contiguous ranges of a valid block order and the gates inside
// a window keep their per-qubit order, so the resulting plan computes the
// same state (exact arithmetic) as the circuit; only rounding differs.
#include <algorithm>
#include <cmath>
#include <limits>

#include "internal.h"

namespace qs {

void pass_features(int n, qs_dtype dt, const HPass &ps, const std::vector<HBlock> &blocks, float *f) {
    // block kinds as the pass kernel will run them (staged passes also put
    // 3-qubit dense blocks on MFMA)
    const bool staged = pass_staged(blocks, ps, dt);
    int nd[4] = {0, 0, 0, 0}, n3m = 0, n4 = 0, n5 = 0, nmono = 0, nwide = 0, nbd = 0;
    double flops = 0;
    for (int64_t b = ps.block0; b < ps.block0 + ps.nblocks; ++b) {
        const HBlock &blk = blocks[b];
        const int k = (int)blk.qubits.size();
        const int kind = block_kind(blk, ps.t, dt, nullptr, staged);
        if (kind == BK_MONO) {
            ++nmono;
            if (k > 4) ++nwide;
            flops += 6;
        } else if (kind == BK_PAULI) {
            ++nbd;
            flops += 16.0;
        } else if (kind == BK_BDIAG || kind == BK_BDMFMA || kind == BK_PERM) {
            ++nbd;
            flops += 8.0 * (1 << bdiag_log_width(blk));
        } else if (kind == BK_MFMA) {
            (k == 3 ? n3m : k == 4 ? n4 : n5)++;   // n5: 5- and 6-qubit MFMA blocks
            flops += 8.0 * (1 << k);
        } else {
            if (k <= 3) ++nd[k];
            else ++nwide;
            flops += 8.0 * (1 << k);
        }
    }
    f[0] = n / 32.0f;
    f[1] = ps.t / 16.0f;
    f[2] = ps.c / 16.0f;
    f[3] = dt == QS_C128 ? 1.0f : 0.0f;
    f[4] = (float)ps.nblocks / 16.0f;
    f[5] = nd[1] / 8.0f;
    f[6] = nd[2] / 8.0f;
    f[7] = nd[3] / 8.0f;
    f[8] = n4 / 8.0f;
    f[9] = n5 / 8.0f;
    f[10] = nmono / 8.0f;
    f[11] = nwide / 8.0f;
    f[12] = (float)(std::log2(1.0 + flops) / 10.0);
    f[13] = (float)(ps.nblocks > 0 ? std::log2(1.0 + flops / ps.nblocks) / 10.0 : 0.0);
    f[14] = staged ? 1.0f : 0.0f;
    f[15] = n3m / 8.0f;
    f[16] = nbd / 8.0f;
}

namespace {

struct Candidate {
    int k = 0;                    // fusion width of this re-contraction
    int span = 1;                 // consecutive windows it covers
    bool rot = false;             // Pauli-strategy contraction of the run
    bool ref = false;             // the reference plan's own window (no switching margin)
    std::vector<HBlock> blocks;   // member indices are global gate indices
    std::vector<HPass> passes;    // block0 relative to `blocks`
    double cost = 0;
};

// A window leaves the reference contraction only for a predicted gain of at
// least this fraction: the reference plan is the fallback, and the model's
// error on a single window is of that order.  The same margin separates the
// rotation-window cover from the greedy-window cover.
constexpr double kSwitchMargin = 0.03;
// Longest run of consecutive windows re-contracted as one candidate
// (rotation candidates: a rotation's gates often straddle two or three greedy
// windows, so their runs may be longer).
constexpr int kMaxSpan = 3;
constexpr int kMaxSpanRot = 5;

struct Cover {
    std::vector<Candidate> picked;   // in window order
    double cost = 0;                 // predicted time (no margins)
};

// The cheapest predicted cover of the windows (gate sets of the reference
// plan's passes, in pass order) by runs of consecutive windows, each run
// re-contracted greedily at some width or, with rotations, as the Pauli
// strategy does.  ref_rot: the reference plan is the rotation contraction
// (its windows' own form is then the rotation candidate).
qs_status cover_windows(const qs_plan_s &p, int t, int c, const std::vector<std::vector<int64_t>> &window,
                        bool ref_rot, bool rotations, int max_x, int kcap, qs_dtype dt, Cover &out) {
    const qs_contract_opts &o = p.opts;
    const size_t nw = window.size();
    const bool commute = o.commute != 0;
    int wgate = 1;
    for (const HGate &g : p.gates) wgate = std::max(wgate, g.nq);
    const int span_max = rotations ? kMaxSpanRot : kMaxSpan;
    std::vector<std::vector<Candidate>> cand(nw);   // cand[e]: runs ending at window e
    std::vector<float> feats;
    std::vector<std::pair<size_t, size_t>> owner;  // (end window, candidate) of each feature row
    auto add_rows = [&](size_t e, const Candidate &cd) {
        for (const HPass &ps : cd.passes) {
            feats.resize(feats.size() + kNumFeatures);
            pass_features(p.n, dt, ps, cd.blocks, feats.data() + feats.size() - kNumFeatures);
            owner.push_back({e, cand[e].size()});
        }
    };
    for (size_t e = 0; e < nw; ++e) {
        for (int r = 1; r <= span_max && (size_t)r <= e + 1; ++r) {
            std::vector<int64_t> gids;
            for (size_t w = e + 1 - r; w <= e; ++w) gids.insert(gids.end(), window[w].begin(), window[w].end());
            std::sort(gids.begin(), gids.end());
            std::vector<HGate> sub;
            sub.reserve(gids.size());
            for (int64_t gi : gids) sub.push_back(p.gates[gi]);
            bool rot_found = false;
            if (rotations) {
                const std::vector<PauliWindow> win = pauli_windows(sub, o.k_max, max_x);
                if (!win.empty()) {
                    rot_found = true;
                    Candidate cd;
                    cd.k = o.k_max;
                    cd.span = r;
                    cd.rot = true;
                    cd.ref = ref_rot && r == 1;
                    pauli_contract(sub, p.n, o.k_max, win, cd.blocks, commute);
                    for (HBlock &b : cd.blocks) {
                        if (!b.pauli) block_matrix(sub, b);
                        for (int64_t &m : b.members) m = gids[m];
                    }
                    pack_passes(p, cd.blocks, t, c, cd.passes);
                    add_rows(e, cd);
                    for (HBlock &b : cd.blocks) {
                        b.U.clear();
                        b.U.shrink_to_fit();
                    }
                    cand[e].push_back(std::move(cd));
                }
            }
            if (r > kMaxSpan) continue;
            for (int k = 1; k <= kcap; ++k) {
                if (t < p.n && std::max(k, wgate) > t - 1) continue;
                if (r > 1 && k == o.k_max) continue;   // the greedy width over several windows is the windows themselves
                Candidate cd;
                cd.k = k;
                cd.span = r;
                // the reference window: the greedy width, or (rotation
                // reference) the greedy width where the window holds no rotation
                cd.ref = r == 1 && k == o.k_max && (!ref_rot || !rot_found);
                greedy_blocks(sub, p.n, k, cd.blocks, nullptr, commute);
                for (HBlock &b : cd.blocks) {
                    block_matrix(sub, b);   // for the block kinds in the features; dropped below
                    for (int64_t &m : b.members) m = gids[m];
                }
                pack_passes(p, cd.blocks, t, c, cd.passes);
                add_rows(e, cd);
                for (HBlock &b : cd.blocks) {
                    b.U.clear();
                    b.U.shrink_to_fit();
                }
                cand[e].push_back(std::move(cd));
            }
        }
    }
    // predicted cost (device inference), then the cheapest cover of the
    // windows by runs (dynamic programme); a run other than the reference
    // window pays the margin
    std::vector<float> pred(owner.size());
    qs_status st = costmodel_predict_device(feats.data(), (int)owner.size(), pred.data());
    if (st != QS_OK) return st;
    for (size_t r = 0; r < owner.size(); ++r) cand[owner[r].first][owner[r].second].cost += std::exp((double)pred[r]);
    std::vector<double> best(nw + 1, 0.0);
    std::vector<size_t> pick(nw, 0);
    for (size_t e = 0; e < nw; ++e) {
        best[e + 1] = std::numeric_limits<double>::infinity();
        for (size_t i = 0; i < cand[e].size(); ++i) {
            const Candidate &cd = cand[e][i];
            const double v = best[e + 1 - cd.span] + cd.cost * (cd.ref ? 1.0 : 1.0 / (1.0 - kSwitchMargin));
            if (v < best[e + 1]) {
                best[e + 1] = v;
                pick[e] = i;
            }
        }
    }
    out.picked.clear();
    out.cost = 0;
    for (size_t e = nw; e > 0;) {
        Candidate &cd = cand[e - 1][pick[e - 1]];
        out.cost += cd.cost;
        e -= (size_t)cd.span;
        out.picked.push_back(std::move(cd));
    }
    std::reverse(out.picked.begin(), out.picked.end());
    return QS_OK;
}

// gate sets of a plan's passes, in pass order
std::vector<std::vector<int64_t>> pass_windows(const std::vector<HBlock> &blocks, const std::vector<HPass> &passes) {
    std::vector<std::vector<int64_t>> window(passes.size());
    for (size_t w = 0; w < passes.size(); ++w) {
        for (int64_t b = passes[w].block0; b < passes[w].block0 + passes[w].nblocks; ++b)
            window[w].insert(window[w].end(), blocks[b].members.begin(), blocks[b].members.end());
        std::sort(window[w].begin(), window[w].end());
    }
    return window;
}

}  // namespace

qs_status learned_partition(qs_plan_s &p, int t, int c) {
    const qs_contract_opts &o = p.opts;
    const qs_dtype dt = o.dtype == QS_C128 ? QS_C128 : QS_C64;
    const bool commute = o.commute != 0;
    int kcap = dt == QS_C128 ? kMaxK128 : kMaxK;
    if (t < p.n) kcap = std::min(kcap, t - 1);
    // X parts must fit the tile's free slots beside the c low qubits
    const int max_x = std::min(8, std::min(t, p.n) - c);
    const std::vector<PauliWindow> rot_win =
        max_x >= 1 ? pauli_windows(p.gates, o.k_max, max_x) : std::vector<PauliWindow>();
    const bool rotations = !rot_win.empty();
    // 1. windows of the greedy plan (the fallback), covered by the model's
    //    cheapest runs
    std::vector<HBlock> ref;
    greedy_blocks(p.gates, p.n, o.k_max, ref, nullptr, commute);
    std::vector<HPass> ref_passes;
    pack_passes(p, ref, t, c, ref_passes);
    Cover cover;
    qs_status st = cover_windows(p, t, c, pass_windows(ref, ref_passes), false, rotations, max_x, kcap, dt, cover);
    if (st != QS_OK) return st;
    // 2. with rotations, also the windows of the rotation contraction (a
    //    rotation's gates then never straddle two windows); its cover replaces
    //    the greedy one for a predicted gain of at least the margin
    if (rotations) {
        std::vector<HBlock> rref;
        pauli_contract(p.gates, p.n, o.k_max, rot_win, rref, commute);
        for (HBlock &b : rref)
            if (!b.pauli) block_matrix(p.gates, b);
        std::vector<HPass> rref_passes;
        pack_passes(p, rref, t, c, rref_passes);
        Cover rcover;
        st = cover_windows(p, t, c, pass_windows(rref, rref_passes), true, true, max_x, kcap, dt, rcover);
        if (st != QS_OK) return st;
        if (rcover.cost < cover.cost * (1.0 - kSwitchMargin)) cover = std::move(rcover);
    }
    p.blocks.clear();
    p.passes.clear();
    for (Candidate &cd : cover.picked) {
        const int64_t off = (int64_t)p.blocks.size();
        for (HPass ps : cd.passes) {
            ps.block0 += off;
            p.passes.push_back(std::move(ps));
        }
        for (HBlock &b : cd.blocks) {
            if (!b.pauli) block_matrix(p.gates, b);
            p.blocks.push_back(std::move(b));
        }
    }
    return QS_OK;
}

}  // namespace qs
