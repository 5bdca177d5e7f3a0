// Learned gate-contraction partition.
//
// Section 3.4 contracts gates greedily; this library's greedy rule uses one
// fixed width k_max for the whole circuit.  The learned strategy keeps the
// greedy rule but chooses its width per window of the circuit with a cost
// model trained on measured pass times:
//   1. plan the circuit with the fixed-width greedy rule (width k_max) and
//      take each of its passes as a window (the set of gates in that pass);
//   2. re-contract every window's gates, in program order, with each width
//      k = 1 .. kcap and pack the blocks into passes;
//   3. predict every candidate pass's time with the MLP (device inference),
//      and keep, per window, the width with the smallest predicted total.
// Windows are contiguous ranges of a valid block order and the gates inside
// a window keep their per-qubit order, so the resulting plan computes the
// same state (exact arithmetic) as the circuit; only rounding differs.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace qs {

void pass_features(int n, qs_dtype dt, const HPass &ps, const std::vector<HBlock> &blocks, float *f) {
    int nd[4] = {0, 0, 0, 0}, n4 = 0, n5 = 0, nmono = 0, nwide = 0;
    double flops = 0;
    for (int64_t b = ps.block0; b < ps.block0 + ps.nblocks; ++b) {
        const HBlock &blk = blocks[b];
        const int k = (int)blk.qubits.size();
        const int kind = block_kind(blk, ps.t, dt, nullptr);
        if (kind == BK_MONO) {
            ++nmono;
            if (k > 4) ++nwide;
            flops += 6;
        } else if (kind == BK_MFMA) {
            (k == 4 ? n4 : n5)++;
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
}

namespace {

struct Candidate {
    std::vector<HBlock> blocks;   // member indices are global gate indices
    std::vector<HPass> passes;    // block0 relative to `blocks`
    double cost = 0;
};

}  // namespace

qs_status learned_partition(qs_plan_s &p, int t, int c) {
    const qs_contract_opts &o = p.opts;
    const qs_dtype dt = o.dtype == QS_C128 ? QS_C128 : QS_C64;
    int kcap = dt == QS_C128 ? kMaxK128 : kMaxK;
    if (t < p.n) kcap = std::min(kcap, t - 1);
    // 1. reference windows
    std::vector<HBlock> ref;
    greedy_blocks(p.gates, p.n, o.k_max, ref);
    std::vector<HPass> ref_passes;
    pack_passes(p, ref, t, c, ref_passes);
    const size_t nw = ref_passes.size();
    std::vector<std::vector<int64_t>> window(nw);
    for (size_t w = 0; w < nw; ++w) {
        for (int64_t b = ref_passes[w].block0; b < ref_passes[w].block0 + ref_passes[w].nblocks; ++b)
            window[w].insert(window[w].end(), ref[b].members.begin(), ref[b].members.end());
        std::sort(window[w].begin(), window[w].end());
    }
    // 2. candidates per window and width
    int wgate = 1;
    for (const HGate &g : p.gates) wgate = std::max(wgate, g.nq);
    std::vector<std::vector<Candidate>> cand(nw);
    std::vector<float> feats;
    std::vector<std::pair<size_t, size_t>> owner;  // (window, candidate) of each feature row
    for (size_t w = 0; w < nw; ++w) {
        std::vector<HGate> sub;
        sub.reserve(window[w].size());
        for (int64_t gi : window[w]) sub.push_back(p.gates[gi]);
        for (int k = 1; k <= kcap; ++k) {
            if (t < p.n && std::max(k, wgate) > t - 1) continue;
            Candidate cd;
            greedy_blocks(sub, p.n, k, cd.blocks);
            for (HBlock &b : cd.blocks) {
                block_matrix(sub, b);
                for (int64_t &m : b.members) m = window[w][m];
            }
            pack_passes(p, cd.blocks, t, c, cd.passes);
            for (const HPass &ps : cd.passes) {
                feats.resize(feats.size() + kNumFeatures);
                pass_features(p.n, dt, ps, cd.blocks, feats.data() + feats.size() - kNumFeatures);
                owner.push_back({w, cand[w].size()});
            }
            cand[w].push_back(std::move(cd));
        }
    }
    // 3. predicted cost (device inference) and choice
    std::vector<float> pred(owner.size());
    qs_status st = costmodel_predict_device(feats.data(), (int)owner.size(), pred.data());
    if (st != QS_OK) return st;
    for (size_t r = 0; r < owner.size(); ++r) cand[owner[r].first][owner[r].second].cost += std::exp((double)pred[r]);
    p.blocks.clear();
    p.passes.clear();
    for (size_t w = 0; w < nw; ++w) {
        size_t best = 0;
        for (size_t i = 1; i < cand[w].size(); ++i)
            if (cand[w][i].cost < cand[w][best].cost) best = i;
        Candidate &cd = cand[w][best];
        const int64_t off = (int64_t)p.blocks.size();
        for (HPass ps : cd.passes) {
            ps.block0 += off;
            p.passes.push_back(std::move(ps));
        }
        for (HBlock &b : cd.blocks) p.blocks.push_back(std::move(b));
    }
    return QS_OK;
}

}  // namespace qs
