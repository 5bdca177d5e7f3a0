// Host planner: dependency-aware gate contraction (Section 3.4) and the
// packing of fused blocks into streamed tile passes.
//
// DAG.  Gates that share a qubit (controls included) are ordered by program
// order; gates with no path between them commute (Section 3.4).  The DAG is
// never materialised: `last[q]` (the block holding the most recent gate on
// qubit q) carries exactly the information the merge needs.
//
// Merge.  The paper merges greedily without fixing the rule; this library's
// fixed-width greedy rule (width k_max) is: for gate g with qubit set Q,
// f = max_{q in Q} last[q]; g joins the lowest block j >= max(f, 1) with
// |Q_j u Q| <= k_max, else a new block.  Blocks after f hold no qubit of Q, so
// for j > f the test is |Q_j| + |Q| <= k_max; a segment tree over block widths
// finds that j in O(log blocks).  Block products compose the member gates in
// program order (Kronecker embedding of each gate into the block's qubits, the
// same-qubit product M2 M1 and the controlled merge being special cases).
//
// Passes.  Consecutive blocks are packed into one pass while the union of
// their qubits with the always-present low qubits {0..c-1} stays within t
// qubits; a pass is one read and one write of the state (one tile kernel).
#include <algorithm>
#include <cstring>
#include <limits>
#include <stdexcept>

#include "internal.h"

namespace qs {

int default_tile(qs_dtype dt) { return dt == QS_C128 ? 12 : 13; }

namespace {

// Segment tree over block widths: first index > f whose width <= s.
struct MinTree {
    int size = 1;
    std::vector<int> v;
    explicit MinTree(size_t cap) {
        while ((size_t)size < cap + 1) size <<= 1;
        v.assign(2 * size, std::numeric_limits<int>::max());
    }
    void set(int i, int val) {
        i += size;
        v[i] = val;
        for (i >>= 1; i; i >>= 1) v[i] = std::min(v[2 * i], v[2 * i + 1]);
    }
    // smallest index >= lo with value <= s, or -1
    int first_le(int lo, int s) const { return find(1, 0, size, lo, s); }
    int find(int node, int l, int r, int lo, int s) const {
        if (r <= lo || v[node] > s) return -1;
        if (r - l == 1) return l;
        int m = (l + r) / 2;
        int a = find(2 * node, l, m, lo, s);
        return a >= 0 ? a : find(2 * node + 1, m, r, lo, s);
    }
};

}  // namespace

uint64_t diagonal_qubits(const HGate &g) {
    if (g.m.empty()) return 0;
    const int d = 1 << g.nq;
    uint64_t out = 0;
    for (int j = 0; j < g.nq; ++j) {
        bool diag = true;
        for (int r = 0; r < d && diag; ++r)
            for (int c = 0; c < d; ++c)
                if (((r ^ c) >> j) & 1 && g.m[(size_t)r * d + c] != cd(0, 0)) {
                    diag = false;
                    break;
                }
        if (diag) out |= 1ull << g.q[j];
    }
    return out;
}

void greedy_blocks(const std::vector<HGate> &gates, int n, int kmax, std::vector<HBlock> &blocks,
                   const std::vector<char> *solo, bool commute) {
    blocks.clear();
    std::vector<int> last(n, 0);                 // 1-based block index, 0 = none
    std::vector<int> last_nd(n, 0);              // latest block acting non-diagonally on the qubit
    std::vector<uint64_t> qmask;                 // qubit mask per block
    std::vector<int> width;
    std::vector<char> closed;                    // blocks that take no further gates (solo units)
    MinTree tree(gates.size() + 1);
    for (size_t gi = 0; gi < gates.size(); ++gi) {
        const HGate &g = gates[gi];
        const uint64_t dq = commute ? diagonal_qubits(g) : 0;
        uint64_t gm = 0;
        int f = 0, L = 0;   // f: latest block g must follow; L: latest block touching g's qubits
        for (int j = 0; j < g.nq; ++j) {
            const int q = g.q[j];
            gm |= 1ull << q;
            f = std::max(f, ((dq >> q) & 1) ? last_nd[q] : last[q]);
            L = std::max(L, last[q]);
        }
        const int w = g.nq;
        const bool alone = solo && (*solo)[gi];
        int j = -1;  // 1-based
        if (w <= kmax && !alone) {
            // lowest block >= max(f, 1) whose qubits with g's stay within kmax:
            // blocks up to L may share qubits with g (only when it commutes
            // past them), blocks after L share none (width test in the tree)
            for (int b = std::max(f, 1); b <= L && j < 0; ++b)
                if (!closed[b - 1] && __builtin_popcountll(qmask[b - 1] | gm) <= kmax) j = b;
            if (j < 0) {
                int idx = tree.first_le(std::max(L + 1, 1), kmax - w);  // tree index = 1-based block id
                if (idx >= 1 && idx <= (int)blocks.size()) j = idx;
            }
        }
        if (j < 0) {
            blocks.emplace_back();
            qmask.push_back(0);
            width.push_back(0);
            closed.push_back(alone ? 1 : 0);
            j = (int)blocks.size();
        }
        blocks[j - 1].members.push_back((int64_t)gi);
        qmask[j - 1] |= gm;
        width[j - 1] = __builtin_popcountll(qmask[j - 1]);
        tree.set(j, closed[j - 1] ? 64 : width[j - 1]);
        for (int q = 0; q < g.nq; ++q) {
            const int qq = g.q[q];
            last[qq] = std::max(last[qq], j);
            if (!((dq >> qq) & 1)) last_nd[qq] = std::max(last_nd[qq], j);
        }
    }
    for (size_t b = 0; b < blocks.size(); ++b) {
        blocks[b].qubits.clear();
        for (int q = 0; q < 64; ++q)
            if ((qmask[b] >> q) & 1) blocks[b].qubits.push_back(q);
    }
}

// U_B = G_m ... G_1 with each gate embedded into the block's qubits.
void block_matrix(const std::vector<HGate> &gates, HBlock &b) {
    const int k = (int)b.qubits.size();
    const int d = 1 << k;
    b.U.assign((size_t)d * d, cd(0, 0));
    for (int i = 0; i < d; ++i) b.U[(size_t)i * d + i] = 1;
    std::vector<cd> tmp;
    for (int64_t gi : b.members) {
        const HGate &g = gates[gi];
        int lp[8];
        for (int j = 0; j < g.nq; ++j)
            lp[j] = (int)(std::find(b.qubits.begin(), b.qubits.end(), g.q[j]) - b.qubits.begin());
        const int gd = 1 << g.nq;
        int gmask = 0;
        for (int j = 0; j < g.nq; ++j) gmask |= 1 << lp[j];
        std::vector<int> off(gd);
        for (int a = 0; a < gd; ++a) {
            int o = 0;
            for (int j = 0; j < g.nq; ++j)
                if ((a >> j) & 1) o |= 1 << lp[j];
            off[a] = o;
        }
        tmp.assign(gd, cd(0, 0));
        // left-multiply: every column of U is a vector the gate acts on
        for (int col = 0; col < d; ++col) {
            for (int base = 0; base < d; ++base) {
                if (base & gmask) continue;
                for (int a = 0; a < gd; ++a) {
                    cd acc = 0;
                    for (int c2 = 0; c2 < gd; ++c2)
                        acc += g.m[(size_t)a * gd + c2] * b.U[(size_t)(base | off[c2]) * d + col];
                    tmp[a] = acc;
                }
                for (int a = 0; a < gd; ++a) b.U[(size_t)(base | off[a]) * d + col] = tmp[a];
            }
        }
    }
}

// Passes: list scheduling of the blocks over their dependence order (Section
// 3.4: blocks sharing a qubit keep their order; two Pauli-rotation blocks with
// commuting strings may swap).  A pass starts from the first
// pending block and its tile {0..c-1}; pending blocks are scanned in order and
// a block joins the pass if its qubits fit the tile (at most t qubits).  A block
// that does not fit is left for a later pass and its qubits are marked: no
// later block touching them may run ahead of it, but blocks on other qubits may
// still join.  The scan stops kLookahead blocks after the first one left out.
// The blocks are reordered into execution order (pass by pass), so a pass is a
// contiguous range; any order produced this way keeps every pair of blocks that
// share a qubit in program order, hence the same state in exact arithmetic.
constexpr size_t kLookahead = 64;

namespace {
// entries of a block product below this are rounding residue of exact zeros
// (the same threshold as the monomial test of the tile kernels)
constexpr double kDiagTol = 1e-14;

// qubits on which a (non-rotation) block acts diagonally, from its matrix
uint64_t block_diagonal(const HBlock &b) {
    const int k = (int)b.qubits.size(), d = 1 << k;
    if (b.U.size() != (size_t)d * d) return 0;
    uint64_t out = 0;
    for (int j = 0; j < k; ++j) {
        bool diag = true;
        for (int r = 0; r < d && diag; ++r)
            for (int c = 0; c < d; ++c)
                if (((r ^ c) >> j) & 1 && std::abs(b.U[(size_t)r * d + c]) > kDiagTol) {
                    diag = false;
                    break;
                }
        if (diag) out |= 1ull << b.qubits[j];
    }
    return out;
}
}  // namespace

void pack_passes(const qs_plan_s &p, std::vector<HBlock> &blocks, int t, int c, std::vector<HPass> &out) {
    out.clear();
    const int n = p.n;
    t = std::min(t, n);
    c = std::min(c, t);
    const uint64_t low = c >= 64 ? ~0ull : ((1ull << c) - 1);
    // dm: qubits a block depends on (its support); bm: qubits it needs in the
    // tile (the support, or the X part of a Pauli rotation: its Z part outside
    // the tile is a per-tile sign)
    std::vector<uint64_t> bm(blocks.size(), 0), dm(blocks.size(), 0);
    for (size_t b = 0; b < blocks.size(); ++b) {
        for (int q : blocks[b].qubits) dm[b] |= 1ull << q;
        bm[b] = blocks[b].pauli ? blocks[b].px : dm[b];
    }
    // Two Pauli-rotation blocks whose strings commute commute as operators
    // (each is c I + d P), so one may overtake the other although they share
    // qubits.  With the commute option, so may two blocks that are both
    // diagonal on every qubit they share (dg: qubits a block acts on
    // diagonally, from its matrix with entries below kDiagTol taken as the
    // rounding residue of exact zeros; a rotation is diagonal off its X
    // part).  Every other pair sharing a qubit keeps its order.
    const bool by_diag = p.opts.commute != 0;
    std::vector<uint64_t> dg(blocks.size(), 0);
    if (by_diag)
        for (size_t b = 0; b < blocks.size(); ++b) dg[b] = blocks[b].pauli ? dm[b] & ~blocks[b].px : block_diagonal(blocks[b]);
    auto commute = [&](size_t a, size_t b) {
        const HBlock &A = blocks[a], &B = blocks[b];
        if (A.pauli && B.pauli &&
            ((__builtin_popcountll(A.px & B.pz) + __builtin_popcountll(A.pz & B.px)) & 1) == 0)
            return true;
        const uint64_t shared = dm[a] & dm[b];
        return by_diag && (shared & ~(dg[a] & dg[b])) == 0;
    };
    std::vector<size_t> pending(blocks.size()), rest;
    for (size_t b = 0; b < blocks.size(); ++b) pending[b] = b;
    std::vector<HBlock> ordered;
    ordered.reserve(blocks.size());
    while (!pending.empty()) {
        HPass ps;
        ps.block0 = (int64_t)ordered.size();
        uint64_t cur = low, blocked = 0;
        size_t scanned_after_skip = 0, i = 0;
        bool skipped = false;
        rest.clear();
        for (; i < pending.size(); ++i) {
            if (skipped && scanned_after_skip++ >= kLookahead) break;
            const size_t b = pending[i];
            bool free = (dm[b] & blocked) == 0;
            if (!free && (blocks[b].pauli || by_diag)) {
                // overtaking is allowed past skipped blocks it commutes with
                free = true;
                for (size_t r : rest)
                    if ((dm[r] & dm[b]) && !commute(r, b)) {
                        free = false;
                        break;
                    }
            }
            if (free && __builtin_popcountll(cur | bm[b]) <= t) {
                cur |= bm[b];
                ordered.push_back(std::move(blocks[b]));
            } else {
                blocked |= dm[b];
                rest.push_back(b);
                skipped = true;
            }
        }
        rest.insert(rest.end(), pending.begin() + (int64_t)i, pending.end());
        ps.nblocks = (int64_t)ordered.size() - ps.block0;
        // the first pending block always fits (c is sized for the widest block)
        if (ps.nblocks == 0) throw std::logic_error("pass packing made no progress");
        // fill the tile up to t qubits with the lowest unused qubits
        uint64_t m = cur;
        for (int q = 0; q < n && __builtin_popcountll(m) < t; ++q) m |= 1ull << q;
        ps.t = t;
        for (int q = 0; q < n; ++q)
            if ((m >> q) & 1) ps.tile.push_back(q);
        int cc = 0;
        while (cc < (int)ps.tile.size() && ps.tile[cc] == cc) ++cc;
        ps.c = cc;
        // the planner sizes c so that every pass holds exactly t qubits and qubit 0
        if ((int)ps.tile.size() != t || cc < 1) throw std::logic_error("pass tile invariant broken");
        out.push_back(std::move(ps));
        pending.swap(rest);
    }
    blocks.swap(ordered);
}

std::vector<PauliWindow> pauli_windows(const std::vector<HGate> &gates, int k_max, int max_x_weight) {
    std::vector<PauliWindow> win = find_pauli_windows(gates, max_x_weight);
    // a diagonal rotation (no X part) no wider than k_max is left to the
    // greedy rule, which merges several of them (and their neighbours) into
    // one diagonal block: one block per rotation would cost a tile round trip
    // each (QAOA's ZZ terms)
    win.erase(std::remove_if(win.begin(), win.end(),
                             [&](const PauliWindow &w) { return w.x == 0 && (int)w.support.size() <= k_max; }),
              win.end());
    return win;
}

void pauli_contract(const std::vector<HGate> &gates, int n, int k_max, const std::vector<PauliWindow> &win,
                    std::vector<HBlock> &blocks, bool commute) {
    // units: each window, and every gate outside the windows, in program
    // order; a window is a block of its own, the gates merge greedily
    std::vector<HGate> units;
    std::vector<char> solo;
    std::vector<int64_t> first;   // window: its index; gate: its program index
    size_t wi = 0;
    for (int64_t gi = 0; gi < (int64_t)gates.size();) {
        if (wi < win.size() && win[wi].begin == gi) {
            HGate u;
            u.nq = (int)win[wi].support.size();
            for (int j = 0; j < u.nq; ++j) u.q[j] = win[wi].support[j];
            units.push_back(std::move(u));
            solo.push_back(1);
            first.push_back((int64_t)wi);
            gi = win[wi].end;
            ++wi;
        } else {
            units.push_back(gates[gi]);
            solo.push_back(0);
            first.push_back(gi);
            ++gi;
        }
    }
    greedy_blocks(units, n, k_max, blocks, &solo, commute);
    for (HBlock &b : blocks) {
        if (b.members.size() == 1 && solo[b.members[0]]) {
            const PauliWindow &w = win[first[b.members[0]]];
            b.pauli = true;
            b.px = w.x;
            b.pz = w.z;
            b.pc = w.c;
            b.pd = w.d;
            b.members.clear();
            for (int64_t gi = w.begin; gi < w.end; ++gi) b.members.push_back(gi);
        } else {
            for (int64_t &m : b.members) m = first[m];
        }
    }
}

qs_status build_plan(qs_plan_s &p) {
    qs_contract_opts &o = p.opts;
    const qs_dtype dt = o.dtype == QS_C128 ? QS_C128 : QS_C64;
    const int kcap = dt == QS_C128 ? kMaxK128 : kMaxK;
    if (o.k_max == 0) o.k_max = 5;
    QS_CHECK(o.k_max >= 1 && o.k_max <= kcap, QS_EINVAL, "k_max %d outside 1..%d", o.k_max, kcap);
    if (o.tile_qubits == 0) o.tile_qubits = default_tile(dt);
    const int tcap = dt == QS_C128 ? kMaxTile128 : kMaxTile;
    QS_CHECK(o.tile_qubits >= 2 && o.tile_qubits <= tcap, QS_EINVAL, "tile_qubits %d outside 2..%d",
             o.tile_qubits, tcap);
    if (o.low_qubits == 0) o.low_qubits = std::min(6, o.tile_qubits);
    QS_CHECK(o.low_qubits >= 1 && o.low_qubits <= o.tile_qubits, QS_EINVAL, "low_qubits %d invalid",
             o.low_qubits);
    const int t = std::min(o.tile_qubits, p.n);
    // Every block (a gate wider than k_max is a block of its own) must fit in a
    // tile next to at least one low qubit, so that qubit 0 is always in the
    // tile and tiles start with a contiguous run.
    QS_CHECK(o.strategy >= QS_STRATEGY_NONE && o.strategy <= QS_STRATEGY_PAULI, QS_EINVAL, "strategy %d unknown",
             o.strategy);
    QS_CHECK(o.commute == 0 || o.commute == 1, QS_EINVAL, "commute must be 0 or 1 (got %d)", o.commute);
    int wmax = o.k_max;
    for (const HGate &g : p.gates) wmax = std::max(wmax, g.nq);
    std::vector<PauliWindow> win;
    if (o.strategy == QS_STRATEGY_PAULI) {
        // X parts up to 8 qubits and below the tile (qubit 0 keeps a slot)
        win = pauli_windows(p.gates, o.k_max, std::min(8, std::min(o.tile_qubits, p.n) - 1));
        for (const PauliWindow &w : win) wmax = std::max(wmax, __builtin_popcountll(w.x));
    }
    if (t < p.n)
        QS_CHECK(std::min(wmax, p.n) <= t - 1, QS_EINVAL,
                 "blocks of width %d need a tile of at least %d qubits (got %d)", wmax, wmax + 1, t);
    const int c = std::max(1, std::min(o.low_qubits, t - std::min(wmax, t)));

    if (o.strategy == QS_STRATEGY_NONE) {
        p.blocks.clear();
        for (size_t gi = 0; gi < p.gates.size(); ++gi) {
            HBlock b;
            b.members.push_back((int64_t)gi);
            for (int j = 0; j < p.gates[gi].nq; ++j) b.qubits.push_back(p.gates[gi].q[j]);
            std::sort(b.qubits.begin(), b.qubits.end());
            p.blocks.push_back(std::move(b));
        }
    } else if (o.strategy == QS_STRATEGY_LEARNED && costmodel_loaded()) {
        return learned_partition(p, t, c);
    } else if (o.strategy == QS_STRATEGY_PAULI) {
        pauli_contract(p.gates, p.n, o.k_max, win, p.blocks, o.commute != 0);
    } else {
        greedy_blocks(p.gates, p.n, o.k_max, p.blocks, nullptr, o.commute != 0);
    }
    for (HBlock &b : p.blocks)
        if (!b.pauli) block_matrix(p.gates, b);
    pack_passes(p, p.blocks, t, c, p.passes);
    return QS_OK;
}

}  // namespace qs
