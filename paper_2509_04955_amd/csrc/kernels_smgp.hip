// Staggered multi-gate parallelism (Section 3.3; the 2-D thread mapping and
// Table "segment"): the gates of one DAG layer run in the same launches.
//
// A layer is a set of gates on pairwise disjoint qubits (they commute).  For
// m such gates the state is split into M = 2^s segments by s qubits that no
// gate of the layer touches; at time step j, gate i updates segment
// (i + j) mod M, so within a step no two gates touch the same segment and
// after M steps every gate has updated every segment (a cyclic Latin
// square, the table's schedule).  One launch per step: a 2-D grid whose
// y index is the gate and whose x range covers the amplitude pairs of that
// gate's segment, one thread per pair (the paper's one-pair-per-thread
// mapping, extended by the gate dimension).  The launches of a layer run in
// stream order, which is the barrier between steps.
//
// Every gate still reads and writes every amplitude it touches once (2S per
// layer and gate, as gate by gate): this is the form the paper measured
// against its one-dimensional baseline, kept here as the ablation beside the
// tile passes, which stream 2S for many gates at once.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace qs {

namespace {

constexpr int kSmgpThreads = 256;
constexpr int kSmgpMaxLog = 5;     // at most 32 segments (and gates) per layer launch
constexpr uint32_t kSmgpMaxGridX = 1u << 16;

// The layer's table travels as a kernel argument (by value; at most 32 gates
// keeps it well inside the argument limit), so a layer needs no device
// allocation or copy.
template <typename R>
struct SmgpGate {
    R ur[4], ui[4];           // 2x2 on the target (control = 1 for controlled gates), row-major
    int8_t t, c;              // target, control (-1: none)
    int8_t npos;              // fixed bit positions (segment bits, target, control), ascending
    int8_t pos[kSmgpMaxLog + 2];
};

template <typename R>
struct SmgpLayer {
    SmgpGate<R> g[1 << kSmgpMaxLog];
    int8_t seg_pos[kSmgpMaxLog];    // the segment qubits: bit b of the segment number -> seg_pos[b]
    int8_t s;                       // log2 of the segment count
};
static_assert(sizeof(SmgpLayer<double>) <= 3072, "layer table must fit the kernel argument space");

__device__ __forceinline__ uint64_t ins0(uint64_t x, int p) {
    const uint64_t lo = x & ((1ull << p) - 1);
    return ((x - lo) << 1) | lo;
}

// step j of a layer: gate i = blockIdx.y on segment (i + j) mod M
template <typename R, typename A>
__global__ __launch_bounds__(kSmgpThreads) void k_smgp_step(A *__restrict__ psi, const SmgpLayer<R> L, uint32_t step,
                                                            uint64_t pairs_uc, uint64_t pairs_c) {
    const SmgpGate<R> &g = L.g[blockIdx.y];
    const int s = L.s;
    const uint32_t M = 1u << s;
    const uint32_t seg = (blockIdx.y + step) & (M - 1);
    uint64_t fixed = g.c >= 0 ? 1ull << g.c : 0;   // the control bit is 1
    for (int b = 0; b < s; ++b)
        if ((seg >> b) & 1) fixed |= 1ull << L.seg_pos[b];
    const uint64_t tbit = 1ull << g.t;
    const uint64_t npairs = g.c >= 0 ? pairs_c : pairs_uc;
    for (uint64_t k = (uint64_t)blockIdx.x * kSmgpThreads + threadIdx.x; k < npairs;
         k += (uint64_t)gridDim.x * kSmgpThreads) {
        uint64_t i0 = k;
        for (int p = 0; p < g.npos; ++p) i0 = ins0(i0, g.pos[p]);
        i0 |= fixed;
        const uint64_t i1 = i0 | tbit;
        const A a = psi[i0], b = psi[i1];
        A x, y;
        x.x = g.ur[0] * a.x - g.ui[0] * a.y + g.ur[1] * b.x - g.ui[1] * b.y;
        x.y = g.ur[0] * a.y + g.ui[0] * a.x + g.ur[1] * b.y + g.ui[1] * b.x;
        y.x = g.ur[2] * a.x - g.ui[2] * a.y + g.ur[3] * b.x - g.ui[3] * b.y;
        y.y = g.ur[2] * a.y + g.ui[2] * a.x + g.ur[3] * b.y + g.ui[3] * b.x;
        psi[i0] = x;
        psi[i1] = y;
    }
}

// one-qubit gates and controlled one-qubit gates (control q[0], target q[1])
bool smgp_supported(const HGate &g) {
    if (g.nq == 1) return true;
    return g.nq == 2 && g.kind >= QS_CNOT && g.kind < QS_SWAP;
}

template <typename R>
void fill_gate(const HGate &g, SmgpGate<R> &d) {
    const bool ctl = g.nq == 2;
    d.t = (int8_t)(ctl ? g.q[1] : g.q[0]);
    d.c = (int8_t)(ctl ? g.q[0] : -1);
    // 2x2 block acting on the target: rows/columns with control = 1 (local
    // index = control bit + 2 target bit) or the gate itself
    const int D = 1 << g.nq;
    const int r0 = ctl ? 1 : 0, r1 = ctl ? 3 : 1;
    const int idx[2] = {r0, r1};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const cd v = g.m[(size_t)idx[a] * D + idx[b]];
            d.ur[2 * a + b] = (R)v.real();
            d.ui[2 * a + b] = (R)v.imag();
        }
}

template <typename R>
qs_status run_layer(qs_state_s &s, const std::vector<const HGate *> &gates, const std::vector<int> &seg_pos) {
    using A = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
    SmgpLayer<R> L{};
    L.s = (int8_t)seg_pos.size();
    for (int b = 0; b < L.s; ++b) L.seg_pos[b] = (int8_t)seg_pos[b];
    const int m = (int)gates.size();
    for (int i = 0; i < m; ++i) {
        SmgpGate<R> &d = L.g[i];
        fill_gate<R>(*gates[i], d);
        std::vector<int> pos(seg_pos);
        pos.push_back(d.t);
        if (d.c >= 0) pos.push_back(d.c);
        std::sort(pos.begin(), pos.end());
        d.npos = (int8_t)pos.size();
        for (size_t p = 0; p < pos.size(); ++p) d.pos[p] = (int8_t)pos[p];
    }
    const int n = s.n;
    const uint64_t pairs_uc = 1ull << (n - L.s - 1);
    const uint64_t pairs_c = n - L.s - 2 >= 0 ? 1ull << (n - L.s - 2) : 0;
    const uint64_t blocks = (pairs_uc + kSmgpThreads - 1) / kSmgpThreads;
    const dim3 grid((unsigned)std::min<uint64_t>(blocks, kSmgpMaxGridX), (unsigned)m);
    const uint32_t M = 1u << L.s;
    const double S = std::ldexp((double)sizeof(A), n);
    // bytes: every gate reads and writes its pairs once (controlled: half)
    double bytes = 0;
    for (const HGate *g : gates) bytes += (g->nq == 2 ? 1.0 : 2.0) * S;
    prof_begin(s.stream, QS_PROF_PLAIN, bytes, 14.0 * std::ldexp(1.0, n) * m);
    for (uint32_t j = 0; j < M; ++j)
        hipLaunchKernelGGL((k_smgp_step<R, A>), grid, dim3(kSmgpThreads), 0, s.stream, (A *)s.amp, L, j, pairs_uc,
                           pairs_c);
    prof_end(s.stream);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

}  // namespace

qs_status launch_smgp(qs_state_s &s, const std::vector<HGate> &gates) {
    const int n = s.n;
    // DAG layers: level(g) = 1 + the largest level among earlier gates sharing
    // a qubit; gates of one level share no qubit, and running the levels in
    // order keeps every dependency
    std::vector<int> last(n, 0);
    std::vector<std::vector<size_t>> levels;
    for (size_t gi = 0; gi < gates.size(); ++gi) {
        int lv = 0;
        for (int j = 0; j < gates[gi].nq; ++j) lv = std::max(lv, last[gates[gi].q[j]]);
        if ((size_t)lv >= levels.size()) levels.resize(lv + 1);
        levels[lv].push_back(gi);
        for (int j = 0; j < gates[gi].nq; ++j) last[gates[gi].q[j]] = lv + 1;
    }
    qs_status st = QS_OK;
    for (const std::vector<size_t> &lev : levels) {
        std::vector<const HGate *> batch;
        for (size_t gi : lev) {
            if (smgp_supported(gates[gi])) batch.push_back(&gates[gi]);
            else if ((st = launch_plain(s, gates[gi])) != QS_OK) break;
        }
        if (st != QS_OK) break;
        // chunks of the batch: m gates need s = ceil(log2 m) segment qubits
        // outside their own qubits (at most kSmgpMaxLog)
        size_t b0 = 0;
        while (b0 < batch.size() && st == QS_OK) {
            size_t m = std::min<size_t>(batch.size() - b0, (size_t)1 << kSmgpMaxLog);
            std::vector<int> seg;
            for (;; m = (m + 1) / 2) {
                uint64_t used = 0;
                for (size_t i = b0; i < b0 + m; ++i)
                    for (int j = 0; j < batch[i]->nq; ++j) used |= 1ull << batch[i]->q[j];
                int lg = 0;
                while ((size_t)1 << lg < m) ++lg;
                seg.clear();
                for (int q = n - 1; q >= 0 && (int)seg.size() < lg; --q)   // the highest free qubits
                    if (!((used >> q) & 1)) seg.push_back(q);
                if ((int)seg.size() == lg) break;
            }
            std::sort(seg.begin(), seg.end());
            if (m == 1) {
                st = launch_plain(s, *batch[b0]);
            } else {
                std::vector<const HGate *> chunk(batch.begin() + (int64_t)b0, batch.begin() + (int64_t)(b0 + m));
                st = s.dtype == QS_C64 ? run_layer<float>(s, chunk, seg) : run_layer<double>(s, chunk, seg);
            }
            b0 += m;
        }
        if (st != QS_OK) break;
    }
    return st;
}

}  // namespace qs
