// Autotuner: picks the fusion width k_max, the tile size t and the number of
// fixed contiguous low qubits per tile for a circuit by running candidate
// plans on the device and keeping the fastest.
//
// Stage 1 crosses k_max in 3..5 with t in 11..14 (complex64; 11..12 for
// complex128; capped by n and by the dtype's LDS limit) at 4 and 6 low qubits; stage 2 tries 3 and 5 low qubits
// for the winning (k_max, t).  Fewer fixed low qubits leave more tile slots to
// the qubits the gates touch (fewer passes) at the price of shorter coalesced
// runs per tile segment.  Each candidate's plan runs on a scratch state once
// to warm up and is then timed with hipEvents; circuits longer than
// kTunePrefix gates are tuned on their first kTunePrefix gates (4 kTunePrefix
// for the Pauli-rotation strategy; the passes of
// a long circuit repeat the same structure).  Results are cached per
// (n, dtype, strategy, gate structure) for the life of the process.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.h"

namespace {

constexpr size_t kTunePrefix = 1536;

uint64_t structure_hash(const qs_gate *g, size_t n) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        h ^= v;
        h *= 1099511628211ull;
    };
    for (size_t i = 0; i < n; ++i) {
        mix((uint64_t)g[i].kind);
        mix((uint64_t)g[i].nq);
        for (int j = 0; j < g[i].nq && j < 8; ++j) mix((uint64_t)g[i].qubits[j]);
    }
    return h;
}

std::mutex g_mu;
std::map<std::tuple<int, int, int, uint64_t>, qs_contract_opts> g_cache;

}  // namespace

extern "C" qs_status qs_autotune(int n, qs_dtype dtype, const qs_gate *gates, size_t n_gates,
                                 const qs_contract_opts *base, qs_contract_opts *best) {
    QS_ABI_TRY
    QS_CHECK(best != nullptr && (gates != nullptr || n_gates == 0), QS_EINVAL, "null argument");
    // the scratch state is a full state (2^34 complex64 = 128 GiB at the limit)
    QS_CHECK(n >= 1 && n <= 34, QS_EINVAL, "autotune supports 1 <= n <= 34 (got %d)", n);
    qs_contract_opts b{};
    if (base) b = *base;
    else {
        b.strategy = QS_STRATEGY_GREEDY;
        b.renorm = 1;
    }
    b.dtype = dtype;
    // a rotation-contracted plan has a pass per several dozen gates: a longer
    // prefix gives it as many passes to time as a greedy plan gets
    const size_t ng = std::min(n_gates, b.strategy == QS_STRATEGY_PAULI ? 4 * kTunePrefix : kTunePrefix);
    const auto key = std::make_tuple(n, (int)dtype, (int)b.strategy, structure_hash(gates, ng));
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            *best = it->second;
            best->renorm = b.renorm;
            return QS_OK;
        }
    }
    const int tcap = dtype == QS_C128 ? 12 : 14;
    int wmax = 1;
    for (size_t i = 0; i < ng; ++i) wmax = std::max(wmax, (int)gates[i].nq);
    struct Cand {
        int k, t, low;
        bool operator==(const Cand &o) const { return k == o.k && t == o.t && low == o.low; }
    };
    std::vector<Cand> cand;
    auto add = [&](int k, int t, int low) {
        const int tt = std::min(t, n), kk = std::min(k, n);
        if (tt < n && std::max(kk, wmax) > tt - 1) return;
        const Cand c{kk, tt, std::min(low, tt)};
        if (std::find(cand.begin(), cand.end(), c) == cand.end()) cand.push_back(c);
    };
    for (int k = 3; k <= 5; ++k)
        for (int t = 11; t <= tcap; ++t)
            for (int low : {4, 6}) add(k, t, low);
    if (cand.empty()) cand.push_back({std::min(2, n), std::min(tcap, n), std::min(6, n)});
    qs_state s = nullptr;
    qs_status st = qs_state_create(n, dtype, nullptr, nullptr, &s);
    if (st != QS_OK) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    float best_ms = 1e30f;
    qs_contract_opts win = b;
    win.k_max = cand[0].k;
    win.tile_qubits = cand[0].t;
    win.low_qubits = cand[0].low;
    auto run = [&](size_t from) {
        for (size_t i = from; i < cand.size(); ++i) {
            qs_contract_opts o = b;
            o.k_max = cand[i].k;
            o.tile_qubits = cand[i].t;
            o.low_qubits = cand[i].low;
            qs_plan p = nullptr;
            if (qs_contract(n, gates, ng, &o, &p) != QS_OK) continue;  // candidate not valid for this circuit
            float ms = 0;
            bool ok = qs_state_set_basis(s, 0) == QS_OK && qs_apply_plan(s, p) == QS_OK;
            if (ok) {
                hipEventRecord(e0, nullptr);
                ok = qs_apply_plan(s, p) == QS_OK;
                hipEventRecord(e1, nullptr);
                ok = ok && hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
            }
            qs_plan_destroy(p);
            if (ok && ms < best_ms) {
                best_ms = ms;
                win = o;
            }
        }
    };
    run(0);
    if (best_ms < 1e30f) {
        const size_t n1 = cand.size();
        for (int low : {3, 5}) add(win.k_max, win.tile_qubits, low);
        run(n1);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    qs_state_destroy(s);
    QS_CHECK(best_ms < 1e30f, QS_EDEVICE, "autotune: no candidate plan could be timed");
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[key] = win;
    }
    *best = win;
    return QS_OK;
    QS_ABI_CATCH
}
