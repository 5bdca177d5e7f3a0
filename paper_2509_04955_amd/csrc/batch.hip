// Batches of independent states run by one persistent kernel in a hipGraph.
//
// Each state (its own qubit count, circuit and Pauli-sum Hamiltonian) gets a
// contraction plan; all passes of all states and all expectation work become
// one work queue:
//   * pass items (state s, pass p, tiles i..i+G-1): the tile kernel's work for
//     a group of consecutive tiles (G up to 16), with the next tile's loads in
//     registers while the current one is processed;
//   * energy items (state s, group of 8 terms, chunk of 2^16 amplitudes):
//     Pauli expectation partials.
// Items are ordered pass-major across states (all first passes, then all
// second passes, ..., then the energy items), so an item only ever waits for
// items earlier in the queue.  The grid never exceeds the resident workgroup
// count, so every earlier item is held by a running workgroup and every wait
// ends; a bounded spin (with an error flag) guarantees termination anyway.
//
// Synchronisation: a finished pass item releases its tile (device-scope fence,
// then an atomic increment of the state's done counter); a dependent item
// acquires it (atomic load until the counter reaches the tiles completed by
// earlier passes, then a fence).  The renormalisation scale of pass p is the
// fixed-order FP64 sum of pass p-1's tile partials, recomputed by every
// consumer, so all of them see the same value.  Energies are reduced by a
// second kernel in fixed order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>

#include "tile_device.h"

namespace qs {
const char *last_error();

namespace {
using namespace tiledev;

constexpr int kPassItem = 0, kEnergyItem = 1;
// A dependency wait gives up after kWaitSeconds of wall-clock time (the device
// wall clock, read with s_memrealtime): a wait that long means the item it
// waits for will not arrive, and the kernel then drains with an error record.
constexpr double kWaitSeconds = 1.0;
// energy items: kTermsPerItem terms of one state over kAmpsPerItem amplitudes
constexpr uint64_t kAmpsPerItem = 1ull << 16;
constexpr int kTermsPerItem = 8;

struct Seg {
    uint64_t first;   // first item index
    uint64_t count;
    int32_t state;
    int32_t kind;
    int32_t pass;     // pass index within the state (pass items)
    int32_t pad;
};

struct PassDev {
    PassArgs pa;
    uint64_t ntiles;
    uint64_t tiles_per_item;   // a pass item covers this many consecutive tiles
    const BlockDev *blocks;
    const void *pool;
    uint64_t need_done;      // tiles of this state completed by earlier passes
    uint64_t part_off;       // this pass's partials (offset into the batch partial array)
    uint64_t prev_part_off;  // previous pass's partials
    uint32_t prev_nparts;    // 0 for the first pass
    uint32_t pad;
};

struct StateDev {
    void *amp;
    int32_t n;
    int32_t npasses;
    uint64_t pass0;         // index of the state's first PassDev
    uint64_t total_tiles;   // tile items over all passes
    uint64_t last_part_off; // partials of the last pass (norm of the stored state)
    uint32_t last_nparts;
    uint32_t nterms;
    uint64_t term0;         // first term in the batch term arrays
    uint32_t terms_per_item;
    uint32_t nchunks;
    uint64_t epart0;        // first energy partial (nterms * nchunks of them)
};

__device__ __forceinline__ uint32_t atomic_load_acq(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// The persistent kernel below is written without lane-divergent branches:
// control work runs on wave 0 under a condition made wave-uniform with
// readfirstlane, lane-0-only effects are selects, and per-wave results are
// stored by every lane of the wave (same value, same address).  This keeps the
// compiler from restructuring the work loop around divergent regions (with a
// `threadIdx.x == 0` region at the loop tail it produced a nested loop in which
// lanes other than lane 0 re-entered the barrier without a new dequeue).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
           (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
}

// Fixed-order FP64 sum of one value per thread over the workgroup.
__device__ double wg_sum_values(double s, double *red) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    __syncthreads();
    red[wave_id()] = s;
    __syncthreads();
    double t = 0;
#pragma unroll
    for (int w = 0; w < TT / 64; ++w) t += red[w];
    __syncthreads();
    return t;
}

// Fixed-order FP64 sum over `count` doubles by the whole workgroup.
__device__ double wg_sum(const double *v, uint32_t count, double *red) {
    double s = 0;
    for (uint32_t i = threadIdx.x; i < count; i += TT) s += v[i];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    __syncthreads();
    red[wave_id()] = s;  // every lane holds the wave sum
    __syncthreads();
    double t = 0;
#pragma unroll
    for (int w = 0; w < TT / 64; ++w) t += red[w];
    __syncthreads();
    return t;
}

// Tiles [t0, t1) of one pass of one state: each tile is loaded into LDS,
// every block of the pass is applied, and the tile is written back with its
// FP64 norm partial (parts[tile]).  The next tile's first kBatchPrefetch
// vectors per thread are loaded into registers while the current tile is
// processed (as in the single-state pass kernel); the rest follow in batches.
// Addresses of vectors past a small tile are clamped (every lane loads), and
// only the LDS writes and global stores are predicated.
constexpr int kBatchPrefetch = 4;

template <typename R, bool WIDE>
__device__ void run_tiles(typename AmpOf<R>::A *psi, const PassDev &pd, uint64_t t0, uint64_t t1, R sc,
                          typename AmpOf<R>::A *tile, double *red, double *parts) {
    using A = typename AmpOf<R>::A;
    constexpr bool F32 = sizeof(R) == 4;
    constexpr uint32_t APV = F32 ? 2 : 1;
    constexpr int PF = kBatchPrefetch;
    const PassArgs &pa = pd.pa;
    const uint32_t nvec = (1u << pa.t) / APV;
    const uint32_t nj = (nvec + TT - 1) / TT;   // vectors per thread (uniform)
    float4 pre[PF];
    auto gptr = [&](uint64_t base, uint32_t j) {
        uint32_t vi = threadIdx.x + j * TT;
        vi = vi < nvec ? vi : nvec - 1;
        return reinterpret_cast<float4 *>(psi + (base | tile_offset(vi * APV, pa)));
    };
    auto put = [&](uint32_t j, float4 v) {
        const uint32_t vi = threadIdx.x + j * TT;
        if (vi < nvec) {
            if constexpr (F32) {
                v.x *= sc;
                v.y *= sc;
                v.z *= sc;
                v.w *= sc;
                *reinterpret_cast<float4 *>(tile + sw(vi * APV)) = v;
            } else {
                double2 d = __builtin_bit_cast(double2, v);
                d.x *= sc;
                d.y *= sc;
                tile[sw(vi)] = d;
            }
        }
    };
    auto load_rest = [&](uint64_t base) {
        for (uint32_t j0 = PF; j0 < nj; j0 += PF) {
#pragma unroll
            for (int i = 0; i < PF; ++i)
                if (j0 + i < nj) pre[i] = *gptr(base, j0 + i);
#pragma unroll
            for (int i = 0; i < PF; ++i)
                if (j0 + i < nj) put(j0 + i, pre[i]);
        }
    };
    uint64_t tl = t0;
    uint64_t base = tile_base(tl, pa);
#pragma unroll
    for (int j = 0; j < PF; ++j)
        if ((uint32_t)j < nj) pre[j] = *gptr(base, j);
#pragma unroll
    for (int j = 0; j < PF; ++j)
        if ((uint32_t)j < nj) put(j, pre[j]);
    load_rest(base);
    const R *pool = reinterpret_cast<const R *>(pd.pool);
    for (;;) {
        __syncthreads();
        const uint64_t nxt = tl + 1;
        const bool more = nxt < t1;   // uniform
        const uint64_t nbase = more ? tile_base(nxt, pa) : base;
#pragma unroll
        for (int j = 0; j < PF; ++j)
            if ((uint32_t)j < nj) pre[j] = *gptr(nbase, j);
        for (int b = 0; b < pa.nblocks; ++b) {
            if (pd.blocks[pa.block0 + b].kind == BK_SKIP) continue;   // folded into a group (uniform)
            apply_block<R, WIDE, false, TT, false>(TilePtr{reinterpret_cast<unsigned char *>(tile)}, pa.t,
                                                   pd.blocks + pa.block0 + b, pool, base);
            __syncthreads();
        }
        double nacc = 0;
        for (uint32_t j = 0; j < nj; ++j) {
            const uint32_t vi = threadIdx.x + j * TT;
            if (vi < nvec) {
                const float4 v = *reinterpret_cast<const float4 *>(tile + sw(vi * APV));
                *gptr(base, j) = v;
                if constexpr (F32) {
                    nacc += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
                } else {
                    const double2 d = __builtin_bit_cast(double2, v);
                    nacc += d.x * d.x + d.y * d.y;
                }
            }
        }
        const double tot = wg_sum_values(nacc, red);   // ends with a barrier: the tile is free again
        if (wave_id() == 0) parts[tl] = tot;  // same value from every lane of wave 0
        if (!more) break;
#pragma unroll
        for (int j = 0; j < PF; ++j)
            if ((uint32_t)j < nj) put(j, pre[j]);
        load_rest(nbase);
        tl = nxt;
        base = nbase;
    }
}

__device__ __forceinline__ uint64_t ins0(uint64_t x, int p) {
    const uint64_t lo = x & ((1ull << p) - 1);
    return ((x - lo) << 1) | lo;
}

// Expectation partials of kTermsPerItem Pauli terms over one amplitude chunk.
// P = i^{n_Y} X^x Z^z (Y = i X Z on each qubit where x and z are both set)
// maps |k> to i^{n_Y} (-1)^{popcount(k & z)} |k xor x>, so
//   <psi|P|psi> = Re( i^{n_Y} sum_k (-1)^{popcount(k & z)} conj(psi[k xor x]) psi[k] ).
// Each thread loads its own 16-byte vector once and gathers the partner
// psi[k xor x] for every term of the group; products and sums are FP64.
// Every lane runs the same number of iterations (vectors past the chunk are
// clamped and weighted by zero): the persistent kernel has no lane-divergent
// control flow.  Term t's sum over the chunk goes to out[t * stride].
template <typename R>
__device__ void energy_item(const typename AmpOf<R>::A *__restrict__ psi, int n, uint64_t chunk,
                            const uint64_t *__restrict__ xs, const uint64_t *__restrict__ zs, uint32_t nterms,
                            double *__restrict__ out, uint64_t stride, double *red) {
    constexpr int G = kTermsPerItem;
    constexpr uint32_t APV = sizeof(R) == 4 ? 2 : 1;
    const uint64_t namps = 1ull << n;
    const uint64_t C = namps < kAmpsPerItem ? namps : kAmpsPerItem;
    const uint64_t a0 = chunk * C;
    const uint32_t nv = (uint32_t)(C / APV);   // n >= 1, so C >= APV
    const uint32_t iters = (nv + TT - 1) / TT;
    uint64_t x[G], z[G];
    double sg[G];   // +1 or -1: the real factor of i^{n_Y}
    bool im[G];     // i^{n_Y} is imaginary: the term takes Im of the sum
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const bool ok = (uint32_t)g < nterms;
        const int gi = ok ? g : 0;   // index 0 always exists (nterms >= 1): no load past the arrays
        x[g] = ok ? xs[gi] : 0;
        z[g] = ok ? zs[gi] : 0;
        const int ny = __popcll(x[g] & z[g]) & 3;
        im[g] = ny & 1;
        sg[g] = (ny == 1 || ny == 2) ? -1.0 : 1.0;
    }
    double acc[G];
#pragma unroll
    for (int g = 0; g < G; ++g) acc[g] = 0.0;
    for (uint32_t it = 0; it < iters; ++it) {
        const uint32_t v = it * TT + threadIdx.x;
        const double on = v < nv ? 1.0 : 0.0;
        const uint64_t k0 = a0 + (uint64_t)(v < nv ? v : nv - 1) * APV;
        if constexpr (APV == 2) {
            const float4 own = reinterpret_cast<const float4 *>(psi)[k0 >> 1];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const uint64_t p0 = k0 ^ x[g];
                const float4 pv = reinterpret_cast<const float4 *>(psi)[p0 >> 1];
                const bool swp = p0 & 1;   // partner of amplitude k0 is the odd half
                const double b0r = swp ? pv.z : pv.x, b0i = swp ? pv.w : pv.y;
                const double b1r = swp ? pv.x : pv.z, b1i = swp ? pv.y : pv.w;
                const double s0 = (__popcll(k0 & z[g]) & 1) ? -1.0 : 1.0;
                const double s1 = (__popcll((k0 + 1) & z[g]) & 1) ? -1.0 : 1.0;
                const double w0 = im[g] ? b0r * own.y - b0i * own.x : b0r * own.x + b0i * own.y;
                const double w1 = im[g] ? b1r * own.w - b1i * own.z : b1r * own.z + b1i * own.w;
                acc[g] += on * sg[g] * (s0 * w0 + s1 * w1);
            }
        } else {
            const typename AmpOf<R>::A a = psi[k0];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const typename AmpOf<R>::A bb = psi[k0 ^ x[g]];
                const double s0 = (__popcll(k0 & z[g]) & 1) ? -1.0 : 1.0;
                const double w0 = im[g] ? (double)bb.x * a.y - (double)bb.y * a.x : (double)bb.x * a.x + (double)bb.y * a.y;
                acc[g] += on * sg[g] * s0 * w0;
            }
        }
    }
    // fixed-order reduction: lanes (shuffles), then the waves in order
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) acc[g] += __shfl_xor(acc[g], o);
        red[g * (TT / 64) + wave_id()] = acc[g];   // every lane holds the wave sum
    }
    __syncthreads();
    if (wave_id() == 0) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            double t = 0;
#pragma unroll
            for (int w = 0; w < TT / 64; ++w) t += red[g * (TT / 64) + w];
            if ((uint32_t)g < nterms) out[g * stride] = t;   // same value from every lane
        }
    }
    __syncthreads();
}

template <typename R, bool WIDE>
__global__ __launch_bounds__(TT, WIDE ? 1 : 2) void k_batch(const Seg *__restrict__ segs, int nsegs, uint64_t total_items,
                                              const StateDev *__restrict__ states, const PassDev *__restrict__ passes,
                                              const uint64_t *__restrict__ xs, const uint64_t *__restrict__ zs,
                                              double *__restrict__ partials, double *__restrict__ eparts,
                                              uint32_t *__restrict__ done, unsigned long long *__restrict__ queue,
                                              uint32_t *__restrict__ error, unsigned long long *__restrict__ diag,
                                              uint64_t wait_ticks) {
    using A = typename AmpOf<R>::A;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    A *tile = reinterpret_cast<A *>(smem_raw);
    __shared__ double red[TT / 64];
    __shared__ double ered[kTermsPerItem * (TT / 64)];
    __shared__ unsigned long long s_item;
    __shared__ int s_ok;
    const bool lane0 = (threadIdx.x & 63) == 0;
    const bool w0 = wave_id() == 0;
    for (;;) {
        // ---- dequeue (wave 0; lane 0 adds 1, the other lanes add 0) ----
        if (w0) {
            const unsigned long long t = atomicAdd(queue, lane0 ? 1ull : 0ull);
            s_item = uniform64(t);
        }
        __syncthreads();
        const uint64_t item = uniform64(s_item);
        __syncthreads();
        if (item >= total_items) break;
        int lo = 0, hi = nsegs - 1;  // last segment with first <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (segs[mid].first <= item) lo = mid;
            else hi = mid - 1;
        }
        const Seg sg = segs[lo];
        const StateDev st = states[sg.state];
        const uint64_t local = item - sg.first;
        uint64_t need;
        const PassDev *pd = nullptr;
        if (sg.kind == kPassItem) {
            pd = passes + st.pass0 + sg.pass;
            need = pd->need_done;
        } else {
            need = st.total_tiles;
        }
        // ---- acquire: wave 0 waits for the items this one depends on ----
        if (w0) {
            int ok = 1;
            uint32_t seen = __builtin_amdgcn_readfirstlane(atomic_load_acq(done + sg.state));
            if (seen < need) {
                const uint64_t t0 = uniform64(wall_clock64());
                for (;;) {
                    __builtin_amdgcn_s_sleep(8);
                    const uint32_t err = __builtin_amdgcn_readfirstlane(
                        __hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                    if (err) {
                        ok = 0;
                        break;
                    }
                    if (uniform64(wall_clock64()) - t0 > wait_ticks) {
                        const uint32_t prev = __builtin_amdgcn_readfirstlane(atomicCAS(error, 0u, lane0 ? 1u : 0u));
                        if (prev == 0u) {
                            diag[0] = (unsigned long long)sg.state;
                            diag[1] = need;
                            diag[2] = seen;
                            diag[3] = item;
                        }
                        ok = 0;
                        break;
                    }
                    seen = __builtin_amdgcn_readfirstlane(atomic_load_acq(done + sg.state));
                    if (seen >= need) break;
                }
            }
            s_ok = ok;
        }
        __syncthreads();
        const int ok_all = __builtin_amdgcn_readfirstlane(s_ok);
        if (!ok_all) break;
        __threadfence();
        A *psi = reinterpret_cast<A *>(st.amp);
        if (sg.kind == kPassItem) {
            R sc = (R)1;
            if (pd->prev_nparts) {
                const double N = wg_sum(partials + pd->prev_part_off, pd->prev_nparts, red);
                sc = (R)(N > 0 ? 1.0 / sqrt(N) : 1.0);
            }
            const uint64_t t0 = local * pd->tiles_per_item;
            const uint64_t t1 = t0 + pd->tiles_per_item < pd->ntiles ? t0 + pd->tiles_per_item : pd->ntiles;
            run_tiles<R, WIDE>(psi, *pd, t0, t1, sc, tile, red, partials + pd->part_off);
            __syncthreads();
            // ---- release: wave 0 publishes the finished tiles ----
            if (w0) {
                __threadfence();
                atomicAdd(done + sg.state, lane0 ? (uint32_t)(t1 - t0) : 0u);
            }
        } else {
            // energy item: (term group, chunk)
            const uint64_t chunk = local % st.nchunks;
            const uint64_t tg = local / st.nchunks;
            const uint64_t t0 = tg * kTermsPerItem;
            const uint32_t left = st.nterms - (uint32_t)t0;
            energy_item<R>(psi, st.n, chunk, xs + st.term0 + t0, zs + st.term0 + t0,
                           left < (uint32_t)kTermsPerItem ? left : (uint32_t)kTermsPerItem,
                           eparts + st.epart0 + t0 * st.nchunks + chunk, st.nchunks, ered);
        }
        __syncthreads();
    }
}

// zero every state, then |0...0>; reset counters (a fill kernel: graph-safe)
__global__ __launch_bounds__(256) void k_batch_reset(uint4 *__restrict__ amps, uint64_t words,
                                                     uint32_t *__restrict__ done, int nstates,
                                                     unsigned long long *__restrict__ queue,
                                                     uint32_t *__restrict__ error) {
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += stride) amps[i] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < nstates; i += 256) done[i] = 0;
        if (threadIdx.x == 0) {
            *queue = 0;
            *error = 0;
        }
    }
}

template <typename A>
__global__ void k_batch_basis(const StateDev *__restrict__ states, int nstates) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nstates) {
        A one;
        one.x = 1;
        one.y = 0;
        reinterpret_cast<A *>(states[i].amp)[0] = one;
    }
}

// one workgroup per state: fixed-order sums
__global__ __launch_bounds__(256) void k_batch_energy(const StateDev *__restrict__ states,
                                                      const double *__restrict__ coeff,
                                                      const double *__restrict__ partials,
                                                      const double *__restrict__ eparts, double *__restrict__ energies) {
    __shared__ double red[4];
    const StateDev st = states[blockIdx.x];
    const double N = wg_sum(partials + st.last_part_off, st.last_nparts, red);
    double e = 0;
    for (uint32_t t = 0; t < st.nterms; ++t) {
        const double v = wg_sum(eparts + st.epart0 + (uint64_t)t * st.nchunks, st.nchunks, red);
        e += coeff[st.term0 + t] * v;
    }
    if (threadIdx.x == 0) energies[blockIdx.x] = e / N;
}

}  // namespace
}  // namespace qs

using namespace qs;

struct qs_batch_s {
    qs_dtype dtype = QS_C64;
    hipStream_t stream = nullptr;
    int nstates = 0;
    std::vector<qs_plan_s *> plans;
    std::vector<int> n;
    std::vector<uint64_t> amp_off;  // bytes
    void *d_amps = nullptr;
    uint64_t amp_bytes = 0;
    Seg *d_segs = nullptr;
    int nsegs = 0;
    uint64_t total_items = 0;
    StateDev *d_states = nullptr;
    PassDev *d_passes = nullptr;
    uint64_t *d_x = nullptr, *d_z = nullptr;
    double *d_coeff = nullptr, *d_partials = nullptr, *d_eparts = nullptr, *d_energy = nullptr;
    uint32_t *d_done = nullptr, *d_error = nullptr;
    unsigned long long *d_queue = nullptr, *d_diag = nullptr;
    uint64_t wait_ticks = 0;
    bool wide = false;
    size_t lds = 0;
    unsigned grid = 1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~qs_batch_s() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        void *bufs[] = {d_amps, d_segs, d_states, d_passes, d_x, d_z, d_coeff, d_partials, d_eparts, d_energy,
                        d_done, d_error, d_queue, d_diag};
        for (void *b : bufs)
            if (b) hipFree(b);
        for (qs_plan_s *p : plans) qs_plan_destroy(p);
    }
};

namespace {

template <typename T>
qs_status upload(T **dst, const std::vector<T> &src) {
    QS_HIP(hipMalloc((void **)dst, std::max<size_t>(1, src.size()) * sizeof(T)));
    if (!src.empty()) QS_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return QS_OK;
}

template <typename R, bool WIDE>
const void *batch_kernel() {
    return reinterpret_cast<const void *>(&k_batch<R, WIDE>);
}

qs_status enqueue_batch(qs_batch_s &b, hipStream_t st) {
    const uint64_t words = b.amp_bytes / 16;
    hipLaunchKernelGGL(k_batch_reset, dim3(1024), dim3(256), 0, st, (uint4 *)b.d_amps, words, b.d_done, b.nstates,
                       b.d_queue, b.d_error);
    const unsigned nb = (unsigned)((b.nstates + 255) / 256);
    if (b.dtype == QS_C64)
        hipLaunchKernelGGL(k_batch_basis<float2>, dim3(nb), dim3(256), 0, st, b.d_states, b.nstates);
    else
        hipLaunchKernelGGL(k_batch_basis<double2>, dim3(nb), dim3(256), 0, st, b.d_states, b.nstates);
#define QS_BATCH(R, W)                                                                                        \
    hipLaunchKernelGGL((k_batch<R, W>), dim3(b.grid), dim3(TT), b.lds, st, b.d_segs, b.nsegs, b.total_items,   \
                       b.d_states, b.d_passes, b.d_x, b.d_z, b.d_partials, b.d_eparts, b.d_done, b.d_queue,   \
                       b.d_error, b.d_diag, b.wait_ticks)
    if (b.dtype == QS_C64) {
        if (b.wide) QS_BATCH(float, true);
        else QS_BATCH(float, false);
    } else {
        if (b.wide) QS_BATCH(double, true);
        else QS_BATCH(double, false);
    }
#undef QS_BATCH
    hipLaunchKernelGGL(k_batch_energy, dim3(b.nstates), dim3(256), 0, st, b.d_states, b.d_coeff, b.d_partials,
                       b.d_eparts, b.d_energy);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

}  // namespace

extern "C" {

qs_status qs_batch_create(int n_states, const int *n_qubits, const qs_gate *const *circuits, const size_t *n_gates,
                          const uint64_t *const *x, const uint64_t *const *z, const double *const *coeff,
                          const size_t *n_terms, const qs_contract_opts *opts, void *stream, qs_batch *out) {
    QS_ABI_TRY
    QS_CHECK(out && n_qubits && circuits && n_gates && x && z && coeff && n_terms, QS_EINVAL, "null argument");
    QS_CHECK(n_states >= 1 && n_states <= 65536, QS_EINVAL, "n_states %d outside 1..65536", n_states);
    qs_contract_opts base{};
    if (opts) base = *opts;
    if (base.strategy == 0 && !opts) base.strategy = QS_STRATEGY_GREEDY;
    if (!opts) base.renorm = 1;
    const qs_dtype dt = base.dtype == QS_C128 ? QS_C128 : QS_C64;
    for (int i = 0; i < n_states; ++i) {
        QS_CHECK(n_qubits[i] >= 1 && n_qubits[i] <= 26, QS_EINVAL, "state %d: n=%d outside 1..26", i, n_qubits[i]);
        QS_CHECK(n_terms[i] >= 1 && n_terms[i] <= (1u << 16), QS_EINVAL, "state %d: n_terms outside 1..65536", i);
        const uint64_t lim = (1ull << n_qubits[i]) - 1;
        for (size_t k = 0; k < n_terms[i]; ++k)
            QS_CHECK((x[i][k] & ~lim) == 0 && (z[i][k] & ~lim) == 0, QS_EINVAL, "state %d term %zu out of range", i, k);
    }
    qs_batch_s *b = new (std::nothrow) qs_batch_s();
    QS_CHECK(b != nullptr, QS_ENOMEM, "host allocation failed");
    b->dtype = dt;
    b->stream = (hipStream_t)stream;
    b->nstates = n_states;
    auto fail = [&](qs_status s) {
        delete b;
        return s;
    };
    // ---- plans (autotuned per qubit count when k_max or tile is 0) ----
    std::map<int, qs_contract_opts> tuned;
    for (int i = 0; i < n_states; ++i) {
        qs_contract_opts o = base;
        o.dtype = dt;
        if (base.k_max == 0 || base.tile_qubits == 0) {
            auto it = tuned.find(n_qubits[i]);
            if (it == tuned.end()) {
                qs_contract_opts best{};
                qs_status st = qs_autotune(n_qubits[i], dt, circuits[i], n_gates[i], &o, &best);
                if (st != QS_OK) return fail(st);
                it = tuned.emplace(n_qubits[i], best).first;
            }
            o = it->second;
        }
        // The batch kernel applies complex128 blocks wider than 3 qubits on the
        // vector ALU in its wide variant (no staged FP64 MFMA there), which the
        // single-state timings of the autotuner do not see: keep them narrow.
        if (dt == QS_C128 && (base.k_max == 0 || base.tile_qubits == 0)) o.k_max = std::min(o.k_max, 3);
        // The single-state pass kernel runs 2^13- and 2^14-amplitude tiles with
        // 512 and 1024 threads; the batch kernel has 256, where such tiles hold
        // a CU to one or two workgroups.  Tuned tiles stay at 2^12 here.
        if ((base.k_max == 0 || base.tile_qubits == 0) && o.tile_qubits > 12) o.tile_qubits = 12;
        qs_plan p = nullptr;
        qs_status st = qs_contract(n_qubits[i], circuits[i], n_gates[i], &o, &p);
        if (st != QS_OK) {
            std::string m = last_error();
            set_error("state %d: %s", i, m.c_str());
            return fail(st);
        }
        b->plans.push_back(p);
        b->n.push_back(n_qubits[i]);
        st = plan_upload(*p, dt, false);
        if (st != QS_OK) return fail(st);
    }
    // ---- device layout ----
    const size_t ab = dt == QS_C64 ? 8 : 16;
    uint64_t off = 0;
    for (int i = 0; i < n_states; ++i) {
        b->amp_off.push_back(off);
        off += ((ab << b->n[i]) + 255) / 256 * 256;
    }
    b->amp_bytes = off;
    hipError_t e = hipMalloc(&b->d_amps, off);
    if (e != hipSuccess) return fail(hip_fail(e, "hipMalloc(batch states)"));
    std::vector<StateDev> sd(n_states);
    std::vector<PassDev> pdv;
    std::vector<uint64_t> hx, hz;
    std::vector<double> hc;
    uint64_t parts = 0, eparts = 0;
    int maxt = 1;
    size_t maxpasses = 0;
    for (int i = 0; i < n_states; ++i) {
        qs_plan_s &p = *b->plans[i];
        StateDev &s = sd[i];
        std::memset(&s, 0, sizeof s);
        s.amp = (unsigned char *)b->d_amps + b->amp_off[i];
        s.n = b->n[i];
        s.npasses = (int)p.passes.size();
        s.pass0 = pdv.size();
        uint64_t done_before = 0, prev_off = 0;
        uint32_t prev_n = 0;
        const int di = dt == QS_C64 ? 0 : 1;
        for (size_t pi = 0; pi < p.passes.size(); ++pi) {
            const HPass &ps = p.passes[pi];
            PassDev d;
            std::memset(&d, 0, sizeof d);
            d.pa.t = ps.t;
            d.pa.c = ps.c;
            d.pa.nblocks = (int32_t)ps.nblocks;
            d.pa.block0 = (int32_t)ps.block0;
            for (int j = 0; j < ps.t - ps.c; ++j) d.pa.hi[j] = ps.tile[ps.c + j];
            d.pa.want_norm = 1;
            d.ntiles = 1ull << (s.n - ps.t);
            // items of up to 16 tiles, at least 4 items per pass when the pass has them
            d.tiles_per_item = std::min<uint64_t>(16, std::max<uint64_t>(1, d.ntiles / 4));
            d.blocks = p.d_blocks[di];
            d.pool = p.d_pool[di];
            d.need_done = done_before;
            d.part_off = parts;
            d.prev_part_off = prev_off;
            d.prev_nparts = prev_n;
            prev_off = parts;
            prev_n = (uint32_t)d.ntiles;
            parts += d.ntiles;
            done_before += d.ntiles;
            maxt = std::max(maxt, ps.t);
            if (p.pass_wide[di][pi]) b->wide = true;
            pdv.push_back(d);
        }
        maxpasses = std::max(maxpasses, p.passes.size());
        s.total_tiles = done_before;
        s.last_part_off = prev_off;
        s.last_nparts = prev_n;
        s.nterms = (uint32_t)n_terms[i];
        s.term0 = hx.size();
        s.nchunks = (uint32_t)std::max<uint64_t>(1, (1ull << s.n) / kAmpsPerItem);
        s.terms_per_item = (uint32_t)kTermsPerItem;
        s.epart0 = eparts;
        eparts += (uint64_t)s.nterms * s.nchunks;
        for (size_t k = 0; k < n_terms[i]; ++k) {
            hx.push_back(x[i][k]);
            hz.push_back(z[i][k]);
            hc.push_back(coeff[i][k]);
        }
    }
    // an empty circuit still needs the norm of |0>: give such states one identity pass
    for (int i = 0; i < n_states; ++i)
        if (sd[i].npasses == 0) {
            set_error("state %d has an empty circuit", i);
            return fail(QS_EINVAL);
        }
    // ---- queue: pass-major over states, then energy items ----
    std::vector<Seg> segs;
    uint64_t item = 0;
    for (size_t pi = 0; pi < maxpasses; ++pi)
        for (int i = 0; i < n_states; ++i)
            if ((int)pi < sd[i].npasses) {
                const PassDev &pd = pdv[sd[i].pass0 + pi];
                Seg s{item, (pd.ntiles + pd.tiles_per_item - 1) / pd.tiles_per_item, i, kPassItem, (int32_t)pi, 0};
                segs.push_back(s);
                item += s.count;
            }
    for (int i = 0; i < n_states; ++i) {
        const uint64_t groups = (sd[i].nterms + sd[i].terms_per_item - 1) / sd[i].terms_per_item;
        Seg s{item, groups * sd[i].nchunks, i, kEnergyItem, 0, 0};
        segs.push_back(s);
        item += s.count;
    }
    b->total_items = item;
    b->nsegs = (int)segs.size();
    qs_status st;
    if ((st = upload(&b->d_segs, segs)) != QS_OK) return fail(st);
    if ((st = upload(&b->d_states, sd)) != QS_OK) return fail(st);
    if ((st = upload(&b->d_passes, pdv)) != QS_OK) return fail(st);
    if ((st = upload(&b->d_x, hx)) != QS_OK) return fail(st);
    if ((st = upload(&b->d_z, hz)) != QS_OK) return fail(st);
    if ((st = upload(&b->d_coeff, hc)) != QS_OK) return fail(st);
    e = hipMalloc(&b->d_partials, std::max<uint64_t>(1, parts) * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&b->d_eparts, std::max<uint64_t>(1, eparts) * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&b->d_energy, n_states * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&b->d_done, n_states * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&b->d_error, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&b->d_queue, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(&b->d_diag, 4 * sizeof(unsigned long long));
    if (e != hipSuccess) return fail(hip_fail(e, "hipMalloc(batch)"));
    {
        int dev0 = 0, khz = 0;
        e = hipGetDevice(&dev0);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev0);
        if (e != hipSuccess || khz <= 0) return fail(e != hipSuccess ? hip_fail(e, "wall clock rate") : QS_EDEVICE);
        b->wait_ticks = (uint64_t)(kWaitSeconds * 1000.0 * khz);
    }
    // ---- persistent grid: resident workgroups only ----
    b->lds = ab << maxt;
    const void *kern = dt == QS_C64 ? (b->wide ? batch_kernel<float, true>() : batch_kernel<float, false>())
                                    : (b->wide ? batch_kernel<double, true>() : batch_kernel<double, false>());
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds);
    if (e != hipSuccess) return fail(hip_fail(e, "hipFuncSetAttribute(batch)"));
    int per_cu = 0, dev = 0;
    hipDeviceProp_t prop;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, TT, b->lds);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return fail(hip_fail(e, "occupancy query"));
    QS_CHECK(per_cu >= 1, QS_EDEVICE, "batch kernel cannot be resident");
    b->grid = (unsigned)std::min<uint64_t>((uint64_t)per_cu * prop.multiProcessorCount, std::max<uint64_t>(1, item));
    // ---- capture the whole batch in one graph ----
    hipStream_t cap = nullptr;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(hip_fail(e, "hipStreamCreate"));
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = enqueue_batch(*b, cap);
        hipError_t e2 = hipStreamEndCapture(cap, &b->graph);
        if (st == QS_OK && e2 != hipSuccess) st = hip_fail(e2, "hipStreamEndCapture");
    } else {
        st = hip_fail(e, "hipStreamBeginCapture");
    }
    hipStreamDestroy(cap);
    if (st != QS_OK) return fail(st);
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return fail(hip_fail(e, "hipGraphInstantiate"));
    *out = b;
    return QS_OK;
    QS_ABI_CATCH
}

qs_status qs_batch_destroy(qs_batch b) {
    if (!b) return QS_OK;
    hipStreamSynchronize(b->stream);
    delete b;
    return QS_OK;
}

qs_status qs_batch_run(qs_batch b, double *energies) {
    QS_CHECK(b != nullptr, QS_EINVAL, "null batch");
    QS_HIP(hipGraphLaunch(b->exec, b->stream));
    uint32_t err = 0;
    unsigned long long dg[4] = {0, 0, 0, 0};
    QS_HIP(hipMemcpyAsync(&err, b->d_error, sizeof err, hipMemcpyDeviceToHost, b->stream));
    QS_HIP(hipMemcpyAsync(dg, b->d_diag, sizeof dg, hipMemcpyDeviceToHost, b->stream));
    if (energies)
        QS_HIP(hipMemcpyAsync(energies, b->d_energy, b->nstates * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    QS_HIP(hipStreamSynchronize(b->stream));
    QS_CHECK(err == 0, QS_EDEVICE,
             "batch kernel: dependency wait timed out (state %llu needed %llu finished tiles, saw %llu; item %llu)",
             dg[0], dg[1], dg[2], dg[3]);
    return QS_OK;
}

qs_status qs_batch_state_copy_out(qs_batch b, int i, double *host) {
    QS_CHECK(b && host, QS_EINVAL, "null argument");
    QS_CHECK(i >= 0 && i < b->nstates, QS_EINVAL, "state index out of range");
    QS_HIP(hipStreamSynchronize(b->stream));
    const qs_plan_s &p = *b->plans[i];
    (void)p;
    const int n = b->n[i];
    const uint64_t cnt = 1ull << n;
    // the stored amplitudes carry the last pass's pending scale: read the partials back
    double N = 0;
    {
        // norm of the stored state = fixed-order sum of the last pass's partials
        StateDev sd;
        QS_HIP(hipMemcpy(&sd, b->d_states + i, sizeof sd, hipMemcpyDeviceToHost));
        std::vector<double> parts(sd.last_nparts);
        QS_HIP(hipMemcpy(parts.data(), b->d_partials + sd.last_part_off, parts.size() * sizeof(double),
                         hipMemcpyDeviceToHost));
        for (double v : parts) N += v;
    }
    const double scale = N > 0 ? 1.0 / std::sqrt(N) : 1.0;
    const unsigned char *src = (const unsigned char *)b->d_amps + b->amp_off[i];
    if (b->dtype == QS_C64) {
        std::vector<float> f(2 * cnt);
        QS_HIP(hipMemcpy(f.data(), src, f.size() * sizeof(float), hipMemcpyDeviceToHost));
        for (uint64_t k = 0; k < 2 * cnt; ++k) host[k] = f[k] * scale;
    } else {
        QS_HIP(hipMemcpy(host, src, 2 * cnt * sizeof(double), hipMemcpyDeviceToHost));
        for (uint64_t k = 0; k < 2 * cnt; ++k) host[k] *= scale;
    }
    return QS_OK;
}

}  // extern "C"
