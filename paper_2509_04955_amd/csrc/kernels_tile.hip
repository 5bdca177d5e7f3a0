// Streamed tile passes: the fused hot path.
//
// A pass reads the whole state once and writes it once (one kernel), and
// applies every fused block of the pass in between.  The state is split into
// tiles of 2^t amplitudes: tile positions 0..c-1 are the contiguous low qubits
// (coalesced runs of 2^c amplitudes) and positions c..t-1 are high qubits
// chosen by the planner, so each tile is 2^(t-c) strided segments (the
// grouping idea of Section 2.2, Algorithms 3-4, taken to whole sets of
// qubits).  A workgroup stages its tile in LDS, applies the blocks in order
// (each block is a dense 2^k x 2^k unitary on k of the tile's qubits, Eq. 6
// generalised), and writes the tile back.  Tiles partition the index space,
// so passes need no atomics on amplitudes (the conflict-freedom that the
// staggered schedule of Section 3.3 obtains by construction).
//
// Block arithmetic:
//   * k <= 3 (complex64) or any k (complex128): vector ALU, one group of 2^k
//     amplitudes per lane, matrix entries wave-uniform (scalar loads).
//   * k = 4, 5 (complex64): MFMA.  Y = U X is the real GEMM
//     [[Ur, -Ui], [Ui, Ur]] [Xr; Xi] with M = K = 2^(k+1), N = 16 tile columns
//     per v_mfma_f32_16x16x4f32 chain, FP32 accumulation.  The A operand is
//     pre-swizzled on the host so each lane loads its 4^(k+1)/64 values once.
//   * Renormalisation: a pass multiplies by the previous pass's 1/sqrt(N) on
//     load and accumulates sum |a|^2 in FP64 on store, one partial per
//     workgroup over its tiles in tile order; a single workgroup then sums the
//     partials in a fixed order (deterministic for a given grid).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "tile_device.h"

namespace qs {

namespace {

constexpr uint32_t kMaxTileGrid = 1u << 20;
using namespace tiledev;

// Amplitude vectors each lane prefetches for the next tile while the current
// tile is being processed (16-byte vectors: 2 complex64 or 1 complex128).
constexpr int kPrefetch = 6;

// Streaming accesses to the state bypass cache retention (non-temporal): each
// amplitude is read once and written once per pass.  A thread moves 16-byte
// vectors: two complex64 amplitudes (4 floats) or one complex128 (2 doubles).
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef double vd2 __attribute__((ext_vector_type(2)));
template <typename R>
struct Vec16;
template <>
struct Vec16<float> {
    using V = vf4;
};
template <>
struct Vec16<double> {
    using V = vd2;
};
template <typename V>
__device__ __forceinline__ V ld_nt(const V *p) {
    return __builtin_nontemporal_load(p);
}
template <typename V>
__device__ __forceinline__ void st_nt(V *p, V v) {
    __builtin_nontemporal_store(v, p);
}

// A double moved between lanes by a DPP pattern within rows of 16 lanes.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes of a wave (every lane active), the same value in
// every lane, in a fixed order: within each row of 16 lanes by DPP moves
// (lane ^ 1, lane ^ 2, mirror within 8, mirror within 16; after each step
// partner lanes hold the same sum, IEEE addition being commutative), then the
// four row sums read from lanes 0, 16, 32, 48.  No LDS traffic and no waits.
__device__ __forceinline__ double wave_sum_f64(double v) {
    v += dpp_f64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);   // row_half_mirror
    v += dpp_f64<0x140>(v);   // row_mirror
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Tile index li of 16-byte vector vi = tid + NT*j (NT threads per workgroup)
// splits into a per-thread part (tid*APV, below NT*APV) and a per-j part
// (j*NT*APV); both the global
// offset map and the LDS swizzle are bitwise, so each address is the per-thread
// constant combined with a wave-uniform per-j value.
//
// NJ > 0 fixes the number of 16-byte vectors per thread at compile time (the
// tile is exactly NJ*NT*APV amplitudes): every load and store is then
// unconditional and the next tile's vectors beyond the prefetch depth are
// loaded into registers after the blocks, before the stores.
// NJ = 0 handles any tile size; vectors beyond the prefetch depth are then
// loaded in batches whose loads are all issued before the first of them is
// waited on.
// Waves per SIMD the register budget is sized for: complex64 tiles of up to
// 2^12 amplitudes run 4 workgroups per CU; 2^13-amplitude complex64 tiles and
// complex128 tiles are held to 2 per CU by LDS or registers anyway, so those
// variants take twice the registers and prefetch the whole next tile.
// With the pass's block operands staged in LDS (CL) a 2^12-amplitude
// complex64 tile runs 3 workgroups per CU, leaving about 20 KB of LDS per
// workgroup for the operands.  Unstaged 2^13- and 2^14-amplitude complex64
// tiles run with 512 and 1024 threads (8 vectors per thread, 4 waves per
// SIMD): 2 workgroups per CU and 1, the same wave count as 2^12 tiles.  The
// staged 512-thread variant prefetches 6 of its 8 vectors: 6 leave the
// compiler three spilled registers, reloaded only in the staged 5- and
// 6-qubit monomial paths (measured 1.8 % faster per pass than 4 on the
// 30-qubit UCC circuit); with all 8 the reloads move into the store phase.
template <typename R, bool WIDE, int NJ, bool CL, int NT = TT>
constexpr int tile_waves() {
    // NJ = 0 (tiles below 2^9 complex64 amplitudes) never fills a CU anyway
    if (NT > TT) return 4;
    return WIDE ? 1 : (sizeof(R) == 4 && NJ > 0 && NJ < 16 ? (CL && NJ == 8 ? 3 : 4) : 2);
}

// LDS of a tile pass.  Unstaged variants of a fixed tile size hold the tile,
// the per-wave norm slots and the ticket slots in static LDS and take no
// dynamic LDS.  The others declare no static LDS; their dynamic region is the
// tile (2^t amplitudes), the norm slots, the ticket slots, then the staged
// block operands.  Either way the tile sits at an LDS address aligned to
// kTileAlign (block code then forms addresses with OR and XOR alone).
constexpr size_t kRedBytes = 128 + 16;   // NT / 64 doubles for up to 1024 threads, two ticket slots

template <typename R, bool WIDE, int NJ, bool CL, int NT = TT>
__global__ __launch_bounds__(NT, (tile_waves<R, WIDE, NJ, CL, NT>())) void k_tile_pass(
    typename AmpOf<R>::A *__restrict__ psi, uint64_t ntiles, PassArgs pa, const BlockDev *__restrict__ blocks,
    const R *__restrict__ pool, const double *__restrict__ scale_in, double *__restrict__ partials,
    unsigned long long *__restrict__ tickets, unsigned long long ticket0) {
    using A = typename AmpOf<R>::A;
    constexpr bool F32 = sizeof(R) == 4;
    constexpr uint32_t APV = F32 ? 2 : 1;  // amplitudes per 16-byte vector
    constexpr int PFMAX = NT > TT && CL ? 6 : tile_waves<R, WIDE, NJ, CL, NT>() <= 3 ? (sizeof(R) == 8 ? 8 : 16) : kPrefetch;
    constexpr int PF = NJ > 0 ? (NJ < PFMAX ? NJ : PFMAX) : kPrefetch;
    constexpr int EX = NJ > PF ? NJ - PF : 0;   // compile-time tiles: vectors loaded after the blocks
    static_assert(NT / 64 * sizeof(double) + 2 * sizeof(uint64_t) <= kRedBytes, "norm and ticket slots");
    const int T = pa.t;
    const uint32_t tsize = 1u << T;
    A *tile;
    double *red;
    uint64_t *next_slot;
    R *cst = nullptr;
    if constexpr (NJ > 0 && !CL) {
        // fixed tile size, no staged operands: tile and slots in static LDS,
        // whose addresses are constants the compiler folds into every access
        // (the staged variants keep the dynamic layout: with a static tile
        // their register allocation spills)
        __shared__ __align__(kTileAlign) A tile_s[NJ * NT * APV];
        __shared__ double red_s[NT / 64];
        __shared__ uint64_t next_s[2];
        tile = tile_s;
        red = red_s;
        next_slot = next_s;
    } else {
        // no static LDS in these variants: the dynamic region starts at LDS
        // address 0, which meets the declared alignment
        extern __shared__ __align__(kTileAlign) unsigned char smem_raw[];
        tile = reinterpret_cast<A *>(smem_raw);
        red = reinterpret_cast<double *>(smem_raw + (size_t)tsize * sizeof(A));
        next_slot = reinterpret_cast<uint64_t *>(smem_raw + (size_t)tsize * sizeof(A) + 128);
        cst = reinterpret_cast<R *>(smem_raw + (size_t)tsize * sizeof(A) + kRedBytes);
    }
    const TileAligned tl{lds_addr(tile)};
    const R sc = pa.apply_scale ? (R)(*scale_in) : (R)1;
    const uint32_t my_li = threadIdx.x * APV;
    const bool active = NJ > 0 || my_li < tsize;   // small tiles: fewer vectors than threads
    const uint64_t g_t = active ? tile_offset(my_li, pa) : 0;
    const uint32_t s_t = sw(my_li);
    const uint32_t nj = NJ > 0 ? (uint32_t)NJ : (tsize + NT * APV - 1) / (NT * APV);   // vectors per thread
    using V = typename Vec16<R>::V;
    V pre[PF];
    auto gaddr = [&](uint64_t base, uint32_t j) -> V * {
        return reinterpret_cast<V *>(psi + (base | g_t | tile_offset(j * NT * APV, pa)));
    };
    const uint32_t h_t = tl.grp(s_t * (uint32_t)sizeof(A));   // this thread's first vector
    auto lds_put = [&](uint32_t j, V v) { *tl.template at<V>(h_t, sw(j * NT * APV) * (uint32_t)sizeof(A)) = v * sc; };
    // Vectors of a generic tile beyond the prefetch depth: loaded in batches
    // through the prefetch registers once those are in LDS.
    auto load_rest = [&](uint64_t base) {
        for (uint32_t j0 = PF; j0 < nj; j0 += PF) {
#pragma unroll
            for (int i = 0; i < PF; ++i)
                if (j0 + i < nj) pre[i] = ld_nt(gaddr(base, j0 + i));
#pragma unroll
            for (int i = 0; i < PF; ++i)
                if (j0 + i < nj) lds_put(j0 + i, pre[i]);
        }
    };
    // Tiles are handed out in ascending order by a ticket counter (the state's,
    // advanced by ntiles + grid per pass: every workgroup draws until it gets
    // a ticket past the last tile), so a workgroup that runs faster than its
    // neighbour on the same CU takes more tiles.  Thread 0 draws the ticket
    // after next into an LDS slot; the loop-top barrier publishes it.
    if (threadIdx.x == 0) {
        next_slot[0] = atomicAdd(tickets, 1ull) - ticket0;
        // exactly one ticket past the last tile per workgroup
        next_slot[1] = next_slot[0] < ntiles ? atomicAdd(tickets, 1ull) - ticket0 : ntiles;
    }
    __syncthreads();
    uint64_t tileid = next_slot[0];
    uint64_t nxt = next_slot[1];
    if (tileid >= ntiles) return;   // whole workgroup
    // block operands of the pass -> LDS behind the tile (once per workgroup;
    // pool entries are 16-byte aligned and cl_len a multiple of 16 bytes)
    if constexpr (CL) {
        constexpr int EPV = 16 / sizeof(R);
        for (int i = threadIdx.x * EPV; i < pa.cl_len; i += NT * EPV)
            *reinterpret_cast<V *>(cst + i) = *reinterpret_cast<const V *>(pool + pa.cl_off + i);
    }
    uint64_t base = tile_base(tileid, pa);
    if (active) {
#pragma unroll
        for (int j = 0; j < PF; ++j)
            if ((uint32_t)j < nj) pre[j] = ld_nt(gaddr(base, j));
        if constexpr (EX > 0) {
            V ex[EX];
#pragma unroll
            for (int i = 0; i < EX; ++i) ex[i] = ld_nt(gaddr(base, PF + i));
#pragma unroll
            for (int j = 0; j < PF; ++j) lds_put(j, pre[j]);
#pragma unroll
            for (int i = 0; i < EX; ++i) lds_put(PF + i, ex[i]);
        } else {
#pragma unroll
            for (int j = 0; j < PF; ++j)
                if ((uint32_t)j < nj) lds_put(j, pre[j]);
            if constexpr (NJ == 0) load_rest(base);
        }
    }
    // Loop invariant: the tile `tileid` is in LDS (after the barrier).  The
    // next tile's loads are issued before this tile's stores (prefetch
    // registers before the blocks, the remaining vectors after them), so the
    // waits for them at the bottom of the loop leave the stores in flight.
    // On the last tile the loads re-read the current tile (in bounds, unused).
    int slot = 0;
    for (;;) {
        __syncthreads();
        if (slot) nxt = next_slot[slot & 1];
        // the ticket after next, read by every thread behind the next loop-top barrier
        if (threadIdx.x == 0 && nxt < ntiles) next_slot[(slot + 1) & 1] = atomicAdd(tickets, 1ull) - ticket0;
        const bool more = nxt < ntiles;   // uniform over the workgroup
        const uint64_t nbase = more ? tile_base(nxt, pa) : base;
        if (active) {
#pragma unroll
            for (int j = 0; j < PF; ++j)
                if ((uint32_t)j < nj) pre[j] = ld_nt(gaddr(nbase, j));
        }
        // ---- blocks ----
        for (int b = 0; b < pa.nblocks; ++b) {
            if (blocks[pa.block0 + b].kind == BK_SKIP) continue;   // folded into a group (uniform)
            apply_block<R, WIDE, CL, NT>(tl, T, blocks + pa.block0 + b, pool, base, cst, pa.cl_off);
            __syncthreads();
        }
        V ex[EX > 0 ? EX : 1];
        if constexpr (EX > 0) {
#pragma unroll
            for (int i = 0; i < EX; ++i) ex[i] = ld_nt(gaddr(nbase, PF + i));
        }
        // ---- store + FP64 norm partial ----
        double nacc = 0.0;
        auto norm_of = [](const V &v) -> double {
            if constexpr (F32) return (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
            else return v.x * v.x + v.y * v.y;
        };
        if constexpr (NJ > 0) {
            // every LDS read issued before the first store: one wait chain
            // instead of a read latency per stored vector
            V vals[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) vals[j] = *tl.template at<const V>(h_t, sw(j * NT * APV) * (uint32_t)sizeof(A));
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                st_nt(gaddr(base, j), vals[j]);
                nacc += norm_of(vals[j]);
            }
        } else if (active) {
            for (uint32_t j = 0; j < nj; ++j) {
                const V v = *tl.template at<const V>(h_t, sw(j * NT * APV) * (uint32_t)sizeof(A));
                st_nt(gaddr(base, j), v);
                nacc += norm_of(v);
            }
        }
        if (pa.want_norm) red[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)] = wave_sum_f64(nacc);
        __syncthreads();  // every read of this tile from LDS is done, every norm slot written
        // Thread 0 sums the slots after that barrier; they are written again
        // only in the next tile's store phase, behind the loop-top barrier
        // that wave 0 reaches after these reads.
        if (pa.want_norm && threadIdx.x == 0) {
            double s = 0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) s += red[w];
            partials[tileid] = s;   // one partial per tile: the reduction order does not depend on the schedule
        }
        if (!more) break;
        if (active) {
#pragma unroll
            for (int j = 0; j < PF; ++j)
                if ((uint32_t)j < nj) lds_put(j, pre[j]);
            if constexpr (EX > 0) {
#pragma unroll
                for (int i = 0; i < EX; ++i) lds_put(PF + i, ex[i]);
            } else if constexpr (NJ == 0) {
                load_rest(nbase);
            }
        }
        tileid = nxt;
        base = nbase;
        ++slot;
    }
}

// one workgroup: fixed-order FP64 sum of the partials; slot[0] = N, slot[1] = 1/sqrt(N).
// Each thread takes eight independent loads per round (partials i + u 1024,
// u = 0..7) and adds them pairwise in a fixed order: the loads overlap (one
// dependent load per step took 33 us for 2^17 partials) and the result does
// not depend on timing.
__global__ __launch_bounds__(1024) void k_norm_reduce(const double *__restrict__ parts, uint64_t n,
                                                      double *__restrict__ slots) {
    __shared__ double sh[1024];
    double s = 0;
    uint64_t i = threadIdx.x;
    for (; i + 7 * 1024 < n; i += 8 * 1024) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = parts[i + (uint64_t)u * 1024];
        s += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    }
    for (; i < n; i += 1024) s += parts[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        slots[0] = sh[0];
        slots[1] = sh[0] > 0 ? 1.0 / sqrt(sh[0]) : 1.0;
    }
}

// per-workgroup FP64 partial of sum |a|^2 over a contiguous chunk
template <typename A>
__global__ __launch_bounds__(256) void k_norm_parts(const A *__restrict__ psi, uint64_t namps, uint64_t chunk,
                                                    double *__restrict__ parts) {
    __shared__ double red[4];
    const uint64_t b0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t e = b0 + chunk < namps ? b0 + chunk : namps;
    double s = 0;
    for (uint64_t i = b0 + threadIdx.x; i < e; i += 256) {
        const A v = psi[i];
        s += (double)v.x * v.x + (double)v.y * v.y;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) parts[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// 2^13 / 2^14-amplitude complex64 tiles in 512 / 1024-thread workgroups
// (QS_TILE_BIG=0: 256 threads)
bool big_tiles_enabled() {
    static int v = -1;
    if (v < 0) {
        const char *e = getenv("QS_TILE_BIG");
        v = e ? atoi(e) != 0 : 1;
    }
    return v == 1;
}

template <typename R>
using TileKernel = void (*)(typename AmpOf<R>::A *, uint64_t, PassArgs, const BlockDev *, const R *, const double *,
                            double *, unsigned long long *, unsigned long long);

// Kernel variant for a pass: register footprint (wide), LDS-staged operands
// (cl) and, for the narrow variant, the compile-time vector count.
template <typename R>
TileKernel<R> pick_tile_kernel(bool wide, int t, bool cl, int &threads, bool &static_tile) {
    constexpr int APV = sizeof(R) == 4 ? 2 : 1;
    const int vpt = (1 << t) / (TT * APV);   // 16-byte vectors per thread
    threads = TT;
    static_tile = false;
    if (wide) return k_tile_pass<R, true, 0, false>;
    if constexpr (sizeof(R) == 4) {
        // unstaged 2^13 / 2^14 tiles: more threads per workgroup, 8 vectors each
        if (!cl && big_tiles_enabled()) {
            static_tile = t == 13 || t == 14;
            if (t == 13) {
                threads = 512;
                return k_tile_pass<R, false, 8, false, 512>;
            }
            if (t == 14) {
                threads = 1024;
                return k_tile_pass<R, false, 8, false, 1024>;
            }
        }
        if (cl && big_tiles_enabled() && t == 13) {
            threads = 512;
            return k_tile_pass<R, false, 8, true, 512>;
        }

    }
    if ((1 << t) == vpt * TT * APV) {
        if (cl) {
            if constexpr (sizeof(R) == 4) {
                if (vpt == 4) return k_tile_pass<R, false, 4, true>;
                if (vpt == 8) return k_tile_pass<R, false, 8, true>;
                if (vpt == 16) return k_tile_pass<R, false, 16, true>;
            } else {
                if (vpt == 8) return k_tile_pass<R, false, 8, true>;
                if (vpt == 16) return k_tile_pass<R, false, 16, true>;
            }
        }
        static_tile = vpt == 1 || vpt == 2 || vpt == 4 || vpt == 8 || vpt == 16;
        if (vpt == 1) return k_tile_pass<R, false, 1, false>;
        if (vpt == 2) return k_tile_pass<R, false, 2, false>;
        if (vpt == 4) return k_tile_pass<R, false, 4, false>;
        if (vpt == 8) return k_tile_pass<R, false, 8, false>;
        if (vpt == 16) return k_tile_pass<R, false, 16, false>;
    }
    return k_tile_pass<R, false, 0, false>;
}

// LDS bytes a pass may use for staged operands: what is left of the CU's LDS
// share per workgroup at the occupancy the staged variant targets (complex64
// 2^11: 4, 2^12: 3, 2^13: 2 workgroups per CU; complex128 2^11, 2^12: 2),
// minus the tile and a margin that holds the norm slots.  0 = no staged
// variant for this tile.
size_t lds_operand_budget(int t, qs_dtype dt) {
    constexpr size_t kLds = 160 * 1024, kMargin = 512;
    int wgs = 0;
    // complex64 2^13 tiles: 2 workgroups per CU (512 threads, or 256 with
    // QS_TILE_BIG=0); 2^14 tiles are not staged (a staged 1024-thread variant
    // spills registers at 4 waves per SIMD, and a reload waits for the prefetch)
    if (dt == QS_C64) wgs = t == 11 ? 4 : t == 12 ? 3 : t == 13 ? 2 : 0;
    else wgs = t == 11 || t == 12 ? 2 : 0;   // complex128 variants run 2 workgroups per CU
    if (!wgs) return 0;
    const size_t share = (kLds / wgs) & ~(size_t)1023, tile = (size_t)(dt == QS_C64 ? 8 : 16) << t;
    return share > tile + kMargin ? share - tile - kMargin : 0;
}

// Staged complex64 passes in 512-thread workgroups apply 5-qubit blocks with
// the real embedding (the three-product form would spill there).
bool big_staged(int t, qs_dtype dt) { return dt == QS_C64 && t == 13 && big_tiles_enabled(); }

// Raise a kernel's dynamic LDS limit once per (kernel, size).
// Per-kernel caches of launch attributes, shared by every state: one lock
// (a lookup per pass launch is negligible beside the pass).
std::mutex &kernel_cache_lock() {
    static std::mutex m;
    return m;
}

void set_lds_limit(const void *fn, size_t bytes) {
    static std::vector<std::pair<const void *, size_t>> done;
    std::lock_guard<std::mutex> lock(kernel_cache_lock());
    for (auto &d : done)
        if (d.first == fn) {
            if (bytes > d.second) {
                (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
                d.second = bytes;
            }
            return;
        }
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    done.emplace_back(fn, bytes);
}

bool mfma_enabled() {
    static int v = -1;
    if (v < 0) {
        const char *e = getenv("QS_TILE_MFMA");
        v = e ? atoi(e) != 0 : 1;
    }
    return v == 1;
}

// Host-side A-operand swizzle of a complex64 block: entry (R, kk) of the
// real embedding [[Ur, -Ui], [Ui, Ur]] for M-tile mt, step s and lane l is row
// R = 16 mt + l % 16 and input (row 4 (s / 2) + l / 16, part s % 2).
// Layout [mt][s][lane] for mfma_block, [mt][s / 4][lane][s % 4] for
// mfma_block_lds (16-byte LDS reads).
template <typename R>
void swizzle_mfma(const std::vector<cd> &U, int k, bool lds_layout, std::vector<R> &out) {
    const int D = 1 << k, MT = 2 * D / 16, S = 2 * D / 4;
    const size_t o0 = out.size();
    out.resize(o0 + (size_t)MT * S * 64);
    for (int mt = 0; mt < MT; ++mt)
        for (int s = 0; s < S; ++s)
            for (int lane = 0; lane < 64; ++lane) {
                const int i = lane % 16, g = lane / 16;
                const int row = 16 * mt + i;
                const int r = 4 * (s / 2) + g, p = s % 2;
                const int rr = row % D, ro = row / D;
                const cd u = U[(size_t)rr * D + r];
                double v;
                if (ro == 0) v = p == 0 ? u.real() : -u.imag();
                else v = p == 0 ? u.imag() : u.real();
                const size_t idx = lds_layout ? (((size_t)mt * (S / 4) + s / 4) * 64 + lane) * 4 + s % 4
                                              : ((size_t)mt * S + s) * 64 + lane;
                out[o0 + idx] = (R)v;
            }
}

// Host-side operands of mfma3m_block_lds: A_g for g = Ur, Ui, Ur + Ui, entry
// A_g[16 m + l % 16][4 s + l / 16] for M-tile m, step s, lane l, stored as
// [g][m][s / 4][l][s % 4].
template <typename R>
void swizzle_mfma3m(const std::vector<cd> &U, int k, std::vector<R> &out) {
    const int D = 1 << k, MT = D / 16, S = D / 4, S4 = S / 4;
    const size_t o0 = out.size();
    out.resize(o0 + (size_t)3 * MT * S * 64);
    for (int g = 0; g < 3; ++g)
        for (int m = 0; m < MT; ++m)
            for (int s = 0; s < S; ++s)
                for (int lane = 0; lane < 64; ++lane) {
                    const cd u = U[(size_t)(16 * m + lane % 16) * D + (4 * s + lane / 16)];
                    const double v = g == 0 ? u.real() : g == 1 ? u.imag() : u.real() + u.imag();
                    out[o0 + ((((size_t)g * MT + m) * S4 + s / 4) * 64 + lane) * 4 + s % 4] = (R)v;
                }
}

// Structure of a block matrix: monomial (exactly one entry per column with
// |u| > kZeroTol, entries below it being rounding residue of exact zeros of
// the gate product) or dense.
constexpr double kZeroTol = 1e-14;

bool monomial(const std::vector<cd> &U, int D, std::vector<int> &dest) {
    dest.assign(D, -1);
    for (int c = 0; c < D; ++c)
        for (int r = 0; r < D; ++r)
            if (std::abs(U[(size_t)r * D + c]) > kZeroTol) {
                if (dest[c] >= 0) return false;
                dest[c] = r;
            }
    for (int c = 0; c < D; ++c)
        if (dest[c] < 0) return false;
    return true;
}

// every nonzero entry of the monomial U (column c's in row dest[c]) equals 1
// (within kZeroTol: products of CNOT, X and SWAP gates are exact)
bool unit_entries(const std::vector<cd> &U, int D, const std::vector<int> &dest) {
    for (int c = 0; c < D; ++c)
        if (std::abs(U[(size_t)dest[c] * D + c] - cd(1.0, 0.0)) > kZeroTol) return false;
    return true;
}

bool structured_enabled() {
    static int v = -1;
    if (v < 0) {
        const char *e = getenv("QS_TILE_STRUCTURED");
        v = e ? atoi(e) != 0 : 1;
    }
    return v == 1;
}

// Permuted block-diagonal structure: the bipartite graph of U's nonzero
// entries (rows against columns) splits into connected components, each with
// as many rows as columns (U is unitary).  The components are packed (largest
// first, first fit) into 2^(k-s) classes of exactly 2^s rows and 2^s
// columns, with the smallest s that packs; U then acts as 2^(k-s)
// independent 2^s x 2^s matrices between the classes' column and row lists.
// src lists the columns class by class, dst the rows in the same order.
bool bdiag_split(const std::vector<cd> &U, int k, int &s, std::vector<int> &src, std::vector<int> &dst) {
    const int D = 1 << k;
    std::vector<int> parent(2 * D);
    for (int i = 0; i < 2 * D; ++i) parent[i] = i;
    auto find = [&](int x) {
        while (parent[x] != x) x = parent[x] = parent[parent[x]];
        return x;
    };
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c)
            if (std::abs(U[(size_t)r * D + c]) > kZeroTol) parent[find(r)] = find(D + c);
    std::vector<std::vector<int>> rows(2 * D), cols(2 * D);
    for (int r = 0; r < D; ++r) rows[find(r)].push_back(r);
    for (int c = 0; c < D; ++c) cols[find(D + c)].push_back(c);
    std::vector<int> comps;
    size_t widest = 1;
    for (int i = 0; i < 2 * D; ++i) {
        if (rows[i].size() != cols[i].size()) return false;
        if (!rows[i].empty()) {
            comps.push_back(i);
            widest = std::max(widest, rows[i].size());
        }
    }
    std::stable_sort(comps.begin(), comps.end(), [&](int a, int b) { return rows[a].size() > rows[b].size(); });
    for (s = 0; (size_t)1 << s < widest; ++s) {}
    for (; s <= k; ++s) {
        const int DS = 1 << s, NC = D / DS;
        std::vector<std::vector<int>> br(NC), bc(NC);
        bool ok = true;
        for (int cp : comps) {
            int j = 0;
            while (j < NC && br[j].size() + rows[cp].size() > (size_t)DS) ++j;
            if (j == NC) {
                ok = false;
                break;
            }
            br[j].insert(br[j].end(), rows[cp].begin(), rows[cp].end());
            bc[j].insert(bc[j].end(), cols[cp].begin(), cols[cp].end());
        }
        if (!ok) continue;
        src.clear();
        dst.clear();
        for (int j = 0; j < NC; ++j) {
            src.insert(src.end(), bc[j].begin(), bc[j].end());
            dst.insert(dst.end(), br[j].begin(), br[j].end());
        }
        return true;
    }
    return false;
}

// Class widths the tile kernel has permuted block-diagonal code for:
// 0 <= s < k, k = 3 or 4 (s = 0 is used for 4-qubit monomial blocks only) (a lane holds the whole group: 2^5 amplitudes would
// not fit beside the prefetched tile); QS_TILE_BDIAG = 0 turns the kind off,
// a value g > 1 keeps it to s <= k - g.
int bdiag_gap() {
    static int v = -1;
    if (v < 0) {
        const char *e = getenv("QS_TILE_BDIAG");
        v = e ? std::max(0, atoi(e)) : 1;
    }
    return v;
}

bool bdiag_supported(int k, int s, qs_dtype dt) {
    const int gap = bdiag_gap();
    (void)dt;
    return gap > 0 && k >= 3 && k <= 4 && s >= 0 && s <= k - gap;
}

// QS_TILE_BDMFMA=0: permuted block-diagonal blocks stay on the vector ALU in
// staged passes
bool bdmfma_enabled() {
    static int v = -1;
    if (v < 0) {
        const char *e = getenv("QS_TILE_BDMFMA");
        v = e ? atoi(e) != 0 : 1;
    }
    return v == 1;
}

bool staged_enabled() {
    static int v = -1;
    if (v < 0) {
        const char *e = getenv("QS_TILE_STAGED");
        v = e ? atoi(e) != 0 : 1;
    }
    return v == 1;
}

// Pauli-rotation record: X and Z masks over tile positions, the Z mask of the
// qubits outside the tile (64-bit, two entries), then c and d.
template <typename R>
void push_pauli(const HBlock &blk, BlockDev &d, const HPass &ps, std::vector<R> &pool);

// A pool entry holding a 32-bit pattern (read back by bit-cast on the device).
template <typename R>
R pool_entry(uint32_t bits) {
    R v;
    if constexpr (sizeof(R) == 4) {
        std::memcpy(&v, &bits, 4);
    } else {
        const uint64_t b64 = bits;
        std::memcpy(&v, &b64, 8);
    }
    return v;
}

// Coefficient form of a rotation for the device (rot_pair): 1 when c is real
// and d imaginary (a Pauli exponential whose Clifford part cancels exactly),
// 2 when both are real, else 0.  Parts below 1e-15 are rounding residue of
// exact zeros (the Clifford phase is simulated in FP64).
int pauli_mode(const HBlock &b) {
    const double tol = 1e-15;
    if (std::abs(b.pc.imag()) > tol) return 0;
    if (std::abs(b.pd.real()) <= tol) return 1;
    if (std::abs(b.pd.imag()) <= tol) return 2;
    return 0;
}

bool pauli_groups_enabled() {
    static int v = -1;
    if (v < 0) {
        const char *e = getenv("QS_PAULI_GROUP");
        v = e ? atoi(e) != 0 : 1;
    }
    return v == 1;
}

// Rotations from block b on (within the pass ending at `end`) that form one
// group: at most cap (3), all with X parts that are nonzero and linearly
// independent over GF(2).
int pauli_group_size(const std::vector<HBlock> &blocks, int64_t b, int64_t end, int cap) {
    if (!pauli_groups_enabled()) return 1;
    std::vector<uint64_t> red;   // echelon basis, each with a distinct leading bit
    int m = 0;
    for (int64_t i = b; i < end && m < cap; ++i) {
        const HBlock &B = blocks[i];
        if (!B.pauli || B.px == 0) break;
        uint64_t r = B.px;
        for (uint64_t v : red)
            if ((r >> (63 - __builtin_clzll(v))) & 1) r ^= v;
        if (r == 0) break;
        red.push_back(r);
        std::sort(red.begin(), red.end(), [](uint64_t a, uint64_t c) { return a > c; });
        ++m;
    }
    return m;
}

template <typename R>
void push_pauli_group(const HBlock *bl, int m, BlockDev &d, const HPass &ps, std::vector<R> &pool) {
    auto to_tile = [&](uint64_t g, uint64_t *outside) {
        uint32_t t = 0;
        uint64_t tmask = 0;
        for (size_t j = 0; j < ps.tile.size(); ++j) {
            tmask |= 1ull << ps.tile[j];
            if ((g >> ps.tile[j]) & 1) t |= 1u << j;
        }
        if (outside) *outside = g & ~tmask;
        return t;
    };
    uint32_t xt[4], zt[4];
    uint64_t zo[4];
    for (int i = 0; i < m; ++i) {
        uint64_t xo = 0;
        xt[i] = to_tile(bl[i].px, &xo);
        if (xo) throw std::logic_error("Pauli block's X part outside its tile");
        zt[i] = to_tile(bl[i].pz, &zo[i]);
    }
    // pivots: leading bits of an echelon form (each reduced vector is zero at
    // the earlier pivots), so only 0 in the span is zero at every pivot
    std::vector<uint32_t> red;
    std::vector<int> piv;
    for (int i = 0; i < m; ++i) {
        uint32_t r = xt[i];
        for (size_t l = 0; l < red.size(); ++l)
            if ((r >> piv[l]) & 1) r ^= red[l];
        if (r == 0) throw std::logic_error("Pauli group X parts not independent");
        red.push_back(r);
        piv.push_back(31 - __builtin_clz(r));
    }
    std::sort(piv.begin(), piv.end());
    d.kind = BK_PAULIG;
    d.k = m;
    d.mat_off = (int32_t)pool.size();
    uint32_t modes = 0;
    for (int i = 0; i < m; ++i) modes |= (uint32_t)pauli_mode(bl[i]) << (2 * i);
    for (int j = 0; j < 3; ++j) pool.push_back(pool_entry<R>(j < m ? (uint32_t)piv[j] : 0u));
    pool.push_back(pool_entry<R>(modes));
    for (int c = 0; c < 16; ++c) {
        uint32_t v = 0;
        for (int j = 0; j < m; ++j)
            if ((c >> j) & 1) v ^= xt[j];
        pool.push_back(pool_entry<R>(c < (1 << m) ? sw(v) * 2 * (uint32_t)sizeof(R) : 0u));
    }
    for (int i = 0; i < m; ++i) {
        uint32_t pm = 0;
        for (int j = 0; j < m; ++j)
            if (__builtin_popcount(xt[j] & zt[i]) & 1) pm |= 1u << j;
        pool.push_back(pool_entry<R>(zt[i]));
        pool.push_back(pool_entry<R>((uint32_t)zo[i]));
        pool.push_back(pool_entry<R>((uint32_t)(zo[i] >> 32)));
        pool.push_back(pool_entry<R>(pm));
        pool.push_back((R)bl[i].pc.real());
        pool.push_back((R)bl[i].pc.imag());
        pool.push_back((R)bl[i].pd.real());
        pool.push_back((R)bl[i].pd.imag());
    }
}

template <typename R>
void push_pauli(const HBlock &blk, BlockDev &d, const HPass &ps, std::vector<R> &pool) {
    uint32_t xt = 0, zt = 0;
    uint64_t tmask = 0;
    for (size_t j = 0; j < ps.tile.size(); ++j) {
        const int q = ps.tile[j];
        tmask |= 1ull << q;
        if ((blk.px >> q) & 1) xt |= 1u << j;
        if ((blk.pz >> q) & 1) zt |= 1u << j;
    }
    if ((blk.px & ~tmask) != 0) throw std::logic_error("Pauli block's X part outside its tile");
    const uint64_t zo = blk.pz & ~tmask;
    d.kind = BK_PAULI;
    d.k = __builtin_popcount(xt);
    d.sub = pauli_mode(blk);
    d.mat_off = (int32_t)pool.size();
    pool.push_back(pool_entry<R>(xt));
    pool.push_back(pool_entry<R>(zt));
    pool.push_back(pool_entry<R>((uint32_t)zo));
    pool.push_back(pool_entry<R>((uint32_t)(zo >> 32)));
    pool.push_back((R)blk.pc.real());
    pool.push_back((R)blk.pc.imag());
    pool.push_back((R)blk.pd.real());
    pool.push_back((R)blk.pd.imag());
}

template <typename R>
void push_block(const HBlock &blk, BlockDev &d, int t, qs_dtype dt, bool lds, std::vector<R> &pool, bool &wide) {
    const int D = 1 << d.k;
    std::vector<int> dest;
    const int kind = block_kind(blk, t, dt, &dest, lds);
    if (kind == BK_BDMFMA) {
        int sub = 0;
        std::vector<int> src, dst;
        bdiag_split(blk.U, d.k, sub, src, dst);
        d.kind = BK_BDMFMA;
        d.sub = sub;
        d.mat_off = (int32_t)pool.size();
        auto off = [&](int c) {
            uint32_t o = 0;
            for (int j = 0; j < d.k; ++j)
                if ((c >> j) & 1) o |= 1u << d.pos[j];
            return sw(o) * 2 * (uint32_t)sizeof(R);
        };
        const int DS = 1 << sub;
        if (sub < 3) {
            // classes of 2 or 4, see class_mfma_block: source and destination
            // byte offsets class by class, then the classes' real forms M
            // (rows and columns ordered (member, re/im)) as [lane][register]:
            // product n = (class, row tile, step) is register n / 16 of lane
            // quad n % 16, whose lane i holds row i of the row tile
            for (int i = 0; i < D; ++i) pool.push_back(pool_entry<R>(off(src[i])));
            for (int i = 0; i < D; ++i) pool.push_back(pool_entry<R>(off(dst[i])));
            const int K2 = 2 * DS, RT = K2 / 4, NREG = DS;
            std::vector<R> am((size_t)64 * NREG, (R)0);
            for (int c = 0; c < D / DS; ++c)
                for (int rt = 0; rt < RT; ++rt)
                    for (int st = 0; st < K2; ++st) {
                        const int n = (c * RT + rt) * K2 + st, q = n % 16, u = n / 16;
                        for (int i = 0; i < 4; ++i) {
                            const int row = 4 * rt + i;
                            const int r = row / 2, rp = row % 2, cm = st / 2, cp = st % 2;
                            const cd e = blk.U[(size_t)dst[c * DS + r] * D + src[c * DS + cm]];
                            const double v = rp == 0 ? (cp == 0 ? e.real() : -e.imag())
                                                     : (cp == 0 ? e.imag() : e.real());
                            am[(size_t)(4 * q + i) * NREG + u] = (R)v;
                        }
                    }
            pool.insert(pool.end(), am.begin(), am.end());
            while (pool.size() % 4) pool.push_back((R)0);  // 16-byte aligned entries
            return;
        }
        // classes of 8: packs of 8 class members, see bdiag_mfma_block: A of
        // the pack's 16x16 real form as [lane][step], column offsets (members
        // 0,2,4,6 then 1,3,5,7), row offsets
        for (int p0 = 0; p0 < D; p0 += 8) {
            for (int lane = 0; lane < 64; ++lane)
                for (int st = 0; st < 4; ++st) {
                    const int i = lane % 16, kk = 4 * st + lane / 16;
                    const int r = i / 2, rp = i % 2, c = kk / 2, cp = kk % 2;
                    // zero between classes (entries there are rounding residue)
                    const bool same = (p0 + r) / DS == (p0 + c) / DS;
                    const cd u = same ? blk.U[(size_t)dst[p0 + r] * D + src[p0 + c]] : cd(0.0, 0.0);
                    const double v = rp == 0 ? (cp == 0 ? u.real() : -u.imag()) : (cp == 0 ? u.imag() : u.real());
                    pool.push_back((R)v);
                }
            for (int h = 0; h < 2; ++h)
                for (int st = 0; st < 4; ++st) pool.push_back(pool_entry<R>(off(src[p0 + 2 * st + h])));
            for (int r = 0; r < 8; ++r) pool.push_back(pool_entry<R>(off(dst[p0 + r])));
        }
    } else if (kind == BK_BDIAG) {
        // record: 2^k swizzled source offsets (class by class), 2^k swizzled
        // destination offsets, then the classes' 2^s x 2^s matrices
        int sub = 0;
        std::vector<int> src, dst;
        bdiag_split(blk.U, d.k, sub, src, dst);
        d.kind = BK_BDIAG;
        d.sub = sub;
        d.mat_off = (int32_t)pool.size();
        // offsets: LDS byte offsets within the tile, stored as bit patterns
        auto deposit = [&](int c) {
            uint32_t o = 0;
            for (int j = 0; j < d.k; ++j)
                if ((c >> j) & 1) o |= 1u << d.pos[j];
            return pool_entry<R>(sw(o) * 2 * (uint32_t)sizeof(R));
        };
        for (int i = 0; i < D; ++i) pool.push_back(deposit(src[i]));
        for (int i = 0; i < D; ++i) pool.push_back(deposit(dst[i]));
        const int DS = 1 << sub;
        for (int j = 0; j < D / DS; ++j)
            for (int r = 0; r < DS; ++r)
                for (int c = 0; c < DS; ++c) {
                    const cd u = blk.U[(size_t)dst[j * DS + r] * D + src[j * DS + c]];
                    pool.push_back((R)u.real());
                    pool.push_back((R)u.imag());
                }
    } else if (kind == BK_PERM) {
        // record: 2^k swizzled source byte offsets, then the destination of each
        d.kind = BK_PERM;
        d.mat_off = (int32_t)pool.size();
        auto deposit = [&](int c) {
            uint32_t o = 0;
            for (int j = 0; j < d.k; ++j)
                if ((c >> j) & 1) o |= 1u << d.pos[j];
            return pool_entry<R>(sw(o) * 2 * (uint32_t)sizeof(R));
        };
        for (int c = 0; c < D; ++c) pool.push_back(deposit(c));
        for (int c = 0; c < D; ++c) pool.push_back(deposit(dest[c]));
    } else if (kind == BK_MONO) {
        d.kind = BK_MONO;
        d.mat_off = (int32_t)pool.size();
        for (int c = 0; c < D; ++c) {
            const cd u = blk.U[(size_t)dest[c] * D + c];
            uint32_t o = 0;
            for (int j = 0; j < d.k; ++j)
                if ((dest[c] >> j) & 1) o |= 1u << d.pos[j];
            pool.push_back((R)u.real());
            pool.push_back((R)u.imag());
            pool.push_back(pool_entry<R>(sw(o) * 2 * (uint32_t)sizeof(R)));   // LDS byte offset
            pool.push_back((R)0);
        }
    } else if (kind == BK_MFMA) {
        d.kind = BK_MFMA;
        d.mat_off = (int32_t)pool.size();
        if (lds && d.k >= 4 && !(d.k == 5 && big_staged(t, dt))) swizzle_mfma3m<R>(blk.U, d.k, pool);
        else swizzle_mfma<R>(blk.U, d.k, lds, pool);
        if (!lds && (dt == QS_C128 || d.k == 6)) wide = true;
    } else {
        d.kind = BK_DENSE;
        d.mat_off = (int32_t)pool.size();
        for (int i = 0; i < D * D; ++i) {
            pool.push_back((R)blk.U[i].real());
            pool.push_back((R)blk.U[i].imag());
        }
        if (d.k > 3) wide = true;
    }
    while (pool.size() % 4) pool.push_back((R)0);  // 16-byte aligned entries
}

// Class width 2^s of a permuted block-diagonal block.
size_t bdiag_width(const HBlock &b) {
    int sub = 0;
    std::vector<int> src, dst;
    bdiag_split(b.U, (int)b.qubits.size(), sub, src, dst);
    return (size_t)1 << sub;
}

// Real flops per amplitude of one block as the tile kernel applies it.
double block_flops_per_amp(const BlockDev &d) {
    if (d.kind == BK_PAULI) return 16.0;
    if (d.kind == BK_PAULIG) return 16.0 * d.k;
    if (d.kind == BK_SKIP) return 0.0;
    if (d.kind == BK_MONO) return 6.0;
    if (d.kind == BK_PERM) return 0.0;
    if (d.kind == BK_BDIAG || d.kind == BK_BDMFMA) return 8.0 * (1 << d.sub);
    return 8.0 * (1 << d.k);
}

// Pool bytes the blocks of a pass take when staged (the kinds of a staged pass).
size_t pass_operand_bytes(const std::vector<HBlock> &blocks, const HPass &ps, qs_dtype dt) {
    size_t b = 0;
    for (int64_t i = ps.block0; i < ps.block0 + ps.nblocks; ++i) {
        const HBlock &blk = blocks[i];
        const int k = (int)blk.qubits.size(), D = 1 << k;
        const int kind = block_kind(blk, ps.t, dt, nullptr, true);
        size_t e = kind == BK_PAULI   ? 52   // bound: a group record (pivots, 16 offsets, 4 x 8)
                   : kind == BK_BDMFMA  ? (bdiag_width(blk) == 8 ? (size_t)(D / 8) * kBdPackFloats
                                                                  : 2 * (size_t)D + 64 * bdiag_width(blk))
                   : kind == BK_MONO    ? 4 * (size_t)D
                   : kind == BK_PERM    ? 2 * (size_t)D
                   : kind == BK_MFMA  ? (k == 4 || (k == 5 && !big_staged(ps.t, dt)) ? (size_t)3 * D * D
                                                                                      : (size_t)4 * D * D)
                   : kind == BK_BDIAG ? 2 * (size_t)D + 2 * (size_t)D * bdiag_width(blk)
                                      : 2 * (size_t)D * D;
        e = (e + 3) / 4 * 4;
        b += e * (dt == QS_C64 ? 4 : 8);
    }
    return b;
}

// Workgroups of a tile kernel resident at once on the current device.
uint64_t resident_groups(const void *fn, int threads, size_t lds) {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    int per_cu = 0;
    set_lds_limit(fn, lds);
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    return (uint64_t)per_cu * (uint64_t)cus;
}

// A variant whose tile is the start of its dynamic LDS forms tile addresses
// with OR and XOR, which needs the tile at LDS address 0 (the dynamic region
// declares 128 KiB alignment): such a kernel must declare no static LDS.
// Checked once per kernel from its code object's attributes.
bool dynamic_tile_at_zero(const void *fn) {
    static std::vector<std::pair<const void *, bool>> seen;
    std::lock_guard<std::mutex> lock(kernel_cache_lock());
    for (auto &e : seen)
        if (e.first == fn) return e.second;
    hipFuncAttributes attr{};
    const bool ok = hipFuncGetAttributes(&attr, fn) == hipSuccess && attr.sharedSizeBytes == 0;
    seen.emplace_back(fn, ok);
    return ok;
}

}  // namespace

int block_kind(const HBlock &b, int t, qs_dtype dt, std::vector<int> *dest, bool lds) {
    if (b.pauli) return BK_PAULI;
    const int k = (int)b.qubits.size();
    std::vector<int> tmp;
    // 4-qubit monomial blocks go through the class path with classes of one
    // (one lane per group, wave-uniform records), or as a pure permutation
    // when every entry is 1 (CNOT ladders: no arithmetic at all); other
    // widths keep the monomial path
    if (structured_enabled() && monomial(b.U, 1 << k, dest ? *dest : tmp)) {
        if (k != 4 || !bdiag_supported(4, 0, dt)) return BK_MONO;
        return unit_entries(b.U, 1 << k, dest ? *dest : tmp) ? BK_PERM : BK_BDIAG;
    }
    // permuted block-diagonal: 2^s complex multiply-adds per amplitude on the
    // vector ALU instead of a dense product
    int sub = 0;
    std::vector<int> src, dst;
    if (structured_enabled() && bdiag_gap() > 0 && k >= 3 && bdiag_split(b.U, k, sub, src, dst) &&
        bdiag_supported(k, sub, dt)) {
        // complex64 4-qubit blocks in staged passes: classes of 8 as 16x16 real
        // products (32 multiply-adds per amplitude on the vector ALU), classes
        // of 2 and 4 as the 16-block 4x4 product (8 and 16 there) on MFMA
        if (lds && dt == QS_C64 && mfma_enabled() && bdmfma_enabled() && t - k >= 4 && k == 4 && sub >= 1)
            return BK_BDMFMA;
        return BK_BDIAG;
    }
    // complex64: MFMA for k = 4, 5 (k = 3 too when staged) and, unstaged, 6;
    // complex128: FP64 MFMA for k = 3..5 when staged and k = 4, 5 unstaged.
    // Unstaged complex128 and k = 6 blocks run in the wide kernel variant.
    // A staged pass never holds a 6-qubit block (its operands exceed the LDS
    // left beside the tile): asked for a staged pass, k = 6 reports dense.
    if (t - k >= 4 && mfma_enabled()) {
        if (dt == QS_C64 && (k == 4 || k == 5 || (lds && k == 3) || (!lds && k == 6))) return BK_MFMA;
        if (dt == QS_C128 && ((lds && k >= 3 && k <= 5) || (!lds && (k == 4 || k == 5)))) return BK_MFMA;
    }
    return BK_DENSE;
}

int bdiag_log_width(const HBlock &b) {
    int sub = 0;
    std::vector<int> src, dst;
    return bdiag_split(b.U, (int)b.qubits.size(), sub, src, dst) ? sub : (int)b.qubits.size();
}

bool pass_staged(const std::vector<HBlock> &blocks, const HPass &ps, qs_dtype dt) {
    // stage the pass's operands in LDS when they fit and the pass has blocks
    // that read per-lane operands (MFMA, classes of 8 on MFMA, wide monomial).
    // Classes of 2 and 4 go to the matrix cores only in passes staged for
    // those: on their own they run faster in the unstaged variant, whose
    // prefetch covers the whole next tile.
    if (!staged_enabled()) return false;
    const size_t budget = lds_operand_budget(ps.t, dt);
    if (!budget) return false;
    bool per_lane = false, dense_wide = false;
    for (int64_t b = ps.block0; b < ps.block0 + ps.nblocks; ++b) {
        const int k = (int)blocks[b].qubits.size();
        const int kind = block_kind(blocks[b], ps.t, dt, nullptr, true);
        per_lane |= kind == BK_MFMA || (kind == BK_BDMFMA && bdiag_width(blocks[b]) == 8) || (kind == BK_MONO && k >= 4);
        dense_wide |= kind == BK_DENSE && k > 3;
    }
    return per_lane && !dense_wide && pass_operand_bytes(blocks, ps, dt) <= budget;
}

namespace {
qs_status plan_upload_impl(qs_plan_s &p, qs_dtype dt, bool stage_lds);
}  // namespace

// Host invariants of the records (a rotation's X part inside its tile, a
// group's independent X parts) throw; no exception leaves through the ABI.
qs_status plan_upload(qs_plan_s &p, qs_dtype dt, bool stage_lds) {
    try {
        return plan_upload_impl(p, dt, stage_lds);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed while uploading a plan");
        return QS_ENOMEM;
    } catch (const std::exception &e) {
        set_error("plan upload: %s", e.what());
        return QS_EINVAL;
    }
}

namespace {
qs_status plan_upload_impl(qs_plan_s &p, qs_dtype dt, bool stage_lds) {
    const int di = dt == QS_C64 ? 0 : 1;
    if (p.dev_ready[di]) return QS_OK;
    std::vector<BlockDev> hb(p.blocks.size());
    std::vector<float> pool32;
    std::vector<double> pool64;
    p.pass_wide[di].assign(p.passes.size(), 0);
    p.pass_cl_off[di].assign(p.passes.size(), 0);
    p.pass_cl_len[di].assign(p.passes.size(), 0);
    for (size_t pi = 0; pi < p.passes.size(); ++pi) {
        const HPass &ps = p.passes[pi];
        bool wide = false;
        const bool lds = stage_lds && pass_staged(p.blocks, ps, dt);
        const size_t pool0 = dt == QS_C64 ? pool32.size() : pool64.size();
        for (int64_t b = ps.block0; b < ps.block0 + ps.nblocks; ++b) {
            const HBlock &blk = p.blocks[b];
            BlockDev &d = hb[b];
            std::memset(&d, 0, sizeof d);
            if (blk.pauli) {
                // consecutive rotations with independent X parts: one group record
                // (single-state kernel only: plans uploaded for the batch
                // kernel, stage_lds false, keep one record per rotation)
                int m = stage_lds ? pauli_group_size(p.blocks, b, ps.block0 + ps.nblocks, 3) : 1;
                if (m >= 2) {
                    if (dt == QS_C64) push_pauli_group<float>(&p.blocks[b], m, d, ps, pool32);
                    else push_pauli_group<double>(&p.blocks[b], m, d, ps, pool64);
                    for (int j = 1; j < m; ++j) {
                        std::memset(&hb[b + j], 0, sizeof(BlockDev));
                        hb[b + j].kind = BK_SKIP;
                    }
                    b += m - 1;
                } else if (dt == QS_C64) {
                    push_pauli<float>(blk, d, ps, pool32);
                } else {
                    push_pauli<double>(blk, d, ps, pool64);
                }
                continue;
            }
            d.k = (int)blk.qubits.size();
            QS_CHECK(d.k >= 1 && d.k <= (dt == QS_C64 ? kMaxK : kMaxK128), QS_EUNSUPPORTED,
                     "block width %d unsupported for this dtype", d.k);
            for (int j = 0; j < d.k; ++j)
                d.pos[j] = (int)(std::find(ps.tile.begin(), ps.tile.end(), blk.qubits[j]) - ps.tile.begin());
            if (dt == QS_C64) push_block<float>(blk, d, ps.t, dt, lds, pool32, wide);
            else push_block<double>(blk, d, ps.t, dt, lds, pool64, wide);
        }
        p.pass_wide[di][pi] = wide ? 1 : 0;
        if (lds) {
            const size_t pool1 = dt == QS_C64 ? pool32.size() : pool64.size();
            p.pass_cl_off[di][pi] = (int32_t)pool0;
            p.pass_cl_len[di][pi] = (int32_t)(pool1 - pool0);
        }
    }
    p.h_blocks[di] = hb;
    const size_t bbytes = std::max<size_t>(1, hb.size()) * sizeof(BlockDev);
    QS_HIP(hipMalloc(&p.d_blocks[di], bbytes));
    if (!hb.empty()) QS_HIP(hipMemcpy(p.d_blocks[di], hb.data(), hb.size() * sizeof(BlockDev), hipMemcpyHostToDevice));
    const size_t pbytes = dt == QS_C64 ? pool32.size() * sizeof(float) : pool64.size() * sizeof(double);
    QS_HIP(hipMalloc(&p.d_pool[di], std::max<size_t>(pbytes, 16)));
    if (pbytes)
        QS_HIP(hipMemcpy(p.d_pool[di], dt == QS_C64 ? (const void *)pool32.data() : (const void *)pool64.data(), pbytes,
                         hipMemcpyHostToDevice));
    p.dev_ready[di] = 1;
    return QS_OK;
}
}  // namespace

qs_status ensure_partials(qs_state_s &s, size_t count) {
    if (s.partials_cap >= count) return QS_OK;
    if (s.d_partials) {
        QS_HIP(hipStreamSynchronize(s.stream));
        QS_HIP(hipFree(s.d_partials));
        s.d_partials = nullptr;
        s.partials_cap = 0;
    }
    QS_HIP(hipMalloc(&s.d_partials, count * sizeof(double)));
    s.partials_cap = count;
    return QS_OK;
}

qs_status launch_pass(qs_state_s &s, const qs_plan_s &p, const HPass &ps, int64_t pass_index, bool scale_in,
                      bool want_norm, uint64_t *nparts) {
    const int di = s.dtype == QS_C64 ? 0 : 1;
    PassArgs pa;
    std::memset(&pa, 0, sizeof pa);
    pa.t = ps.t;
    pa.c = ps.c;
    pa.nblocks = (int32_t)ps.nblocks;
    pa.block0 = (int32_t)ps.block0;
    for (int j = 0; j < ps.t - ps.c; ++j) pa.hi[j] = ps.tile[ps.c + j];
    pa.apply_scale = scale_in ? 1 : 0;
    pa.want_norm = want_norm ? 1 : 0;
    pa.cl_off = p.pass_cl_off[di][pass_index];
    pa.cl_len = p.pass_cl_len[di][pass_index];
    const bool cl = pa.cl_len > 0;
    const uint64_t ntiles = 1ull << (s.n - ps.t);
    // persistent grid: as many workgroups as fit on the device at once, each
    // walking tiles blockIdx.x, blockIdx.x + grid, ... with the next tile's
    // loads in flight while the current one is processed
    const bool wide = p.pass_wide[di][pass_index] != 0;
    const size_t amp = s.dtype == QS_C64 ? 8 : 16;
    int threads = TT;
    bool static_tile = false;
    TileKernel<float> k32 = nullptr;
    TileKernel<double> k64 = nullptr;
    if (s.dtype == QS_C64) k32 = pick_tile_kernel<float>(wide, ps.t, cl, threads, static_tile);
    else k64 = pick_tile_kernel<double>(wide, ps.t, cl, threads, static_tile);
    // dynamic LDS: none for the static-tile variants, else tile + norm slots + staged operands
    const size_t lds = static_tile ? 0 : (amp << ps.t) + kRedBytes + (size_t)pa.cl_len * (s.dtype == QS_C64 ? 4 : 8);
    const void *fn = k32 ? reinterpret_cast<const void *>(k32) : reinterpret_cast<const void *>(k64);
    QS_CHECK(static_tile || dynamic_tile_at_zero(fn), QS_EDEVICE,
             "tile kernel variant declares static LDS: its dynamic tile would not sit at LDS address 0");
    const uint64_t resident = resident_groups(fn, threads, lds);
    const dim3 grid((unsigned)std::min<uint64_t>(ntiles, std::min<uint64_t>(resident, kMaxTileGrid)));
    if (want_norm) {
        qs_status st = ensure_partials(s, ntiles);
        if (st != QS_OK) return st;
    }
    if (nparts) *nparts = ntiles;   // one norm partial per tile
    const double S = std::ldexp((double)amp, s.n);
    double flops = 0;
    for (int64_t b = ps.block0; b < ps.block0 + ps.nblocks; ++b)
        flops += block_flops_per_amp(p.h_blocks[di][b]) * std::ldexp(1.0, s.n);
    prof_begin(s.stream, QS_PROF_TILE, 2 * S, flops);
    unsigned long long *tickets = reinterpret_cast<unsigned long long *>(s.d_slots + kSlotTickets);
    if (s.dtype == QS_C64)
        hipLaunchKernelGGL(k32, grid, dim3(threads), lds, s.stream, (float2 *)s.amp, ntiles,
                           pa, p.d_blocks[di], (const float *)p.d_pool[di], s.d_slots + 1, s.d_partials, tickets,
                           (unsigned long long)s.tickets);
    else
        hipLaunchKernelGGL(k64, grid, dim3(threads), lds, s.stream, (double2 *)s.amp,
                           ntiles, pa, p.d_blocks[di], (const double *)p.d_pool[di], s.d_slots + 1, s.d_partials,
                           tickets, (unsigned long long)s.tickets);
    prof_end(s.stream);
    QS_HIP(hipGetLastError());
    // every tile's ticket plus one past the end per workgroup
    s.tickets += ntiles + grid.x;
    return QS_OK;
}

qs_status launch_norm_reduce(qs_state_s &s, uint64_t nparts, double *d_out_slots) {
    prof_begin(s.stream, QS_PROF_REDUCE, 8.0 * nparts, nparts);
    hipLaunchKernelGGL(k_norm_reduce, dim3(1), dim3(1024), 0, s.stream, s.d_partials, nparts, d_out_slots);
    prof_end(s.stream);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

qs_status launch_norm_full(qs_state_s &s, double *d_out_slots) {
    const uint64_t namps = 1ull << s.n;
    const uint64_t nwg = std::min<uint64_t>(8192, std::max<uint64_t>(1, namps / 4096));
    const uint64_t chunk = (namps + nwg - 1) / nwg;
    qs_status st = ensure_partials(s, nwg);
    if (st != QS_OK) return st;
    if (s.dtype == QS_C64)
        hipLaunchKernelGGL(k_norm_parts<float2>, dim3((unsigned)nwg), dim3(256), 0, s.stream, (const float2 *)s.amp,
                           namps, chunk, s.d_partials);
    else
        hipLaunchKernelGGL(k_norm_parts<double2>, dim3((unsigned)nwg), dim3(256), 0, s.stream, (const double2 *)s.amp,
                           namps, chunk, s.d_partials);
    QS_HIP(hipGetLastError());
    return launch_norm_reduce(s, nwg, d_out_slots);
}

}  // namespace qs
