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
//     load and emits one FP64 partial of sum |a|^2 per tile on store; a single
//     workgroup then reduces the partials in a fixed order (deterministic).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "internal.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace qs {

namespace {

constexpr int TT = kTileThreads;
constexpr uint32_t kMaxTileGrid = 1u << 20;

__device__ __forceinline__ uint32_t ins0_32(uint32_t x, int p) {
    const uint32_t lo = x & ((1u << p) - 1);
    return ((x - lo) << 1) | lo;
}
__device__ __forceinline__ uint64_t ins0_64(uint64_t x, int p) {
    const uint64_t lo = x & ((1ull << p) - 1);
    return ((x - lo) << 1) | lo;
}

// global offset (in amplitudes, relative to the tile base) of tile index li
__device__ __forceinline__ uint64_t tile_offset(uint32_t li, const PassArgs &pa) {
    uint64_t off = li & ((1u << pa.c) - 1);
    const uint32_t h = li >> pa.c;
    const int nh = pa.t - pa.c;
#pragma unroll
    for (int j = 0; j < kMaxTile; ++j)
        if (j < nh && ((h >> j) & 1)) off |= 1ull << pa.hi[j];
    return off;
}

__device__ __forceinline__ uint64_t tile_base(uint64_t tile, const PassArgs &pa) {
    uint64_t b = tile << pa.c;
    const int nh = pa.t - pa.c;
#pragma unroll
    for (int j = 0; j < kMaxTile; ++j)
        if (j < nh) b = ins0_64(b, pa.hi[j]);
    return b;
}

template <typename R>
struct AmpOf;
template <>
struct AmpOf<float> {
    using A = float2;
};
template <>
struct AmpOf<double> {
    using A = double2;
};

// ---- vector-ALU block: one group of 2^K amplitudes per lane -------------
template <int K, typename R>
__device__ __forceinline__ void valu_block(typename AmpOf<R>::A *tile, int T, const BlockDev *bd,
                                           const R *__restrict__ U) {
    using A = typename AmpOf<R>::A;
    constexpr int D = 1 << K;
    int pos[K];
#pragma unroll
    for (int j = 0; j < K; ++j) pos[j] = bd->pos[j];
    uint32_t off[D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if ((r >> j) & 1) o |= 1u << pos[j];
        off[r] = o;
    }
    const uint32_t G = 1u << (T - K);
    for (uint32_t g = threadIdx.x; g < G; g += TT) {
        uint32_t b = g;
#pragma unroll
        for (int j = 0; j < K; ++j) b = ins0_32(b, pos[j]);
        A v[D];
#pragma unroll
        for (int r = 0; r < D; ++r) v[r] = tile[b + off[r]];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            R yr = 0, yi = 0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const R ur = U[2 * (r * D + c)], ui = U[2 * (r * D + c) + 1];
                yr = fma(ur, v[c].x, yr);
                yr = fma(-ui, v[c].y, yr);
                yi = fma(ur, v[c].y, yi);
                yi = fma(ui, v[c].x, yi);
            }
            A y;
            y.x = yr;
            y.y = yi;
            tile[b + off[r]] = y;
        }
    }
}

// ---- MFMA block (complex64, K = 4 or 5) ---------------------------------
// Lane l of a wave: g = l / 16 selects the K-slice of each 16x16x4 step and the
// output row quad, j = l % 16 the tile column.  Step s feeds B row (s/2)*4 + g
// (real part for even s, imaginary for odd s); outputs land as complete
// complex numbers Y[16h + 4g + q] (Re in M-tile h, Im in M-tile MT/2 + h).
template <int K>
__device__ __forceinline__ void mfma_block(float2 *tile, int T, const BlockDev *bd, const float *__restrict__ Asw) {
    constexpr int D = 1 << K;
    constexpr int MT = 2 * D / 16;
    constexpr int S = 2 * D / 4;
    constexpr int NB = D / 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gq = lane >> 4, jc = lane & 15;
    int pos[K];
#pragma unroll
    for (int j = 0; j < K; ++j) pos[j] = bd->pos[j];
    float a[MT][S];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int s = 0; s < S; ++s) a[mt][s] = Asw[(mt * S + s) * 64 + lane];
    auto deposit = [&](int r) {
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if ((r >> j) & 1) o |= 1u << pos[j];
        return o;
    };
    uint32_t offB[NB];
#pragma unroll
    for (int m = 0; m < NB; ++m) offB[m] = deposit(4 * m + gq);
    uint32_t offC[MT / 2][4];
#pragma unroll
    for (int h = 0; h < MT / 2; ++h)
#pragma unroll
        for (int q = 0; q < 4; ++q) offC[h][q] = deposit(16 * h + 4 * gq + q);
    const uint32_t nchunks = (1u << (T - K)) / 16;
    for (uint32_t ch = wave; ch < nchunks; ch += TT / 64) {
        uint32_t cb = ch * 16 + jc;
#pragma unroll
        for (int j = 0; j < K; ++j) cb = ins0_32(cb, pos[j]);
        float2 bv[NB];
#pragma unroll
        for (int m = 0; m < NB; ++m) bv[m] = tile[cb + offB[m]];
        floatx4 acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const float b = (s & 1) ? bv[s >> 1].y : bv[s >> 1].x;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt][s], b, acc[mt], 0, 0, 0);
        }
#pragma unroll
        for (int h = 0; h < MT / 2; ++h)
#pragma unroll
            for (int q = 0; q < 4; ++q) tile[cb + offC[h][q]] = make_float2(acc[h][q], acc[MT / 2 + h][q]);
    }
}

// ---- the pass kernel ------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(TT) void k_tile_pass(typename AmpOf<R>::A *__restrict__ psi, uint64_t ntiles, PassArgs pa,
                                                  const BlockDev *__restrict__ blocks, const R *__restrict__ pool,
                                                  const double *__restrict__ scale_in, double *__restrict__ partials) {
    using A = typename AmpOf<R>::A;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    A *tile = reinterpret_cast<A *>(smem_raw);
    __shared__ double red[TT / 64];
    const int T = pa.t;
    const uint32_t tsize = 1u << T;
    const R sc = pa.apply_scale ? (R)(*scale_in) : (R)1;
    for (uint64_t tileid = blockIdx.x; tileid < ntiles; tileid += gridDim.x) {
        const uint64_t base = tile_base(tileid, pa);
        // ---- load (scaled) ----
        if constexpr (sizeof(R) == 4) {
            for (uint32_t li = threadIdx.x * 2; li < tsize; li += TT * 2) {
                const uint64_t gidx = base | tile_offset(li, pa);
                float4 v = *reinterpret_cast<const float4 *>(psi + gidx);
                v.x *= sc;
                v.y *= sc;
                v.z *= sc;
                v.w *= sc;
                *reinterpret_cast<float4 *>(tile + li) = v;
            }
        } else {
            for (uint32_t li = threadIdx.x; li < tsize; li += TT) {
                A v = psi[base | tile_offset(li, pa)];
                v.x *= sc;
                v.y *= sc;
                tile[li] = v;
            }
        }
        __syncthreads();
        // ---- blocks ----
        for (int b = 0; b < pa.nblocks; ++b) {
            const BlockDev *bd = blocks + pa.block0 + b;
            const int k = bd->k;
            const R *U = pool + bd->mat_off;
            if constexpr (sizeof(R) == 4) {
                if (bd->mfma) {
                    if (k == 4) mfma_block<4>(tile, T, bd, U);
                    else mfma_block<5>(tile, T, bd, U);
                    __syncthreads();
                    continue;
                }
            }
            switch (k) {
            case 1: valu_block<1, R>(tile, T, bd, U); break;
            case 2: valu_block<2, R>(tile, T, bd, U); break;
            case 3: valu_block<3, R>(tile, T, bd, U); break;
            case 4: valu_block<4, R>(tile, T, bd, U); break;
            case 5: valu_block<5, R>(tile, T, bd, U); break;
            default:
                if constexpr (sizeof(R) == 4) valu_block<6, R>(tile, T, bd, U);
                break;
            }
            __syncthreads();
        }
        // ---- store + FP64 norm partial ----
        double nacc = 0.0;
        if constexpr (sizeof(R) == 4) {
            for (uint32_t li = threadIdx.x * 2; li < tsize; li += TT * 2) {
                const float4 v = *reinterpret_cast<const float4 *>(tile + li);
                *reinterpret_cast<float4 *>(psi + (base | tile_offset(li, pa))) = v;
                nacc += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
            }
        } else {
            for (uint32_t li = threadIdx.x; li < tsize; li += TT) {
                const A v = tile[li];
                psi[base | tile_offset(li, pa)] = v;
                nacc += v.x * v.x + v.y * v.y;
            }
        }
        if (pa.want_norm) {
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) nacc += __shfl_xor(nacc, o);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nacc;
            __syncthreads();
            if (threadIdx.x == 0) {
                double s = 0;
#pragma unroll
                for (int w = 0; w < TT / 64; ++w) s += red[w];
                partials[tileid] = s;
            }
        }
        __syncthreads();  // the tile buffer is reused by the next tile
    }
}

// one workgroup: fixed-order FP64 sum of the partials; slot[0] = N, slot[1] = 1/sqrt(N)
__global__ __launch_bounds__(1024) void k_norm_reduce(const double *__restrict__ parts, uint64_t n,
                                                      double *__restrict__ slots) {
    __shared__ double sh[1024];
    double s = 0;
    for (uint64_t i = threadIdx.x; i < n; i += 1024) s += parts[i];
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

template <typename R>
void set_lds_limit(size_t bytes) {
    static size_t done = 0;
    if (bytes > done) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_tile_pass<R>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        done = bytes;
    }
}

bool mfma_enabled() {
    static int v = -1;
    if (v < 0) {
        const char *e = getenv("QS_TILE_MFMA");
        v = e ? atoi(e) != 0 : 1;
    }
    return v == 1;
}

// Host-side A-operand swizzle of a complex64 block for mfma_block<K>.
void swizzle_mfma(const std::vector<cd> &U, int k, std::vector<float> &out) {
    const int D = 1 << k, MT = 2 * D / 16, S = 2 * D / 4;
    for (int mt = 0; mt < MT; ++mt)
        for (int s = 0; s < S; ++s)
            for (int lane = 0; lane < 64; ++lane) {
                const int i = lane % 16, g = lane / 16;
                const int R = 16 * mt + i;
                const int r = 4 * (s / 2) + g, p = s % 2;
                const int rr = R % D, ro = R / D;
                const cd u = U[(size_t)rr * D + r];
                double v;
                if (ro == 0) v = p == 0 ? u.real() : -u.imag();
                else v = p == 0 ? u.imag() : u.real();
                out.push_back((float)v);
            }
}

}  // namespace

qs_status plan_upload(qs_plan_s &p, qs_dtype dt) {
    const int di = dt == QS_C64 ? 0 : 1;
    if (p.dev_ready[di]) return QS_OK;
    std::vector<BlockDev> hb(p.blocks.size());
    std::vector<float> pool32;
    std::vector<double> pool64;
    for (const HPass &ps : p.passes) {
        for (int64_t b = ps.block0; b < ps.block0 + ps.nblocks; ++b) {
            const HBlock &blk = p.blocks[b];
            BlockDev &d = hb[b];
            std::memset(&d, 0, sizeof d);
            d.k = (int)blk.qubits.size();
            QS_CHECK(d.k >= 1 && d.k <= (dt == QS_C64 ? kMaxK : kMaxK128), QS_EUNSUPPORTED,
                     "block width %d unsupported for this dtype", d.k);
            for (int j = 0; j < d.k; ++j)
                d.pos[j] = (int)(std::find(ps.tile.begin(), ps.tile.end(), blk.qubits[j]) - ps.tile.begin());
            const int D = 1 << d.k;
            if (dt == QS_C64) {
                d.mfma = (d.k == 4 || d.k == 5) && ps.t - d.k >= 4 && mfma_enabled();
                d.mat_off = (int32_t)pool32.size();
                if (d.mfma) {
                    swizzle_mfma(blk.U, d.k, pool32);
                } else {
                    for (int i = 0; i < D * D; ++i) {
                        pool32.push_back((float)blk.U[i].real());
                        pool32.push_back((float)blk.U[i].imag());
                    }
                }
                // keep every matrix 16-byte aligned
                while (pool32.size() % 4) pool32.push_back(0.f);
            } else {
                d.mat_off = (int32_t)pool64.size();
                for (int i = 0; i < D * D; ++i) {
                    pool64.push_back(blk.U[i].real());
                    pool64.push_back(blk.U[i].imag());
                }
            }
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
                      bool want_norm) {
    (void)pass_index;
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
    const uint64_t ntiles = 1ull << (s.n - ps.t);
    if (want_norm) {
        qs_status st = ensure_partials(s, ntiles);
        if (st != QS_OK) return st;
    }
    const dim3 grid((unsigned)std::min<uint64_t>(ntiles, kMaxTileGrid));
    const size_t amp = s.dtype == QS_C64 ? 8 : 16;
    const size_t lds = amp << ps.t;
    const double S = std::ldexp((double)amp, s.n);
    double flops = 0;
    for (int64_t b = ps.block0; b < ps.block0 + ps.nblocks; ++b)
        flops += 8.0 * std::ldexp(1.0, (int)p.blocks[b].qubits.size()) * std::ldexp(1.0, s.n);
    prof_begin(s.stream, QS_PROF_TILE, 2 * S, flops);
    if (s.dtype == QS_C64) {
        set_lds_limit<float>(lds);
        hipLaunchKernelGGL(k_tile_pass<float>, grid, dim3(TT), lds, s.stream, (float2 *)s.amp, ntiles, pa,
                           p.d_blocks[di], (const float *)p.d_pool[di], s.d_slots + 1, s.d_partials);
    } else {
        set_lds_limit<double>(lds);
        hipLaunchKernelGGL(k_tile_pass<double>, grid, dim3(TT), lds, s.stream, (double2 *)s.amp, ntiles, pa,
                           p.d_blocks[di], (const double *)p.d_pool[di], s.d_slots + 1, s.d_partials);
    }
    prof_end(s.stream);
    QS_HIP(hipGetLastError());
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
