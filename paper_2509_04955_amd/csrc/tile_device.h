// Device-side building blocks of a tile pass, shared by the single-state pass
// kernel and the persistent batch kernel.  Internal to libqsim.
//
// A tile is 2^t amplitudes held in LDS; tile position j < c is global qubit j,
// position c + i is the i-th "high" qubit of the pass.  Blocks (fused k-qubit
// unitaries) are applied in place to the LDS tile:
//   * dense blocks with k <= 3 (and all complex128 blocks): vector ALU, one
//     group of 2^k amplitudes per lane, matrix entries wave-uniform;
//   * dense complex64 blocks with k = 4, 5: MFMA, Y = [[Ur,-Ui],[Ui,Ur]] [Xr;Xi]
//     with v_mfma_f32_16x16x4f32 and a host-swizzled A operand;
//   * monomial blocks (one nonzero per column, e.g. CNOT/CZ/RZ products):
//     one complex multiply per amplitude and a permuted write.
#pragma once

#include "internal.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace qs {
namespace tiledev {

constexpr int TT = kTileThreads;

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

// LDS layout: amplitude li of the tile lives at sw(li) = li ^ (((li >> 4) & 7) << 1).
// The XOR moves bits 4..6 of the index into bits 1..3, so lanes whose group
// bases differ only above bit 3 (blocks on the low tile positions) land on
// different banks; bit 0 is untouched, so amplitude pairs (2i, 2i+1) stay
// adjacent for 16-byte accesses.  sw is linear over XOR, so for a group base b
// and an in-group offset o on disjoint bits sw(b | o) = sw(b) ^ sw(o): lanes
// swizzle their base once and XOR in wave-uniform swizzled offsets.
__host__ __device__ __forceinline__ uint32_t sw(uint32_t li) { return li ^ (((li >> 4) & 7u) << 1); }

// ---- vector-ALU block: one group of 2^K amplitudes per lane -------------
// Two groups per iteration when K <= 3 so each lane has independent LDS
// loads in flight.
template <int K, typename R>
__device__ __forceinline__ void dense_group(typename AmpOf<R>::A *tile, uint32_t b, const uint32_t *off,
                                            const R *__restrict__ U) {
    using A = typename AmpOf<R>::A;
    constexpr int D = 1 << K;
    A v[D];
#pragma unroll
    for (int r = 0; r < D; ++r) v[r] = tile[b ^ off[r]];
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
        tile[b ^ off[r]] = y;
    }
}

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
        off[r] = sw(o);
    }
    const uint32_t G = 1u << (T - K);
    auto base_of = [&](uint32_t g) {
        uint32_t b = g;
#pragma unroll
        for (int j = 0; j < K; ++j) b = ins0_32(b, pos[j]);
        return sw(b);
    };
    if constexpr (K <= 3) {
        if (G >= 2 * TT) {
            // G is a power of two >= 512: every lane has exactly G / 512 pairs of groups
            for (uint32_t g = threadIdx.x; g < G; g += 2 * TT) {
                const uint32_t b0 = base_of(g), b1 = base_of(g + TT);
                A v0[D], v1[D];
#pragma unroll
                for (int r = 0; r < D; ++r) {
                    v0[r] = tile[b0 ^ off[r]];
                    v1[r] = tile[b1 ^ off[r]];
                }
#pragma unroll
                for (int r = 0; r < D; ++r) {
                    R y0r = 0, y0i = 0, y1r = 0, y1i = 0;
#pragma unroll
                    for (int c = 0; c < D; ++c) {
                        const R ur = U[2 * (r * D + c)], ui = U[2 * (r * D + c) + 1];
                        y0r = fma(ur, v0[c].x, y0r);
                        y0r = fma(-ui, v0[c].y, y0r);
                        y0i = fma(ur, v0[c].y, y0i);
                        y0i = fma(ui, v0[c].x, y0i);
                        y1r = fma(ur, v1[c].x, y1r);
                        y1r = fma(-ui, v1[c].y, y1r);
                        y1i = fma(ur, v1[c].y, y1i);
                        y1i = fma(ui, v1[c].x, y1i);
                    }
                    A y0, y1;
                    y0.x = y0r;
                    y0.y = y0i;
                    y1.x = y1r;
                    y1.y = y1i;
                    tile[b0 ^ off[r]] = y0;
                    tile[b1 ^ off[r]] = y1;
                }
            }
            return;
        }
    }
    for (uint32_t g = threadIdx.x; g < G; g += TT) dense_group<K, R>(tile, base_of(g), off, U);
}

// ---- monomial block: one nonzero per column ---------------------------------
// y[dest(c)] = u_c x[c].  Diagonal blocks are the case dest(c) = c.  Pool entry
// c holds (Re u_c, Im u_c, tile offset of dest(c)) so every lane reads the same
// three values (scalar loads) and each group costs one complex multiply per
// amplitude.  A lane reads its whole group before writing any of it.
template <int K, typename R>
__device__ __forceinline__ void mono_group(typename AmpOf<R>::A *tile, uint32_t sb, const int *pos,
                                           const R *__restrict__ E) {
    using A = typename AmpOf<R>::A;
    constexpr int D = 1 << K;
    A v[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if ((c >> j) & 1) o |= 1u << pos[j];
        v[c] = tile[sb ^ sw(o)];
    }
#pragma unroll
    for (int c = 0; c < D; ++c) {
        const R ur = E[3 * c], ui = E[3 * c + 1];
        const uint32_t dst = (uint32_t)E[3 * c + 2];  // already swizzled on the host
        A y;
        y.x = ur * v[c].x - ui * v[c].y;
        y.y = ur * v[c].y + ui * v[c].x;
        tile[sb ^ dst] = y;
    }
}

template <int K, typename R>
__device__ __forceinline__ void mono_block(typename AmpOf<R>::A *tile, int T, const BlockDev *bd,
                                           const R *__restrict__ E) {
    int pos[K];
#pragma unroll
    for (int j = 0; j < K; ++j) pos[j] = bd->pos[j];
    const uint32_t G = 1u << (T - K);
    auto base_of = [&](uint32_t g) {
        uint32_t b = g;
#pragma unroll
        for (int j = 0; j < K; ++j) b = ins0_32(b, pos[j]);
        return sw(b);
    };
    if constexpr (K <= 3) {
        if (G >= 2 * TT) {
            for (uint32_t g = threadIdx.x; g < G; g += 2 * TT) {
                mono_group<K, R>(tile, base_of(g), pos, E);
                mono_group<K, R>(tile, base_of(g + TT), pos, E);
            }
            return;
        }
    }
    for (uint32_t g = threadIdx.x; g < G; g += TT) mono_group<K, R>(tile, base_of(g), pos, E);
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
    for (int m = 0; m < NB; ++m) offB[m] = sw(deposit(4 * m + gq));
    uint32_t offC[MT / 2][4];
#pragma unroll
    for (int h = 0; h < MT / 2; ++h)
#pragma unroll
        for (int q = 0; q < 4; ++q) offC[h][q] = sw(deposit(16 * h + 4 * gq + q));
    const uint32_t nchunks = (1u << (T - K)) / 16;
    for (uint32_t ch = wave; ch < nchunks; ch += TT / 64) {
        uint32_t cb = ch * 16 + jc;
#pragma unroll
        for (int j = 0; j < K; ++j) cb = ins0_32(cb, pos[j]);
        cb = sw(cb);
        float2 bv[NB];
#pragma unroll
        for (int m = 0; m < NB; ++m) bv[m] = tile[cb ^ offB[m]];
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
            for (int q = 0; q < 4; ++q) tile[cb ^ offC[h][q]] = make_float2(acc[h][q], acc[MT / 2 + h][q]);
    }
}

// ---- the pass kernel ------------------------------------------------------
// WIDE = false keeps register use low (dense VALU blocks up to k = 3; complex64
// k = 4, 5 through MFMA; monomial blocks up to k = 4); WIDE = true adds the
// widest blocks.  The host picks the variant per pass.
template <typename R, bool WIDE>
__device__ __forceinline__ void apply_block(typename AmpOf<R>::A *tile, int T, const BlockDev *bd,
                                            const R *__restrict__ pool) {
    const int k = bd->k;
    const int kind = bd->kind;
    const R *U = pool + bd->mat_off;
    constexpr bool F32 = sizeof(R) == 4;
    if constexpr (F32) {
        if (kind == BK_MFMA) {
            if (k == 4) mfma_block<4>(tile, T, bd, U);
            else mfma_block<5>(tile, T, bd, U);
            return;
        }
    }
    if (kind == BK_MONO) {
        switch (k) {
        case 1: mono_block<1, R>(tile, T, bd, U); return;
        case 2: mono_block<2, R>(tile, T, bd, U); return;
        case 3: mono_block<3, R>(tile, T, bd, U); return;
        case 4: mono_block<4, R>(tile, T, bd, U); return;
        default: break;
        }
        if constexpr (WIDE) {
            if (k == 5) { mono_block<5, R>(tile, T, bd, U); return; }
        }
        if constexpr (F32 && WIDE) {
            if (k == 6) { mono_block<6, R>(tile, T, bd, U); return; }
        }
        return;
    }
    switch (k) {
    case 1: valu_block<1, R>(tile, T, bd, U); return;
    case 2: valu_block<2, R>(tile, T, bd, U); return;
    case 3: valu_block<3, R>(tile, T, bd, U); return;
    default: break;
    }
    if constexpr (WIDE) {
        if (k == 4) valu_block<4, R>(tile, T, bd, U);
        else if (k == 5) valu_block<5, R>(tile, T, bd, U);
        if constexpr (F32) {
            if (k == 6) valu_block<6, R>(tile, T, bd, U);
        }
    }
}

}  // namespace tiledev
}  // namespace qs
