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

#include <type_traits>

#include "internal.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

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

// 16x16x4 MFMA per real type: lane l supplies A[l%16][l/16] and B[l/16][l%16]
// for both types; output item q of lane l is column l%16 and row
// row(l/16, q): 4(l/16) + q for v_mfma_f32_16x16x4f32, (l/16) + 4q for
// v_mfma_f64_16x16x4f64 (measured on gfx950 with a lane-layout probe).
template <typename R>
struct Mfma;
template <>
struct Mfma<float> {
    using V4 = floatx4;
    __device__ __forceinline__ static V4 op(float a, float b, V4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __host__ __device__ static constexpr int row(int g, int q) { return 4 * g + q; }
};
template <>
struct Mfma<double> {
    using V4 = doublex4;
    __device__ __forceinline__ static V4 op(double a, double b, V4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __host__ __device__ static constexpr int row(int g, int q) { return g + 4 * q; }
};

// LDS layout: amplitude li of the tile lives at sw(li) = li ^ (((li >> 4) & 7) << 1).
// The XOR moves bits 4..6 of the index into bits 1..3, so lanes whose group
// bases differ only above bit 3 (blocks on the low tile positions) land on
// different banks; bit 0 is untouched, so amplitude pairs (2i, 2i+1) stay
// adjacent for 16-byte accesses.  sw is linear over XOR, so for a group base b
// and an in-group offset o on disjoint bits sw(b | o) = sw(b) ^ sw(o): lanes
// swizzle their base once and XOR in wave-uniform swizzled offsets.
__host__ __device__ __forceinline__ uint32_t sw(uint32_t li) { return li ^ (((li >> 4) & 7u) << 1); }

// ---- tile references ---------------------------------------------------------
// Block code names an LDS amplitude by a group handle and an in-group byte
// offset: grp(g) for a group whose swizzled byte offset in the tile is g, and
// at<T>(h, o) for the element at tile byte offset g ^ o (the group base and
// the in-group offset are on disjoint index bits and the swizzle is linear
// over XOR, so g ^ o is the swizzled offset of their sum).  TileAligned is a
// tile at an LDS address aligned to kTileAlign, above every tile size, so
// base + (g ^ o) = (base | g) ^ o: a group costs one OR and an access one XOR
// (an LDS base that is only known at link time, as a dynamic region's, would
// otherwise cost an add per access).  TilePtr places a tile at any address.
typedef __attribute__((address_space(3))) unsigned char lds_u8;
constexpr uint32_t kTileAlign = 1u << 17;

__device__ __forceinline__ uint32_t lds_addr(const void *p) { return (uint32_t)(uintptr_t)(const lds_u8 *)p; }

struct TileAligned {
    uint32_t base;   // LDS address, a multiple of kTileAlign
    __device__ __forceinline__ uint32_t grp(uint32_t g) const { return base | g; }
    template <typename T>
    __device__ __forceinline__ T *at(uint32_t h, uint32_t o) const {
        return (T *)(lds_u8 *)(uintptr_t)(h ^ o);
    }
};

struct TilePtr {
    unsigned char *base;
    __device__ __forceinline__ uint32_t grp(uint32_t g) const { return g; }
    template <typename T>
    __device__ __forceinline__ T *at(uint32_t h, uint32_t o) const {
        return reinterpret_cast<T *>(base + (h ^ o));
    }
};

// Matrix-core blocks walk a block's groups in chunks of 16 (column jc of
// chunk ch is group 16 ch + jc).  Inserting the block's zero bits is linear
// over disjoint bit fields and so is the swizzle, so a group's handle is the
// lane's part, grp(sw(dep(jc)) * bytes) formed once per block, XOR the
// chunk's part sw(dep(16 ch)) * bytes, which is uniform over the wave and
// formed on the scalar unit.
template <int K>
__device__ __forceinline__ uint32_t chunk_part(uint32_t ch, const int *pos, uint32_t bytes) {
    uint32_t c = ch * 16;
#pragma unroll
    for (int j = 0; j < K; ++j) c = ins0_32(c, pos[j]);
    return sw(c) * bytes;
}
template <int K, typename TL>
__device__ __forceinline__ uint32_t lane_part(const TL &tl, uint32_t jc, const int *pos, uint32_t bytes) {
    uint32_t c = jc;
#pragma unroll
    for (int j = 0; j < K; ++j) c = ins0_32(c, pos[j]);
    return tl.grp(sw(c) * bytes);
}

// A 32-bit pattern stored in an operand pool entry (bit-cast, not converted).
__device__ __forceinline__ uint32_t pool_bits(float v) { return __float_as_uint(v); }
__device__ __forceinline__ uint32_t pool_bits(double v) { return (uint32_t)__double_as_longlong(v); }

// ---- vector-ALU block: one group of 2^K amplitudes per lane -------------
// Two groups per iteration when K <= 3 so each lane has independent LDS
// loads in flight.
template <int K, typename R, typename TL>
__device__ __forceinline__ void dense_group(TL tl, uint32_t h, const uint32_t *off, const R *__restrict__ U) {
    using A = typename AmpOf<R>::A;
    constexpr int D = 1 << K;
    A v[D];
#pragma unroll
    for (int r = 0; r < D; ++r) v[r] = *tl.template at<A>(h, off[r]);
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
        *tl.template at<A>(h, off[r]) = y;
    }
}

template <int K, typename R, int NT = TT, typename TL>
__device__ __forceinline__ void valu_block(TL tl, int T, const BlockDev *bd, const R *__restrict__ U) {
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
        off[r] = sw(o) * (uint32_t)sizeof(A);
    }
    const uint32_t G = 1u << (T - K);
    auto base_of = [&](uint32_t g) {
        uint32_t b = g;
#pragma unroll
        for (int j = 0; j < K; ++j) b = ins0_32(b, pos[j]);
        return tl.grp(sw(b) * (uint32_t)sizeof(A));
    };
    if constexpr (K <= 3) {
        if (G >= 2 * NT) {
            // G is a power of two >= 512: every lane has exactly G / 512 pairs of groups
            for (uint32_t g = threadIdx.x; g < G; g += 2 * NT) {
                // matrix loads stay in the loop: hoisted, the 2^(2K+1) scalar
                // values would be spilled and re-read lane by lane every iteration
                asm volatile("" ::: "memory");
                const uint32_t b0 = base_of(g), b1 = base_of(g + NT);
                A v0[D], v1[D];
#pragma unroll
                for (int r = 0; r < D; ++r) {
                    v0[r] = *tl.template at<A>(b0, off[r]);
                    v1[r] = *tl.template at<A>(b1, off[r]);
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
                    *tl.template at<A>(b0, off[r]) = y0;
                    *tl.template at<A>(b1, off[r]) = y1;
                }
            }
            return;
        }
    }
    for (uint32_t g = threadIdx.x; g < G; g += NT) {
        asm volatile("" ::: "memory");
        dense_group<K, R>(tl, base_of(g), off, U);
    }
}

// ---- monomial block: one nonzero per column ---------------------------------
// y[dest(c)] = u_c x[c].  Diagonal blocks are the case dest(c) = c.  Pool entry
// c is a 4-value record (Re u_c, Im u_c, swizzled tile byte offset of dest(c)
// as a bit pattern, 0),
// read as wave-uniform scalars when a group fits one lane.  A group of 2^K amplitudes is handled by LPG lanes of
// one wave (LPG = 1 for K <= 3, 2^(K-3) above), each holding 8 or fewer
// sources; the lanes of a wave issue all their LDS reads before any write, so
// the in-place permutation is safe.
template <int K, typename R, int NT = TT, typename TL>
__device__ __forceinline__ void mono_block(TL tl, int T, const BlockDev *bd, const R *__restrict__ E) {
    using A = typename AmpOf<R>::A;
    constexpr int LPG = K <= 3 ? 1 : (1 << (K > 3 ? K - 3 : 0));
    constexpr int SPL = (1 << K) / LPG;
    constexpr int KL = K <= 3 ? K : 3;   // bits of c that index within a lane
    int pos[K];
#pragma unroll
    for (int j = 0; j < K; ++j) pos[j] = bd->pos[j];
    auto deposit = [&](uint32_t c) {
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if ((c >> j) & 1) o |= 1u << pos[j];
        return o;
    };
    const uint32_t G = 1u << (T - K);
    const uint32_t tasks = G * LPG;
    auto group = [&](uint32_t tk) {
        const uint32_t g = tk / LPG, p = tk % LPG;
        uint32_t b = g;
#pragma unroll
        for (int j = 0; j < K; ++j) b = ins0_32(b, pos[j]);
        const uint32_t hs = tl.grp((sw(b) ^ sw(deposit(p << KL))) * (uint32_t)sizeof(A));
        A v[SPL];
#pragma unroll
        for (int i = 0; i < SPL; ++i) v[i] = *tl.template at<A>(hs, sw(deposit((uint32_t)i)) * (uint32_t)sizeof(A));
        const uint32_t hd = tl.grp(sw(b) * (uint32_t)sizeof(A));
        // entry c = p * SPL + i: wave-uniform (scalar loads) when LPG == 1
        const R *Ep = E + 4 * (p * SPL);
#pragma unroll
        for (int i = 0; i < SPL; ++i) {
            const R ur = Ep[4 * i], ui = Ep[4 * i + 1];
            const uint32_t dst = pool_bits(Ep[4 * i + 2]);
            A y;
            y.x = ur * v[i].x - ui * v[i].y;
            y.y = ur * v[i].y + ui * v[i].x;
            *tl.template at<A>(hd, dst) = y;
        }
    };
    if constexpr (K <= 3) {
        if (tasks >= 2 * NT) {
            for (uint32_t tk = threadIdx.x; tk < tasks; tk += 2 * NT) {
                group(tk);
                group(tk + NT);
            }
            return;
        }
    }
    for (uint32_t tk = threadIdx.x; tk < tasks; tk += NT) group(tk);
}


// ---- permuted block-diagonal block ------------------------------------------
// The block's 2^K rows and columns split into 2^(K-S) classes of 2^S that U
// maps onto each other: y[rows of class j] = B_j x[columns of class j].  Pool
// record: 2^K swizzled tile offsets of the columns (class by class), 2^K of the
// rows, then B_0, B_1, ... (2^S x 2^S complex, row-major).  One lane holds a
// whole group, so the in-place update only touches its own amplitudes, and
// every operand is wave-uniform (scalar loads).  The offsets are byte offsets
// stored as bit patterns: one XOR per LDS address.
template <int K, int S, typename R, int NT = TT, typename TL>
__device__ __forceinline__ void bdiag_block(TL tl, int T, const BlockDev *bd, const R *__restrict__ E) {
    using A = typename AmpOf<R>::A;
    constexpr int D = 1 << K, DS = 1 << S, NC = D / DS;
    int pos[K];
#pragma unroll
    for (int j = 0; j < K; ++j) pos[j] = bd->pos[j];
    const R *B = E + 2 * D;
    const uint32_t G = 1u << (T - K);
    for (uint32_t g = threadIdx.x; g < G; g += NT) {
        uint32_t b = g;
#pragma unroll
        for (int j = 0; j < K; ++j) b = ins0_32(b, pos[j]);
        const uint32_t h = tl.grp(sw(b) * (uint32_t)sizeof(A));
        A v[D];
#pragma unroll
        for (int i = 0; i < D; ++i) v[i] = *tl.template at<A>(h, pool_bits(E[i]));
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            // keeps each class's operand loads beside their use (hoisted out of
            // the group loop they would need 2^(K+S+1) scalar registers)
            asm volatile("" ::: "memory");
#pragma unroll
            for (int r = 0; r < DS; ++r) {
                const R *Br = B + 2 * ((j * DS + r) * DS);
                R yr = 0, yi = 0;
#pragma unroll
                for (int c = 0; c < DS; ++c) {
                    const A x = v[j * DS + c];
                    const R ur = Br[2 * c], ui = Br[2 * c + 1];
                    yr = fma(ur, x.x, yr);
                    yr = fma(-ui, x.y, yr);
                    yi = fma(ur, x.y, yi);
                    yi = fma(ui, x.x, yi);
                }
                A y;
                y.x = yr;
                y.y = yi;
                *tl.template at<A>(h, pool_bits(E[D + j * DS + r])) = y;
            }
        }
    }
}

// ---- permutation block ------------------------------------------------------
// y[dest(c)] = x[c] with every nonzero entry 1 (products of CNOT, X, SWAP):
// the class path without its multiplies.  Record: 2^K swizzled source byte
// offsets, then dest(c)'s for c = 0..2^K-1 (bit patterns, wave-uniform).  A
// lane reads its whole group before writing it.
template <int K, typename R, int NT = TT, typename TL>
__device__ __forceinline__ void perm_block(TL tl, int T, const BlockDev *bd, const R *__restrict__ E) {
    using A = typename AmpOf<R>::A;
    constexpr int D = 1 << K;
    int pos[K];
#pragma unroll
    for (int j = 0; j < K; ++j) pos[j] = bd->pos[j];
    const uint32_t G = 1u << (T - K);
    for (uint32_t g = threadIdx.x; g < G; g += NT) {
        uint32_t b = g;
#pragma unroll
        for (int j = 0; j < K; ++j) b = ins0_32(b, pos[j]);
        const uint32_t h = tl.grp(sw(b) * (uint32_t)sizeof(A));
        A v[D];
#pragma unroll
        for (int c = 0; c < D; ++c) v[c] = *tl.template at<A>(h, pool_bits(E[c]));
#pragma unroll
        for (int c = 0; c < D; ++c) *tl.template at<A>(h, pool_bits(E[D + c])) = v[c];
    }
}

// One Pauli-rotation pair update: y0 = c a + sigma1 d b, y1 = c b + sigma0 d a,
// sigma as float sign bits s0, s1.  MODE 0: c, d complex; 1: c real, d = i*dI
// (Pauli exponentials without a phase: 4 products per output instead of 8);
// 2: c and d real.
template <int MODE, typename A, typename R>
__device__ __forceinline__ void rot_pair(A &y0, A &y1, const A a, const A b, uint32_t s0, uint32_t s1, R cr, R ci,
                                         R dr, R di) {
    auto flip = [](R v, uint32_t s) {
        if constexpr (sizeof(R) == 4) return __uint_as_float(__float_as_uint(v) ^ s);
        else return __longlong_as_double(__double_as_longlong(v) ^ ((unsigned long long)s << 32));
    };
    if constexpr (MODE == 1) {
        const R e1 = flip(di, s1), e0 = flip(di, s0);
        y0.x = cr * a.x - e1 * b.y;
        y0.y = cr * a.y + e1 * b.x;
        y1.x = cr * b.x - e0 * a.y;
        y1.y = cr * b.y + e0 * a.x;
    } else if constexpr (MODE == 2) {
        const R e1 = flip(dr, s1), e0 = flip(dr, s0);
        y0.x = cr * a.x + e1 * b.x;
        y0.y = cr * a.y + e1 * b.y;
        y1.x = cr * b.x + e0 * a.x;
        y1.y = cr * b.y + e0 * a.y;
    } else {
        const R e1r = flip(dr, s1), e1i = flip(di, s1), e0r = flip(dr, s0), e0i = flip(di, s0);
        y0.x = cr * a.x - ci * a.y + e1r * b.x - e1i * b.y;
        y0.y = cr * a.y + ci * a.x + e1r * b.y + e1i * b.x;
        y1.x = cr * b.x - ci * b.y + e0r * a.x - e0i * a.y;
        y1.y = cr * b.y + ci * b.x + e0r * a.y + e0i * a.x;
    }
}

// ---- Pauli rotation ------------------------------------------------------------
// y[k] = c psi[k] + d sigma(k ^ x) psi[k ^ x], sigma(j) = (-1)^{|j & z|} over the
// global index j.  Record: x and z over tile positions, the z bits of qubits
// outside the tile (their parity is fixed per tile: gbase, the global index of
// tile position 0, carries them), c, d.  One lane per pair (k, k ^ x), or per
// amplitude when x = 0 (diagonal).
template <typename R, int NT, int MODE, typename TL>
__device__ __forceinline__ void pauli_block_m(TL tl, int T, const R *__restrict__ E, uint64_t gbase) {
    using A = typename AmpOf<R>::A;
    const uint32_t x = pool_bits(E[0]), zt = pool_bits(E[1]);
    const uint64_t zo = (uint64_t)pool_bits(E[2]) | ((uint64_t)pool_bits(E[3]) << 32);
    const uint32_t so = (uint32_t)__builtin_popcountll(gbase & zo) & 1u;
    const R cr = E[4], ci = E[5], dr = E[6], di = E[7];
    // sign of sigma(j) as a float sign bit: ((|j & zt| + so) & 1) << 31
    auto sbit = [&](uint32_t j) { return (((uint32_t)__builtin_popcount(j & zt) ^ so) & 1u) << 31; };
    if (x == 0) {
        const R pr = cr + dr, pi = ci + di, mr = cr - dr, mi = ci - di;
        for (uint32_t k = threadIdx.x; k < (1u << T); k += NT) {
            const bool neg = sbit(k) != 0;
            const R fr = neg ? mr : pr, fi = neg ? mi : pi;
            A *v = tl.template at<A>(tl.grp(sw(k) * (uint32_t)sizeof(A)), 0u);
            const A a = *v;
            A y;
            y.x = fr * a.x - fi * a.y;
            y.y = fr * a.y + fi * a.x;
            *v = y;
        }
        return;
    }
    // pairs (k0, k0 ^ x), k0 with bit h of x clear; the swizzle is linear, so
    // the partner's LDS offset is the pair's XOR a wave-uniform constant, and
    // sigma(k0 ^ x) = sigma(k0) (-1)^{|x & zt|}
    const int h = 31 - __builtin_clz(x);
    const uint32_t swx = sw(x) * (uint32_t)sizeof(A);
    const uint32_t sx = ((uint32_t)__builtin_popcount(x & zt) & 1u) << 31;
    const uint32_t half = 1u << (T - 1);
    auto pair = [&](uint32_t g) {
        const uint32_t k0 = ins0_32(g, h);
        const uint32_t h0 = tl.grp(sw(k0) * (uint32_t)sizeof(A));
        A *p0 = tl.template at<A>(h0, 0u), *p1 = tl.template at<A>(h0, swx);
        const A a = *p0, b = *p1;
        const uint32_t s0 = sbit(k0), s1 = s0 ^ sx;
        A y0, y1;
        rot_pair<MODE>(y0, y1, a, b, s0, s1, cr, ci, dr, di);
        *p0 = y0;
        *p1 = y1;
    };
    if (half >= 2 * NT) {
        // every lane has exactly half / (2 NT) pairs of pairs: two independent
        // chains per iteration
        for (uint32_t g = threadIdx.x; g < half; g += 2 * NT) {
            pair(g);
            pair(g + NT);
        }
        return;
    }
    for (uint32_t g = threadIdx.x; g < half; g += NT) pair(g);
}

// mode (BlockDev.sub): coefficient form, see rot_pair
template <typename R, int NT = TT, typename TL>
__device__ __forceinline__ void pauli_block(TL tl, int T, const R *__restrict__ E, uint64_t gbase, int mode) {
    if (mode == 1) pauli_block_m<R, NT, 1>(tl, T, E, gbase);
    else if (mode == 2) pauli_block_m<R, NT, 2>(tl, T, E, gbase);
    else pauli_block_m<R, NT, 0>(tl, T, E, gbase);
}

// ---- group of M Pauli rotations (M = 2, 3) -------------------------------------
// Consecutive rotations whose X parts x_0..x_{M-1} are linearly independent act
// on the cosets k0 + span(x_j): one lane loads the 2^M amplitudes of a coset
// (member c = k0 ^ sum_j c_j x_j), applies the rotations in order in registers
// (rotation i pairs members c and c ^ 2^i) and stores them.  k0 has zeros at M
// pivot positions (an echelon form of the x_j), which makes the cosets a
// partition of the tile.  Record: pivots (3 entries), the rotations' coefficient
// forms (2 bits each, see rot_pair), swizzled byte offsets of the 2^M members
// (16 entries), then per rotation: z over tile positions, z of the qubits
// outside the tile (two entries), the parities |x_j & z| as a mask over j, c, d.
template <typename R, int M, int NT = TT, typename TL>
__device__ __forceinline__ void pauli_group(TL tl, int T, const R *__restrict__ E, uint64_t gbase) {
    using A = typename AmpOf<R>::A;
    constexpr int NM = 1 << M;
    int piv[M];
#pragma unroll
    for (int j = 0; j < M; ++j) piv[j] = (int)pool_bits(E[j]);
    const uint32_t modes = pool_bits(E[3]);   // 2 bits per rotation (M <= 3 leaves slot 3 free)
    const R *Rt = E + 20;
    const uint32_t G = 1u << (T - M);
    for (uint32_t g = threadIdx.x; g < G; g += NT) {
        uint32_t k0 = g;
#pragma unroll
        for (int j = 0; j < M; ++j) k0 = ins0_32(k0, piv[j]);
        const uint32_t hb = tl.grp(sw(k0) * (uint32_t)sizeof(A));
        A v[NM];
#pragma unroll
        for (int c = 0; c < NM; ++c) v[c] = *tl.template at<A>(hb, pool_bits(E[4 + c]));
#pragma unroll
        for (int i = 0; i < M; ++i) {
            const R *Ri = Rt + 8 * i;
            const uint32_t zt = pool_bits(Ri[0]);
            const uint64_t zo = (uint64_t)pool_bits(Ri[1]) | ((uint64_t)pool_bits(Ri[2]) << 32);
            const uint32_t pm = pool_bits(Ri[3]);
            const R cr = Ri[4], ci = Ri[5], dr = Ri[6], di = Ri[7];
            const uint32_t mode = (modes >> (2 * i)) & 3u;
            // sign of sigma_i at member c: |k0 & z| + |tile base & z outside| + |c & pm|
            const uint32_t s0 =
                (((uint32_t)__builtin_popcount(k0 & zt) ^ (uint32_t)__builtin_popcountll(gbase & zo)) & 1u) << 31;
            auto rot = [&](auto mode_tag) {
                constexpr int MD = decltype(mode_tag)::value;
#pragma unroll
                for (int c = 0; c < NM; ++c) {
                    if (c & (1 << i)) continue;
                    const int c2 = c | (1 << i);
                    const uint32_t sc = s0 ^ (((uint32_t)__builtin_popcount((uint32_t)c & pm) & 1u) << 31);
                    const uint32_t sc2 = s0 ^ (((uint32_t)__builtin_popcount((uint32_t)c2 & pm) & 1u) << 31);
                    const A a = v[c], b = v[c2];
                    rot_pair<MD>(v[c], v[c2], a, b, sc, sc2, cr, ci, dr, di);
                }
            };
            if (mode == 1) rot(std::integral_constant<int, 1>());
            else if (mode == 2) rot(std::integral_constant<int, 2>());
            else rot(std::integral_constant<int, 0>());
        }
#pragma unroll
        for (int c = 0; c < NM; ++c) *tl.template at<A>(hb, pool_bits(E[4 + c])) = v[c];
    }
}

// ---- MFMA block, operands from the pool (K = 4, 5; complex64 also 6) --------
// Y = A X with A = [[Ur, -Ui], [Ui, Ur]] (2D x 2D, D = 2^K) and X the 2D x N
// real view of the tile (rows: Re then Im of the block's 2^K amplitudes;
// columns: the other tile positions).  16x16x4 MFMA (FP32 or FP64): lane l
// supplies A[l%16][kk] and B[kk][l%16] with kk = 4s + l/16 for step s;
// K-order is chosen so step s reads row 4(s/2) + l/16 of X, real part for
// even s and imaginary for odd s, and output register q of lane l is row
// Mfma::row(l/16, q) of the M-tile.  Each wave owns MPW 16-row M-tiles (their
// slice of A stays in MPW * 2^(K-1) registers): with fewer M-tiles than waves
// the waves sharing one split the columns, with more (K = 6: 8 M-tiles over
// 4 waves) each wave runs two.  Columns go in rounds of 4 chunks of 16 per
// wave: all waves read their inputs, a barrier, then all write (in place).
// The A loads are vector loads from the pool: a pass with such blocks waits
// for its tile prefetch at the first of them, which is why complex128 blocks
// and K = 6 take this path only in the wide variant (whose prefetch is short
// and whose other blocks are on the vector ALU anyway).
template <int K, typename R, int NT = TT, typename TL>
__device__ __forceinline__ void mfma_block(TL tl, int T, const BlockDev *bd, const R *__restrict__ Asw) {
    using A = typename AmpOf<R>::A;
    using V4 = typename Mfma<R>::V4;
    constexpr int D = 1 << K;
    constexpr int MT = 2 * D / 16;
    constexpr int S = 2 * D / 4;
    constexpr int NB = D / 4;
    constexpr int NW = NT / 64;
    static_assert(MT % NW == 0 || NW % MT == 0, "M-tiles and waves must divide");
    constexpr int MPW = MT > NW ? MT / NW : 1;   // M-tiles per wave
    constexpr int GW = MT / MPW;                 // wave groups (one per M-tile set)
    constexpr int CPW = NW / GW;                 // waves sharing an M-tile set
    constexpr int CR = 4;                        // chunks per wave per round
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gq = lane >> 4, jc = lane & 15;
    const int mt0 = (wave % GW) * MPW, wsub = wave / GW;
    int pos[K];
#pragma unroll
    for (int j = 0; j < K; ++j) pos[j] = bd->pos[j];
    auto deposit = [&](int r) {
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if ((r >> j) & 1) o |= 1u << pos[j];
        return o;
    };
    R a[MPW][S];
#pragma unroll
    for (int i = 0; i < MPW; ++i)
#pragma unroll
        for (int s = 0; s < S; ++s) a[i][s] = Asw[((mt0 + i) * S + s) * 64 + lane];
    uint32_t offB[NB];
#pragma unroll
    for (int m = 0; m < NB; ++m) offB[m] = sw(deposit(4 * m + gq)) * (uint32_t)sizeof(A);
    // byte offset of output (i, q) from the chunk column's amplitude:
    // sw(row offset) amplitudes, plus one real for the imaginary rows
    uint32_t oc[MPW][4];
#pragma unroll
    for (int i = 0; i < MPW; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = 16 * (mt0 + i) + Mfma<R>::row(gq, q);
            oc[i][q] = ((2u * sw(deposit(row % D))) | (uint32_t)(row / D)) * (uint32_t)sizeof(R);
        }
    const uint32_t nchunks = (1u << (T - K)) / 16;
    const uint32_t hj = lane_part<K>(tl, (uint32_t)jc, pos, (uint32_t)sizeof(A));
    for (uint32_t r0 = 0; r0 < nchunks; r0 += CR * CPW) {
        V4 acc[CR][MPW];
        uint32_t cbs[CR];
        // chunks in pairs: two independent accumulator chains per step
#pragma unroll
        for (int i0 = 0; i0 < CR; i0 += 2) {
            A bv[2][NB];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int i = i0 + h;
#pragma unroll
                for (int m = 0; m < MPW; ++m) acc[i][m] = V4{0, 0, 0, 0};
                const uint32_t ch = r0 + wsub + CPW * i;
                const uint32_t cb = hj ^ chunk_part<K>(ch < nchunks ? ch : 0, pos, (uint32_t)sizeof(A));
                cbs[i] = cb;
#pragma unroll
                for (int m = 0; m < NB; ++m) bv[h][m] = *tl.template at<A>(cb, offB[m]);
            }
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int m = 0; m < MPW; ++m)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        acc[i0 + h][m] = Mfma<R>::op(a[m][s], (s & 1) ? bv[h][s >> 1].y : bv[h][s >> 1].x,
                                                     acc[i0 + h][m]);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < CR; ++i) {
            const uint32_t ch = r0 + wsub + CPW * i;
            if (ch < nchunks) {
#pragma unroll
                for (int m = 0; m < MPW; ++m)
#pragma unroll
                    for (int q = 0; q < 4; ++q) *tl.template at<R>(cbs[i], oc[m][q]) = acc[i][m][q];
            }
        }
        __syncthreads();
    }
}

// ---- MFMA block with the A operand in LDS (complex64, K = 3, 4, 5) --------
// The same real GEMM as mfma_block, organised for a pass whose block operands
// were staged in LDS: each wave owns whole 16-column chunks and runs every
// M-tile over them, re-reading A from LDS (16-byte reads, layout
// [M-tile][step/4][lane][4]).  A chunk's inputs are all in registers before
// any of its outputs is written and no other wave touches the chunk, so the
// block needs no barrier of its own.  Output row R = 16 m + 4 (lane/16) + q is
// amplitude R mod 2^K, real part when R < 2^K (K = 3 has one M-tile holding
// both parts); for FP64 the row of item q is 16 m + lane/16 + 4q.  CPI chunks are in flight per wave (CPI * MT accumulator
// chains).
template <int K, typename R, int NT = TT, typename TL>
__device__ __forceinline__ void mfma_block_lds(TL tl, int T, const BlockDev *bd, const R *As) {
    using A = typename AmpOf<R>::A;
    using V4 = typename Mfma<R>::V4;
    constexpr int D = 1 << K;
    constexpr int MT = 2 * D / 16;
    constexpr int S = 2 * D / 4;
    constexpr int NB = D / 4;
    constexpr int CPI = K >= 5 ? 1 : 2;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gq = lane >> 4, jc = lane & 15;
    int pos[K];
#pragma unroll
    for (int j = 0; j < K; ++j) pos[j] = bd->pos[j];
    auto deposit = [&](int r) {
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if ((r >> j) & 1) o |= 1u << pos[j];
        return o;
    };
    uint32_t offB[NB];
#pragma unroll
    for (int m = 0; m < NB; ++m) offB[m] = sw(deposit(4 * m + gq)) * (uint32_t)sizeof(A);
    // byte offset of output (m, q) from the chunk column's amplitude:
    // sw(row offset) amplitudes, plus one real for the imaginary rows
    uint32_t oc[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = 16 * m + Mfma<R>::row(gq, q);
            oc[m][q] = ((2u * sw(deposit(row % D))) | (uint32_t)(row / D)) * (uint32_t)sizeof(R);
        }
    const V4 *A4 = reinterpret_cast<const V4 *>(As);
    const uint32_t nchunks = (1u << (T - K)) / 16;
    const uint32_t hj = lane_part<K>(tl, (uint32_t)jc, pos, (uint32_t)sizeof(A));
    for (uint32_t ch0 = (uint32_t)wave * CPI; ch0 < nchunks; ch0 += (NT / 64) * CPI) {
        uint32_t cb[CPI];
        A bv[CPI][NB];
#pragma unroll
        for (int h = 0; h < CPI; ++h) {
            const uint32_t ch = ch0 + h < nchunks ? ch0 + h : ch0;   // a short last round re-reads a valid chunk
            cb[h] = hj ^ chunk_part<K>(ch, pos, (uint32_t)sizeof(A));
#pragma unroll
            for (int m = 0; m < NB; ++m) bv[h][m] = *tl.template at<A>(cb[h], offB[m]);
        }
        V4 acc[CPI][MT];
#pragma unroll
        for (int h = 0; h < CPI; ++h)
#pragma unroll
            for (int m = 0; m < MT; ++m) acc[h][m] = V4{0, 0, 0, 0};
#pragma unroll
        for (int s4 = 0; s4 < S / 4; ++s4) {
            V4 a[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m) a[m] = A4[(m * (S / 4) + s4) * 64 + lane];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int s = 4 * s4 + u;
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int h = 0; h < CPI; ++h)
                        acc[h][m] = Mfma<R>::op(a[m][u], (s & 1) ? bv[h][s >> 1].y : bv[h][s >> 1].x, acc[h][m]);
            }
        }
#pragma unroll
        for (int h = 0; h < CPI; ++h) {
            if (ch0 + h < nchunks) {
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int q = 0; q < 4; ++q) *tl.template at<R>(cb[h], oc[m][q]) = acc[h][m][q];
            }
        }
    }
}

// ---- complex GEMM with three real products (complex64, K = 4, 5) ------------
// For staged passes the 2^K x 2^K complex block U = Ur + i Ui is applied with
// Gauss's three-multiplication form: T1 = Ur Xr, T2 = Ui Xi,
// T3 = (Ur + Ui)(Xr + Xi); Re Y = T1 - T2, Im Y = T3 - T1 - T2.  That is three
// real 2^K x 2^K GEMMs (3 * 4^K multiply-adds per column) instead of the
// 2^(K+1)-square real embedding (4 * 4^K).  v_mfma_f32_16x16x4f32, step s
// covers K indices 4s..4s+3: lane l supplies A_g[16m + l%16][4s + l/16] and
// X[4s + l/16][column l%16], and holds output rows 16m + Mfma::row(l/16, q) of all
// three products, so it writes complete amplitudes (re, im).  Operand layout
// in LDS: [g = Ur, Ui, Ur+Ui][M-tile][s/4][lane][s%4].  As in mfma_block_lds
// each wave owns whole chunks: no barrier inside the block.  K = 4 keeps all
// of A in registers for the block; K = 5 re-reads it per chunk.
template <int K, typename R, int NT = TT, typename TL>
__device__ __forceinline__ void mfma3m_block_lds(TL tl, int T, const BlockDev *bd, const R *As) {
    using A = typename AmpOf<R>::A;
    using V4 = typename Mfma<R>::V4;
    static_assert(K == 4 || K == 5, "three-product GEMM needs 2^K >= 16");
    constexpr int D = 1 << K;
    constexpr int MT = D / 16;
    constexpr int S = D / 4;
    constexpr int S4 = S / 4;
    constexpr int CPI = K >= 5 ? 1 : 2;
    constexpr bool HOIST = K == 4;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gq = lane >> 4, jc = lane & 15;
    int pos[K];
#pragma unroll
    for (int j = 0; j < K; ++j) pos[j] = bd->pos[j];
    auto deposit = [&](int r) {
        uint32_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if ((r >> j) & 1) o |= 1u << pos[j];
        return o;
    };
    uint32_t offB[S];
#pragma unroll
    for (int s = 0; s < S; ++s) offB[s] = sw(deposit(4 * s + gq)) * (uint32_t)sizeof(A);
    uint32_t oc[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) oc[m][q] = sw(deposit(16 * m + Mfma<R>::row(gq, q))) * (uint32_t)sizeof(A);
    const V4 *A4 = reinterpret_cast<const V4 *>(As);
    auto aidx = [&](int g, int m, int s4) { return ((g * MT + m) * S4 + s4) * 64 + lane; };
    V4 ah[HOIST ? 3 * MT * S4 : 1];
    if constexpr (HOIST) {
#pragma unroll
        for (int g = 0; g < 3; ++g)
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int s4 = 0; s4 < S4; ++s4) ah[(g * MT + m) * S4 + s4] = A4[aidx(g, m, s4)];
    }
    const uint32_t nchunks = (1u << (T - K)) / 16;
    const uint32_t hj = lane_part<K>(tl, (uint32_t)jc, pos, (uint32_t)sizeof(A));
    for (uint32_t ch0 = (uint32_t)wave * CPI; ch0 < nchunks; ch0 += (NT / 64) * CPI) {
        uint32_t cb[CPI];
        A bv[CPI][S];
#pragma unroll
        for (int h = 0; h < CPI; ++h) {
            const uint32_t ch = ch0 + h < nchunks ? ch0 + h : ch0;   // a short last round re-reads a valid chunk
            cb[h] = hj ^ chunk_part<K>(ch, pos, (uint32_t)sizeof(A));
#pragma unroll
            for (int s = 0; s < S; ++s) bv[h][s] = *tl.template at<A>(cb[h], offB[s]);
        }
        V4 acc[CPI][3][MT];
#pragma unroll
        for (int h = 0; h < CPI; ++h)
#pragma unroll
            for (int g = 0; g < 3; ++g)
#pragma unroll
                for (int m = 0; m < MT; ++m) acc[h][g][m] = V4{0, 0, 0, 0};
#pragma unroll
        for (int s4 = 0; s4 < S4; ++s4) {
            V4 a[3][MT];
#pragma unroll
            for (int g = 0; g < 3; ++g)
#pragma unroll
                for (int m = 0; m < MT; ++m) a[g][m] = HOIST ? ah[(g * MT + m) * S4 + s4] : A4[aidx(g, m, s4)];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int s = 4 * s4 + u;
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int h = 0; h < CPI; ++h) {
                        const R xr = bv[h][s].x, xi = bv[h][s].y;
                        acc[h][0][m] = Mfma<R>::op(a[0][m][u], xr, acc[h][0][m]);
                        acc[h][1][m] = Mfma<R>::op(a[1][m][u], xi, acc[h][1][m]);
                        acc[h][2][m] = Mfma<R>::op(a[2][m][u], xr + xi, acc[h][2][m]);
                    }
            }
        }
#pragma unroll
        for (int h = 0; h < CPI; ++h) {
            if (ch0 + h < nchunks) {
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const R t1 = acc[h][0][m][q], t2 = acc[h][1][m][q], t3 = acc[h][2][m][q];
                        A y;
                        y.x = t1 - t2;
                        y.y = t3 - t1 - t2;
                        *tl.template at<A>(cb[h], oc[m][q]) = y;
                    }
            }
        }
    }
}

// ---- permuted block-diagonal block on MFMA (complex64, staged) -----------
// The classes of a block (2^S rows and columns each; the host uses S = 3) are
// taken eight members at a time ("packs": one class of 8, or two of 4); a pack acts
// on its 8 column amplitudes as an 8x8 complex matrix M (zero between
// classes) and writes its 8 row amplitudes.  Its real form is one 16x16
// product per 16 groups: rows and K both ordered (member, re/im), so with
// v_mfma_f32_16x16x4f32 lane l supplies A[l % 16][4 s + l / 16] and, at step s,
// part (l / 16) % 2 of member 2 s + l / 32 of group l % 16; output q of lane l
// is row 4 (l / 16) + q, i.e. both parts of members 2 (l / 16) and
// 2 (l / 16) + 1.  Staged record per pack: A as [lane][s] (256 floats), the
// column offsets ordered members 0,2,4,6 then 1,3,5,7, the row offsets in
// member order (swizzled LDS byte offsets).  A wave owns whole 16-group
// chunks and reads every pack of a chunk before writing any (a pack's rows
// may be another pack's columns), so the block needs no barrier.
constexpr int kBdPackFloats = 256 + 8 + 8;

template <int K, int NT = TT, typename TL>
__device__ __forceinline__ void bdiag_mfma_block(TL tl, int T, const BlockDev *bd, const float *Es) {
    constexpr int NPK = (1 << K) / 8;
    constexpr int CPI = 2;   // chunks in flight per wave
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4, jc = lane & 15;
    int pos[K];
#pragma unroll
    for (int j = 0; j < K; ++j) pos[j] = bd->pos[j];
    // per pack: this lane's A values, its 4 column offsets (with the part's
    // 4-byte shift), its 2 row offsets
    floatx4 a[NPK];
    uint32_t io[NPK][4], oo[NPK][2];
#pragma unroll
    for (int p = 0; p < NPK; ++p) {
        const float *E = Es + p * kBdPackFloats;
        a[p] = reinterpret_cast<const floatx4 *>(E)[lane];
        const uint32_t *ib = reinterpret_cast<const uint32_t *>(E + 256) + 4 * (g >> 1);
#pragma unroll
        for (int s = 0; s < 4; ++s) io[p][s] = ib[s] | (uint32_t)((g & 1) << 2);
        const uint32_t *ob = reinterpret_cast<const uint32_t *>(E + 264) + 2 * g;
        oo[p][0] = ob[0];
        oo[p][1] = ob[1];
    }
    const uint32_t nchunks = (1u << (T - K)) / 16;
    const uint32_t hj = lane_part<K>(tl, (uint32_t)jc, pos, (uint32_t)sizeof(float2));
    for (uint32_t ch0 = (uint32_t)wave * CPI; ch0 < nchunks; ch0 += (NT / 64) * CPI) {
        uint32_t sb[CPI];
        float x[CPI][NPK][4];
#pragma unroll
        for (int h = 0; h < CPI; ++h) {
            const uint32_t ch = ch0 + h < nchunks ? ch0 + h : ch0;   // a short last round re-reads a valid chunk
            sb[h] = hj ^ chunk_part<K>(ch, pos, (uint32_t)sizeof(float2));
#pragma unroll
            for (int p = 0; p < NPK; ++p)
#pragma unroll
                for (int s = 0; s < 4; ++s) x[h][p][s] = *tl.template at<const float>(sb[h], io[p][s]);
        }
        floatx4 acc[CPI][NPK];
#pragma unroll
        for (int h = 0; h < CPI; ++h)
#pragma unroll
            for (int p = 0; p < NPK; ++p) {
                acc[h][p] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    acc[h][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[p][s], x[h][p][s], acc[h][p], 0, 0, 0);
            }
#pragma unroll
        for (int h = 0; h < CPI; ++h) {
            if (ch0 + h < nchunks) {
#pragma unroll
                for (int p = 0; p < NPK; ++p) {
                    *tl.template at<float2>(sb[h], oo[p][0]) = make_float2(acc[h][p][0], acc[h][p][1]);
                    *tl.template at<float2>(sb[h], oo[p][1]) = make_float2(acc[h][p][2], acc[h][p][3]);
                }
            }
        }
    }
}

// ---- permuted block-diagonal block, classes of 2 or 4, on MFMA (complex64, staged)
// 4x4x1 MFMA whose A operand comes from lane quad Q of the wave for all 16
// blocks (broadcast control 4, block Q); Q must be a constant.
template <int Q = 0>
__device__ __forceinline__ floatx4 mfma4x4_bcast(int q, float a, float b, floatx4 c) {
    if constexpr (Q == 15) return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 15, 0);
    else return q == Q ? __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, Q, 0) : mfma4x4_bcast<Q + 1>(q, a, b, c);
}

// Classes of 2^S members (S = 1, 2) of a 4-qubit block on the 16-block
// v_mfma_f32_4x4x1f32: each of its 16 blocks (4 lanes each) forms a 4x4 outer
// product, and lane 4b + j supplies column j of block b (B operand) and holds
// that column of the result.  One lane keeps one group of 16 amplitudes in
// registers, as the vector-ALU class path does, and lane 4b + j's result is
// its own group's.  Class c's real form M_c (2^(S+1) square, rows and
// columns ordered (member, re/im)) is the same for every group, so all 16
// blocks take the A operand (rows 4 r + i, i = 0..3, of row tile r at step
// st) from one lane quad by the MFMA's broadcast control: product
// n = (c * RT + r) * 2^(S+1) + st reads register n / 16 of quad n % 16.  The
// whole of M then sits in 2^S registers per lane, read from LDS once per
// block.  Output register q of row tile r is part q % 2 of member 2 r + q / 2.
// Record: 2^K source and 2^K destination byte offsets (bit patterns, read as
// wave-uniform scalars from the pool), then M as [lane][register] (the
// staged copy in LDS).  The group's reads all precede its writes and no
// other lane touches the group, so the block needs no barrier of its own.
template <int S, int NT = TT, typename TL>
__device__ __forceinline__ void class_mfma_block(TL tl, int T, const BlockDev *bd, const float *__restrict__ E,
                                                 const float *Es) {
    constexpr int K = 4, D = 1 << K, DS = 1 << S, NC = D / DS, K2 = 2 * DS, RT = K2 / 4;
    constexpr int CG = RT == 1 ? 2 : 1;   // classes per round: two accumulator chains either way
    static_assert(S == 1 || S == 2, "classes of 2 or 4");
    using AV = typename std::conditional<S == 2, floatx4, float __attribute__((ext_vector_type(2)))>::type;
    static_assert(NC * RT * K2 == 16 * DS, "one register per quad and product");
    int pos[K];
#pragma unroll
    for (int j = 0; j < K; ++j) pos[j] = bd->pos[j];
    const AV am = reinterpret_cast<const AV *>(Es + 2 * D)[threadIdx.x & 63];   // every lane, before the group loop
    const uint32_t G = 1u << (T - K);
    for (uint32_t g = threadIdx.x; g < G; g += NT) {
        uint32_t b = g;
#pragma unroll
        for (int j = 0; j < K; ++j) b = ins0_32(b, pos[j]);
        const uint32_t h = tl.grp(sw(b) * (uint32_t)sizeof(float2));
        float2 v[D];
#pragma unroll
        for (int i = 0; i < D; ++i) v[i] = *tl.template at<float2>(h, pool_bits(E[i]));
#pragma unroll
        for (int c0 = 0; c0 < NC; c0 += CG) {
            floatx4 acc[CG][RT];
#pragma unroll
            for (int e = 0; e < CG; ++e)
#pragma unroll
                for (int r = 0; r < RT; ++r) acc[e][r] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int st = 0; st < K2; ++st)
#pragma unroll
                for (int e = 0; e < CG; ++e) {
                    const float2 &xm = v[(c0 + e) * DS + st / 2];
                    const float x = st & 1 ? xm.y : xm.x;
#pragma unroll
                    for (int r = 0; r < RT; ++r) {
                        const int n = ((c0 + e) * RT + r) * K2 + st;
                        acc[e][r] = mfma4x4_bcast(n % 16, am[n / 16], x, acc[e][r]);
                    }
                }
#pragma unroll
            for (int e = 0; e < CG; ++e)
#pragma unroll
                for (int r = 0; r < RT; ++r) {
                    const int m = (c0 + e) * DS + 2 * r;
                    *tl.template at<float2>(h, pool_bits(E[D + m])) = make_float2(acc[e][r][0], acc[e][r][1]);
                    *tl.template at<float2>(h, pool_bits(E[D + m + 1])) = make_float2(acc[e][r][2], acc[e][r][3]);
                }
        }
    }
}

// ---- the pass kernel ------------------------------------------------------
// WIDE = false keeps register use low (dense VALU blocks up to k = 3, complex64
// dense k = 4, 5 through MFMA, monomial blocks of any width); WIDE = true adds
// dense VALU blocks with k >= 4.  The host picks the variant per pass.
// CL = true: the pass's block operands were staged in LDS at `cst` (pool
// element cl_off is cst[0]); MFMA blocks (k = 3 embedded, k = 4, 5
// three-product form; FP32 or FP64 matrix cores) and monomial
// blocks with k >= 4 (per-lane records) read them there, dense VALU blocks and
// narrow monomial blocks keep their wave-uniform scalar loads from the pool.
// PG: rotation groups and coefficient forms compiled in (the single-state pass
// kernel); the batch kernel leaves them out to keep its register budget.
template <typename R, bool WIDE, bool CL = false, int NT = TT, bool PG = true, typename TL>
__device__ __forceinline__ void apply_block(TL tile, int T, const BlockDev *bd,
                                            const R *__restrict__ pool, uint64_t gbase, const R *cst = nullptr,
                                            int cl_off = 0) {
    const int k = bd->k;
    const int kind = bd->kind;
    const R *U = pool + bd->mat_off;
    constexpr bool F32 = sizeof(R) == 4;
    if (kind == BK_PAULI) {
        if constexpr (PG) pauli_block<R, NT>(tile, T, U, gbase, bd->sub);
        else pauli_block_m<R, NT, 0>(tile, T, U, gbase);
        return;
    }
    if constexpr (PG) {
        if (kind == BK_PAULIG) {
            if (k == 2) pauli_group<R, 2, NT>(tile, T, U, gbase);
            else pauli_group<R, 3, NT>(tile, T, U, gbase);
            return;
        }
    }
    if constexpr (CL && F32) {
        if (kind == BK_BDMFMA) {
            const float *Es = cst + (bd->mat_off - cl_off);
            if (bd->sub == 3) bdiag_mfma_block<4, NT>(tile, T, bd, Es);
            else if (bd->sub == 2) class_mfma_block<2, NT>(tile, T, bd, U, Es);
            else class_mfma_block<1, NT>(tile, T, bd, U, Es);
            return;
        }
    }
    if (kind == BK_MFMA) {
        if constexpr (CL) {
            const R *As = cst + (bd->mat_off - cl_off);
            if (k == 3) mfma_block_lds<3, R, NT>(tile, T, bd, As);
            else if (k == 4) mfma3m_block_lds<4, R, NT>(tile, T, bd, As);
            else if constexpr (NT > TT) mfma_block_lds<5, R, NT>(tile, T, bd, As);
            else mfma3m_block_lds<5, R, NT>(tile, T, bd, As);
            return;
        } else if constexpr (F32 && !WIDE) {
            if (k == 4) mfma_block<4, R, NT>(tile, T, bd, U);
            else mfma_block<5, R, NT>(tile, T, bd, U);
            return;
        } else if constexpr (WIDE) {
            // the wide variant: complex128 K = 4, 5 and complex64 K = 4..6
            if (k == 4) mfma_block<4, R, NT>(tile, T, bd, U);
            else if (k == 5) mfma_block<5, R, NT>(tile, T, bd, U);
            else if constexpr (F32) mfma_block<6, R, NT>(tile, T, bd, U);
            return;
        }
    }
    if (kind == BK_PERM) {
        perm_block<4, R, NT>(tile, T, bd, U);
        return;
    }
    if (kind == BK_BDIAG) {
        // class widths 1 <= S < K, K = 3, 4; S = 0 for K = 4 monomial blocks
        const int sub = bd->sub;
        if (k == 3) {
            if (sub == 1) bdiag_block<3, 1, R, NT>(tile, T, bd, U);
            else bdiag_block<3, 2, R, NT>(tile, T, bd, U);
        } else if (k == 4) {
            if (sub == 0) bdiag_block<4, 0, R, NT>(tile, T, bd, U);
            else if (sub == 1) bdiag_block<4, 1, R, NT>(tile, T, bd, U);
            else if (sub == 2) bdiag_block<4, 2, R, NT>(tile, T, bd, U);
            else bdiag_block<4, 3, R, NT>(tile, T, bd, U);
        }
        return;
    }
    if (kind == BK_MONO) {
        switch (k) {
        case 1: mono_block<1, R, NT>(tile, T, bd, U); return;
        case 2: mono_block<2, R, NT>(tile, T, bd, U); return;
        case 3: mono_block<3, R, NT>(tile, T, bd, U); return;
        default: break;
        }
        if constexpr (CL) {
            const R *E = cst + (bd->mat_off - cl_off);
            switch (k) {
            case 4: mono_block<4, R, NT>(tile, T, bd, E); return;
            case 5: mono_block<5, R, NT>(tile, T, bd, E); return;
            default: mono_block<6, R, NT>(tile, T, bd, E); return;
            }
        } else {
            switch (k) {
            case 4: mono_block<4, R, NT>(tile, T, bd, U); return;
            case 5: mono_block<5, R, NT>(tile, T, bd, U); return;
            default: mono_block<6, R, NT>(tile, T, bd, U); return;
            }
        }
    }
    switch (k) {
    case 1: valu_block<1, R, NT>(tile, T, bd, U); return;
    case 2: valu_block<2, R, NT>(tile, T, bd, U); return;
    case 3: valu_block<3, R, NT>(tile, T, bd, U); return;
    default: break;
    }
    if constexpr (WIDE) {
        if (k == 4) valu_block<4, R, NT>(tile, T, bd, U);
        else if (k == 5) valu_block<5, R, NT>(tile, T, bd, U);
        if constexpr (F32) {
            if (k == 6) valu_block<6, R, NT>(tile, T, bd, U);
        }
    }
}

}  // namespace tiledev
}  // namespace qs
