// Pauli-sum expectation on a resident state (the energy of a VQE step,
// Section 1).
//
// For P with X/Y on the bits of x and Z/Y on the bits of z,
//   P|j> = i^{|x&z|} (-1)^{popcount(j&z)} |j^x>,
// so <psi|P|psi> = sum_j conj(psi[j^x]) i^{|x&z|} (-1)^{popcount(j&z)} psi[j].
// Summed over pairs (j, j^x) with w = conj(psi[j^x]) psi[j] and s the sign of
// j, the pair gives 2 s Re w (|x&z| = 0 mod 4), -2 s Im w (1), -2 s Re w (2)
// or 2 s Im w (3).
//
// Reading the state once per group of terms.  Split an index into its low l
// bits (a contiguous tile of 2^l amplitudes) and the high bits H.  The terms
// of a group have high X parts x_h in a span V of dimension at most D; every
// coset H0 + V of the high space (2^D tiles, 2^(l+D) amplitudes) is closed
// under j -> j^x for every term of the group.  One workgroup stages a coset in
// LDS and evaluates all of the group's terms on it, so each group costs one
// read of the state instead of one per term.  Inside a coset an index is
// (a, r): r the tile offset and a_i the coordinate along the i-th basis
// vector v_i of V (reduced echelon form, pivots p_i ascending, so a_i is the
// bit of H at p_i and the coset representative has zeros at every pivot).  A
// term becomes a Pauli on the coset's l + D bits: local x = (coordinates of
// x_h) << l | x_low, local z = (parity(v_i & z_h))_i << l | z_low, times the
// coset's sign parity(H0 & z_h).
//
// Accumulation is FP64: per thread and term over the items it processes, then
// a fixed-order tree per workgroup and a fixed-order sum over workgroups, so
// the result is deterministic.  Complex128 products are FP64; for complex64
// states a pair's Re or Im of conj(c) a is formed in FP32 (relative error
// below 2^-23, so a term's error is at most 2^-23 sum |psi_j psi_{j^x}| <= 2^-24
// for a unit state) and diagonal terms in FP64.  The identity term (the
// squared norm) rides along in the first group at no extra read.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "internal.h"

namespace qs {

namespace {

constexpr int kExpThreads = 1024;   // workgroup of the full-coset variants
constexpr int kExpSmallThreads = 64; // states below the full coset: one wave, cosets of at most 2^10 / 2^9
constexpr int kExpTileBits = 5;      // contiguous amplitudes per tile: 2^5 (256 B complex64); with
                                     // 2^14-amplitude cosets that leaves 9 span dimensions, groups of
                                     // 9 random terms (measured: 23 state reads in 49 ms for 200 terms
                                     // at 30 qubits, against 26 reads in 51 ms with 512 B runs)

__device__ __forceinline__ uint32_t ins0_32(uint32_t x, int p) {
    const uint32_t lo = x & ((1u << p) - 1);
    return ((x - lo) << 1) | lo;
}

__device__ __forceinline__ int par32(uint32_t v) { return __popc(v) & 1; }

// complex amplitude as a native two-element vector (the non-temporal load
// builtin takes native vector types)
typedef float cf2 __attribute__((ext_vector_type(2)));
typedef float cf4 __attribute__((ext_vector_type(4)));   // two complex64 amplitudes
typedef double cd2 __attribute__((ext_vector_type(2)));

// 16-byte load unit per amplitude type: two complex64 or one complex128
template <typename V>
struct LoadUnit;
template <>
struct LoadUnit<cf2> {
    using T = cf4;
    static constexpr int amps = 2;
};
template <>
struct LoadUnit<cd2> {
    using T = cd2;
    static constexpr int amps = 1;
};

template <typename V>
__device__ __forceinline__ V ld_stream(const V *p) {
    return __builtin_nontemporal_load(p);
}

// XOR of the basis vectors selected by the bits of a
__device__ __forceinline__ uint32_t span_vec(const ExpectGroup &g, uint32_t a) {
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < kExpMaxD; ++i)
        if ((a >> i) & 1) v ^= g.v[i];
    return v;
}

// coset representative number c: c's bits spread over the non-pivot positions
__device__ __forceinline__ uint32_t coset_rep(const ExpectGroup &g, uint32_t c, int D) {
    uint32_t r = c;
    for (int i = 0; i < D; ++i) r = ins0_32(r, g.piv[i]);
    return r;
}

// acc[k] += v for a wave-uniform k, keeping every accumulator in registers
__device__ __forceinline__ void add_to(double (&acc)[kExpMaxTerms], int k, double v) {
    switch (k) {
#define QS_ACC_CASE(i) \
    case i: acc[i] += v; break;
        QS_ACC_CASE(0) QS_ACC_CASE(1) QS_ACC_CASE(2) QS_ACC_CASE(3) QS_ACC_CASE(4) QS_ACC_CASE(5) QS_ACC_CASE(6)
        QS_ACC_CASE(7) QS_ACC_CASE(8)
#undef QS_ACC_CASE
    default: break;
    }
}
static_assert(kExpMaxTerms == 9, "add_to lists one case per accumulator");

// Sum over this thread's pairs (j, j^x), j = ins0(t + m T, h) for m < NA/2, of
// sign(j) Re(conj(psi[j^x]) psi[j]) (IMAG: Im), without the thread's own
// sign parity(ins0(t, h) & z).  The LDS reads of H pairs are issued together.
template <typename V, int T, int NA, bool GUARD, bool IMAG>
__device__ __forceinline__ double pair_sum(const V *L, uint32_t t, uint32_t size, const ExpectTerm &tm,
                                           uint32_t lane_j) {
    const char *Lb = (const char *)L;
    const uint32_t lane_off = lane_j * (uint32_t)sizeof(V);
    constexpr int H = NA / 2 < 4 ? NA / 2 : 4;   // pairs whose reads are in flight together
    double P = 0.0;
#pragma unroll
    for (int m0 = 0; m0 < NA / 2; m0 += H) {
        V a[H], c[H];
#pragma unroll
        for (int i = 0; i < H; ++i) {
            if (GUARD && (uint32_t)(m0 + i) * T + t >= size / 2) {
                a[i] = V{0, 0};
                c[i] = V{0, 0};
                continue;
            }
            const uint32_t off = lane_off | tm.jm_off[m0 + i];
            a[i] = *(const V *)(Lb + off);
            c[i] = *(const V *)(Lb + (off ^ tm.x_off));
        }
#pragma unroll
        for (int i = 0; i < H; ++i) {
            double v;
            if constexpr (sizeof(a[i].x) == 4) {
                // complex64: the pair's part of conj(c) a in FP32 (one product and one
                // fused multiply-add: relative error below 2^-23), accumulated in FP64
                v = IMAG ? (double)__builtin_fmaf(c[i].x, a[i].y, -(c[i].y * a[i].x))
                         : (double)__builtin_fmaf(c[i].x, a[i].x, c[i].y * a[i].y);
            } else {
                const double ax = a[i].x, ay = a[i].y, cx = c[i].x, cy = c[i].y;
                v = IMAG ? cx * ay - cy * ax : cx * ax + cy * ay;
            }
            P = fma(tm.sg[m0 + i], v, P);
        }
    }
    return P;
}

// Sum over this thread's amplitudes q = m T + t of sign(q) |psi[q]|^2 for a
// diagonal term (without the thread's own sign parity(t & z)).
template <typename V, int T, int NA, bool GUARD>
__device__ __forceinline__ double diag_sum(const V *L, uint32_t t, uint32_t size, const ExpectTerm &tm) {
    constexpr int H = NA < 4 ? NA : 4;
    double P = 0.0;
#pragma unroll
    for (int m0 = 0; m0 < NA; m0 += H) {
        V a[H];
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const uint32_t q = (uint32_t)(m0 + i) * T + t;
            a[i] = (GUARD && q >= size) ? V{0, 0} : L[q];
        }
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const double mag = (double)a[i].x * (double)a[i].x + (double)a[i].y * (double)a[i].y;
            P = fma(tm.sg[m0 + i], mag, P);
        }
    }
    return P;
}

// One workgroup per (group, coset) item, persistent: workgroup w takes items
// w, w + W, ... (group-major), holding the next item's amplitudes in
// registers while the current one is evaluated from LDS.
//   V   cf2 (complex64) or cd2 (complex128)
//   B   largest coset (log2 amplitudes) the LDS array holds
//   NA  amplitudes each thread stages per item
//   T   threads per workgroup
//   GUARD  the coset may be smaller than T x NA (one-wave variant for small states)
//   LC  tile bits l when fixed at compile time (full cosets), else -1
template <typename V, int B, int T, int NA, bool GUARD, int LC>
__global__ __launch_bounds__(T) void k_expect_coset(
    const V *__restrict__ psi, int l_arg, int D, int b, int log_cosets, uint64_t items,
    const ExpectGroup *__restrict__ groups, const ExpectTerm *__restrict__ terms, int n_terms,
    double *__restrict__ parts) {
    const int l = LC >= 0 ? LC : l_arg;
    static_assert(T * NA == (1 << B), "threads x staged amplitudes = the largest coset");
    __shared__ V L[1 << B];
    __shared__ double red[kExpMaxTerms][T / 64];
    const uint32_t t = threadIdx.x;
    const uint64_t W = gridDim.x, w = blockIdx.x;
    const uint32_t size = 1u << b;            // amplitudes per coset
    const uint32_t lmask = (1u << l) - 1;
    const uint64_t cmask = (1ull << log_cosets) - 1;

    double acc[kExpMaxTerms];
#pragma unroll
    for (int k = 0; k < kExpMaxTerms; ++k) acc[k] = 0.0;

    using LV = typename LoadUnit<V>::T;
    constexpr int AV = LoadUnit<V>::amps;     // amplitudes per 16-byte load
    constexpr int NL = NA / AV;               // loads per thread and item
    LV pre[NL];
    // registers <- the coset of item i: load j of this thread holds amplitudes
    // q = (j T + t) AV + e, e < AV (one tile, since 2^l >= AV)
    auto load_item = [&](uint64_t i) {
        const ExpectGroup &g = groups[i >> log_cosets];
        const uint32_t lane_v = coset_rep(g, (uint32_t)(i & cmask), D) ^ span_vec(g, (t * AV) >> l);
        // amplitude index = ((lane_v ^ mv[j]) << l) | r = lane_idx ^ (mv[j] << l)
        const uint64_t lane_idx = ((uint64_t)lane_v << l) | ((t * AV) & lmask);
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            if (GUARD && ((uint32_t)j * T + t) * AV >= size) break;
            pre[j] = ld_stream((const LV *)(psi + (lane_idx ^ ((uint64_t)g.mv[j] << l))));
        }
    };

    // partials: parts[w][term] for the terms of every group this workgroup
    // has items of (the reduction knows which those are)
    int g_cur = -1;
    auto flush = [&](int gi) {
        const ExpectGroup &g = groups[gi];
        const int nt = g.nterms;
#pragma unroll
        for (int k = 0; k < kExpMaxTerms; ++k) {
            if (k < nt) {
                double v = acc[k];
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
                if ((t & 63) == 0) red[k][t >> 6] = v;
            }
            acc[k] = 0.0;
        }
        __syncthreads();
        const uint32_t nw = T >> 6;
        for (int k = (int)t; k < nt; k += (int)T) {
            double s = 0.0;
            for (uint32_t i = 0; i < nw; ++i) s += red[k][i];
            parts[w * (uint64_t)n_terms + g.term0 + k] = s;
        }
        __syncthreads();
    };

    if (w < items) load_item(w);
    for (uint64_t i = w; i < items; i += W) {
        const int gi = (int)(i >> log_cosets);
        if (gi != g_cur) {
            if (g_cur >= 0) flush(g_cur);
            g_cur = gi;
        }
        const ExpectGroup &g = groups[gi];
        const uint32_t rep = coset_rep(g, (uint32_t)(i & cmask), D);
        __syncthreads();   // the previous item's terms are done with L
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            if (GUARD && ((uint32_t)j * T + t) * AV >= size) break;
            ((LV *)L)[j * T + t] = pre[j];
        }
        __syncthreads();
        if (i + W < items) load_item(i + W);

#pragma unroll 1
        for (int k = 0; k < g.nterms; ++k) {
            const ExpectTerm &tm = terms[g.term0 + k];
            const int sc = par32(rep & tm.zh);
            double P = 0.0;
            int lane_par;
            if (tm.xloc == 0) {
                lane_par = par32(t & tm.zloc);
                P = diag_sum<V, T, NA, GUARD>(L, t, size, tm);
            } else {
                const int h = 31 - __clz(tm.xloc);
                const uint32_t lane_j = ins0_32(t, h);
                lane_par = par32(lane_j & tm.zloc);
                P = tm.imag ? pair_sum<V, T, NA, GUARD, true>(L, t, size, tm, lane_j)
                            : pair_sum<V, T, NA, GUARD, false>(L, t, size, tm, lane_j);
            }
            add_to(acc, k, (lane_par ^ sc) ? -P : P);
        }
    }
    if (g_cur >= 0) flush(g_cur);
}

// out[k] = factor_k * sum of parts[w][k] over the workgroups w that had items
// of term k's group (item i goes to workgroup i mod nw; group g owns items
// [g C, (g + 1) C)), in a fixed order
__global__ __launch_bounds__(256) void k_expect_reduce(const double *__restrict__ parts, uint32_t nw, int n_terms,
                                                       uint64_t cosets, const ExpectTerm *__restrict__ terms,
                                                       double *__restrict__ out) {
    __shared__ double sh[256];
    const int k = blockIdx.x;
    const uint64_t first = (uint64_t)terms[k].group * cosets;   // the group's first item
    double s = 0;
    for (uint32_t i = threadIdx.x; i < nw; i += 256) {
        // offset of workgroup i's first item within the group
        const uint64_t off = ((uint64_t)i + nw - first % nw) % nw;
        if (off < cosets) s += parts[(uint64_t)i * n_terms + k];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = terms[k].factor * sh[0];
}

int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

}  // namespace

// ------------------------------------------------------------ host plan

qs_status expect_plan(int n, qs_dtype dt, const uint64_t *x, const uint64_t *z, size_t n_terms, ExpectPlan &out,
                      uint32_t max_grid) {
    QS_CHECK(n >= 1 && n <= kMaxQubits, QS_EINVAL, "n=%d outside 1..%d", n, kMaxQubits);
    const int bmax = dt == QS_C64 ? kExpCosetBits64 : kExpCosetBits128;
    const int na = dt == QS_C64 ? kExpAmps64 : kExpAmps128;
    ExpectPlan p;
    p.n = n;
    // full cosets of 2^bmax amplitudes when the state holds one; smaller states
    // use one-wave workgroups and cosets of at most 64 x na amplitudes
    p.small = n < bmax;
    p.threads = p.small ? kExpSmallThreads : kExpThreads;
    p.b = p.small ? std::min(n, (int)__builtin_ctz((unsigned)(kExpSmallThreads * na))) : bmax;
    p.l = std::min(kExpTileBits, p.b);
    p.D = p.b - p.l;
    p.log_cosets = n - p.b;
    const int hb = n - p.l;   // high bits
    QS_CHECK(hb <= 32, QS_EUNSUPPORTED, "expectation supports up to %d qubits for this dtype", 32 + p.l);
    // term 0 is the identity (squared norm)
    const size_t NT = n_terms + 1;
    std::vector<uint64_t> X(NT), Z(NT);
    X[0] = Z[0] = 0;
    for (size_t k = 0; k < n_terms; ++k) {
        X[k + 1] = x[k];
        Z[k + 1] = z[k];
    }
    p.terms.resize(NT);
    size_t k0 = 0;
    while (k0 < NT) {
        // greedy: take terms while the span of their high X parts stays within D
        std::vector<uint64_t> basis;   // reduced echelon, pivot = highest bit
        auto reduce = [&](uint64_t v) {
            for (uint64_t e : basis)
                if ((v >> (63 - __builtin_clzll(e))) & 1) v ^= e;
            return v;
        };
        size_t k1 = k0;
        while (k1 < NT && (int)(k1 - k0) < kExpMaxTerms) {
            const uint64_t r = reduce(X[k1] >> p.l);
            if (r) {
                if ((int)basis.size() == p.D) break;
                const int piv = 63 - __builtin_clzll(r);
                for (uint64_t &e : basis)
                    if ((e >> piv) & 1) e ^= r;
                basis.push_back(r);
            }
            ++k1;
        }
        // extend to exactly D vectors with unit vectors at free positions
        for (int pos = 0; (int)basis.size() < p.D && pos < hb; ++pos) {
            bool is_piv = false;
            for (uint64_t e : basis) is_piv |= (63 - __builtin_clzll(e)) == pos;
            if (is_piv) continue;
            const uint64_t u = 1ull << pos;
            for (uint64_t &e : basis)
                if ((e >> pos) & 1) e ^= u;
            basis.push_back(u);
        }
        QS_CHECK((int)basis.size() == p.D, QS_EINVAL, "internal: span basis of size %zu, want %d", basis.size(), p.D);
        std::sort(basis.begin(), basis.end(), [](uint64_t a, uint64_t b) {
            return __builtin_clzll(a) > __builtin_clzll(b);   // ascending pivot
        });
        ExpectGroup g{};
        for (int i = 0; i < p.D; ++i) {
            g.v[i] = (uint32_t)basis[i];
            g.piv[i] = 63 - __builtin_clzll(basis[i]);
        }
        // span vector of the tile coordinate of load m of a thread (the tile of
        // amplitude m * threads * av)
        const int av = dt == QS_C64 ? 2 : 1;
        for (int m = 0; m < kExpMaxAmps; ++m) {
            const uint32_t a = (uint32_t)m * (uint32_t)((p.threads * av) >> p.l);
            uint32_t v = 0;
            for (int i = 0; i < p.D; ++i)
                if ((a >> i) & 1) v ^= g.v[i];
            g.mv[m] = v;
        }
        g.term0 = (int32_t)k0;
        g.nterms = (int32_t)(k1 - k0);
        for (size_t k = k0; k < k1; ++k) {
            const uint64_t xh = X[k] >> p.l, zh = Z[k] >> p.l;
            const uint32_t lm = (1u << p.l) - 1;
            uint32_t xc = 0, zc = 0;
            uint64_t chk = 0;
            for (int i = 0; i < p.D; ++i) {
                if ((xh >> g.piv[i]) & 1) {
                    xc |= 1u << i;
                    chk ^= g.v[i];
                }
                if (__builtin_popcountll(g.v[i] & zh) & 1) zc |= 1u << i;
            }
            QS_CHECK(chk == xh, QS_EINVAL, "internal: term %zu outside its group's span", k);
            ExpectTerm &tm = p.terms[k];
            tm.group = (int32_t)p.groups.size();
            tm.zh = (uint32_t)zh;
            tm.xloc = (xc << p.l) | (uint32_t)(X[k] & lm);
            tm.zloc = (zc << p.l) | (uint32_t)(Z[k] & lm);
            // per staged index m: pair offsets and signs (pairs) or signs (diagonal)
            const uint32_t amp = dt == QS_C64 ? 8 : 16;
            tm.x_off = tm.xloc * amp;
            const int h = tm.xloc ? 31 - __builtin_clz(tm.xloc) : 0;
            for (int m = 0; m < kExpMaxAmps; ++m) {
                const uint32_t u = (uint32_t)m * (uint32_t)p.threads;
                uint32_t j = u;
                if (tm.xloc) {
                    const uint32_t lo = u & ((1u << h) - 1);
                    j = ((u - lo) << 1) | lo;
                    if (m < kExpMaxAmps / 2) tm.jm_off[m] = j * amp;
                }
                tm.sg[m] = (__builtin_popcount(j & tm.zloc) & 1) ? -1.0 : 1.0;
            }
            const int ny = __builtin_popcountll(X[k] & Z[k]) & 3;
            if (X[k] == 0) {
                tm.imag = 0;
                tm.factor = 1.0;   // |x&z| = 0
            } else {
                tm.imag = ny & 1;
                tm.factor = (ny == 0 || ny == 3) ? 2.0 : -2.0;
            }
        }
        p.groups.push_back(g);
        k0 = k1;
    }
    const uint64_t items = (uint64_t)p.groups.size() << p.log_cosets;
    p.items = items;
    uint64_t grid = (uint64_t)device_cus();
    if (max_grid) grid = std::min<uint64_t>(grid, max_grid);
    p.grid = (uint32_t)std::min<uint64_t>(grid, items);
    out = std::move(p);
    return QS_OK;
}

size_t expect_scratch_bytes(const ExpectPlan &p) {
    const size_t NT = p.terms.size();
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    return up(NT * sizeof(ExpectTerm)) + up(p.groups.size() * sizeof(ExpectGroup)) +
           up((size_t)p.grid * NT * sizeof(double)) + up(NT * sizeof(double));
}

qs_status launch_expect(qs_state_s &s, const ExpectPlan &p, void *d_scratch, double **d_out) {
    const size_t NT = p.terms.size();
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    unsigned char *base = (unsigned char *)d_scratch;
    ExpectTerm *d_terms = (ExpectTerm *)base;
    base += up(NT * sizeof(ExpectTerm));
    ExpectGroup *d_groups = (ExpectGroup *)base;
    base += up(p.groups.size() * sizeof(ExpectGroup));
    double *d_parts = (double *)base;
    base += up((size_t)p.grid * NT * sizeof(double));
    double *d_res = (double *)base;
    QS_HIP(hipMemcpyAsync(d_terms, p.terms.data(), NT * sizeof(ExpectTerm), hipMemcpyHostToDevice, s.stream));
    QS_HIP(hipMemcpyAsync(d_groups, p.groups.data(), p.groups.size() * sizeof(ExpectGroup), hipMemcpyHostToDevice,
                          s.stream));
    const double S = std::ldexp((double)(s.dtype == QS_C64 ? 8 : 16), s.n);
    // algorithmic bytes: one read of the state per group; flops: ~10 per pair and term
    prof_begin(s.stream, QS_PROF_EXPECT, S * (double)p.groups.size(), 10.0 * std::ldexp(1.0, s.n) * (double)NT);
    const dim3 grid(p.grid), block(p.threads);
    if (s.dtype == QS_C64) {
        if (p.small)
            hipLaunchKernelGGL((k_expect_coset<cf2, 10, kExpSmallThreads, kExpAmps64, true, -1>), grid, block, 0,
                               s.stream, (const cf2 *)s.amp, p.l, p.D, p.b, p.log_cosets, p.items, d_groups, d_terms,
                               (int)NT, d_parts);
        else
            hipLaunchKernelGGL((k_expect_coset<cf2, kExpCosetBits64, kExpThreads, kExpAmps64, false, kExpTileBits>), grid, block, 0,
                               s.stream, (const cf2 *)s.amp, p.l, p.D, p.b, p.log_cosets, p.items, d_groups, d_terms,
                               (int)NT, d_parts);
    } else {
        if (p.small)
            hipLaunchKernelGGL((k_expect_coset<cd2, 9, kExpSmallThreads, kExpAmps128, true, -1>), grid, block, 0,
                               s.stream, (const cd2 *)s.amp, p.l, p.D, p.b, p.log_cosets, p.items, d_groups, d_terms,
                               (int)NT, d_parts);
        else
            hipLaunchKernelGGL((k_expect_coset<cd2, kExpCosetBits128, kExpThreads, kExpAmps128, false, kExpTileBits>), grid, block,
                               0, s.stream, (const cd2 *)s.amp, p.l, p.D, p.b, p.log_cosets, p.items, d_groups,
                               d_terms, (int)NT, d_parts);
    }
    hipLaunchKernelGGL(k_expect_reduce, dim3((unsigned)NT), dim3(256), 0, s.stream, d_parts, p.grid, (int)NT,
                       (uint64_t)1 << p.log_cosets, d_terms, d_res);
    prof_end(s.stream);
    QS_HIP(hipGetLastError());
    *d_out = d_res;
    return QS_OK;
}

// ------------------------------------------------- library-held scratch
// Device memory for qs_expect_pauli_sum_noalloc: term and group tables,
// per-workgroup partials and results of one launch of at most
// kNoAllocMaxTerms caller terms.  Every device the library runs on holds one
// copy until the process ends.  Nothing in it needs clearing between calls:
// the tables are copied in whole, each partial the reduction reads is written
// by the same launch, and the results are written by the reduction.
namespace {

constexpr size_t up256(size_t v) { return (v + 255) / 256 * 256; }
constexpr size_t kNoAllocScratchBytes =
    up256((kNoAllocMaxTerms + 1) * sizeof(ExpectTerm)) + up256((kNoAllocMaxTerms + 1) * sizeof(ExpectGroup)) +
    up256((size_t)kNoAllocMaxGrid * (kNoAllocMaxTerms + 1) * sizeof(double)) +
    up256((kNoAllocMaxTerms + 1) * sizeof(double));

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

qs_status noalloc_scratch(size_t need, void **ptr) {
    QS_CHECK(need <= kNoAllocScratchBytes, QS_ERANGE, "scratch of %zu bytes exceeds the %zu held", need,
             kNoAllocScratchBytes);
    int dev = 0;
    QS_HIP(hipGetDevice(&dev));
    QS_CHECK(dev >= 0 && dev < kMaxDevices, QS_EDEVICE, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        // the array's device address on the current device (its host-side name
        // is not a device address)
        void *p = nullptr;
        QS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        QS_CHECK(p != nullptr, QS_EDEVICE, "scratch has no device address");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return QS_OK;
}

std::mutex &noalloc_lock() {
    static std::mutex mu;
    return mu;
}

}  // namespace qs
