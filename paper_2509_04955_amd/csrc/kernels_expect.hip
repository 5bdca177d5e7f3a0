// Pauli-sum expectation on a resident state (the energy of a VQE step,
// Section 1).
//
// For P with X/Y on the bits of x and Z/Y on the bits of z,
//   P|j> = i^{|x&z|} (-1)^{popcount(j&z)} |j^x>,
// so <psi|P|psi> = sum_j conj(psi[j^x]) i^{|x&z|} (-1)^{popcount(j&z)} psi[j].
// Amplitudes are visited in pairs (j, j^x) with the highest bit of x clear,
// so every amplitude is read once per term; with w = conj(psi[j^x]) psi[j]
// and signs s, s' of j and j^x the pair adds i^{|x&z|} (s w + s' conj(w)),
// whose real part is +-(s + s') Re w (even |x&z|) or -+(s - s') Im w (odd).
// Accumulation is FP64; one partial per (term, chunk) workgroup and a fixed
// second-stage sum make the result deterministic.  The grid is laid out
// term-major with a chunk count that is a multiple of 8 where possible, so a
// given chunk of the state is always served by the same XCD (and its L2)
// across terms.
#include <algorithm>

#include "internal.h"

namespace qs {

namespace {

__device__ __forceinline__ uint64_t ins0(uint64_t x, int p) {
    const uint64_t lo = x & ((1ull << p) - 1);
    return ((x - lo) << 1) | lo;
}

template <typename A>
__global__ __launch_bounds__(256) void k_expect(const A *__restrict__ psi, int n, const uint64_t *__restrict__ xs,
                                                const uint64_t *__restrict__ zs, uint32_t nchunks,
                                                double *__restrict__ parts) {
    __shared__ double red[4];
    const uint32_t term = blockIdx.x / nchunks, cid = blockIdx.x % nchunks;
    const uint64_t x = xs[term], z = zs[term];
    double s = 0.0;
    if (x == 0) {
        const uint64_t namps = 1ull << n, chunk = namps / nchunks;
        const uint64_t b0 = (uint64_t)cid * chunk;
        for (uint64_t j = b0 + threadIdx.x; j < b0 + chunk; j += 256) {
            const A a = psi[j];
            const double m = (double)a.x * a.x + (double)a.y * a.y;
            s += (__popcll(j & z) & 1) ? -m : m;
        }
    } else {
        const int h = 63 - __clzll(x);
        const int ny = __popcll(x & z) & 3;
        const uint64_t npairs = 1ull << (n - 1), chunk = npairs / nchunks;
        const uint64_t b0 = (uint64_t)cid * chunk;
        for (uint64_t u = b0 + threadIdx.x; u < b0 + chunk; u += 256) {
            const uint64_t j = ins0(u, h), jp = j ^ x;
            const A a = psi[j], b = psi[jp];
            // w = conj(b) * a
            const double wr = (double)b.x * a.x + (double)b.y * a.y;
            const double wi = (double)b.x * a.y - (double)b.y * a.x;
            const double sj = (__popcll(j & z) & 1) ? -1.0 : 1.0;
            const double sp = (__popcll(jp & z) & 1) ? -1.0 : 1.0;
            double v;
            switch (ny) {
            case 0: v = (sj + sp) * wr; break;
            case 1: v = -(sj - sp) * wi; break;
            case 2: v = -(sj + sp) * wr; break;
            default: v = (sj - sp) * wi; break;
            }
            s += v;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) parts[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void k_expect_reduce(const double *__restrict__ parts, uint32_t nchunks,
                                                       double *__restrict__ terms) {
    __shared__ double sh[256];
    const double *p = parts + (uint64_t)blockIdx.x * nchunks;
    double s = 0;
    for (uint32_t i = threadIdx.x; i < nchunks; i += 256) s += p[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) terms[blockIdx.x] = sh[0];
}

}  // namespace

size_t expect_parts_per_term(int n) {
    // chunks of at least 2048 pairs; at most 512 chunks per term
    const uint64_t npairs = n >= 1 ? (1ull << (n - 1)) : 1;
    uint64_t c = std::max<uint64_t>(1, npairs / 2048);
    c = std::min<uint64_t>(c, 512);
    return (size_t)c;  // a power of two that divides 2^(n-1)
}

qs_status launch_expect(qs_state_s &s, const uint64_t *d_x, const uint64_t *d_z, size_t n_terms, double *d_parts,
                        size_t parts_per_term, double *d_terms) {
    const double S = std::ldexp((double)(s.dtype == QS_C64 ? 8 : 16), s.n);
    prof_begin(s.stream, QS_PROF_EXPECT, S * n_terms, 10.0 * std::ldexp(1.0, s.n) * n_terms);
    const unsigned grid = (unsigned)(n_terms * parts_per_term);
    if (s.dtype == QS_C64)
        hipLaunchKernelGGL(k_expect<float2>, dim3(grid), dim3(256), 0, s.stream, (const float2 *)s.amp, s.n, d_x, d_z,
                           (uint32_t)parts_per_term, d_parts);
    else
        hipLaunchKernelGGL(k_expect<double2>, dim3(grid), dim3(256), 0, s.stream, (const double2 *)s.amp, s.n, d_x,
                           d_z, (uint32_t)parts_per_term, d_parts);
    hipLaunchKernelGGL(k_expect_reduce, dim3((unsigned)n_terms), dim3(256), 0, s.stream, d_parts,
                       (uint32_t)parts_per_term, d_terms);
    prof_end(s.stream);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

}  // namespace qs
