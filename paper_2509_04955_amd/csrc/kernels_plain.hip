// Plain gate-by-gate kernels: one sweep of the state per gate.
//
// This is the baseline form of the method: every gate is one pass over the
// amplitude pairs it touches (Section 2.2, Algorithms 1-4; Section 3.3, the
// one-thread-per-pair mapping).  On gfx950 it is laid out for 64-wide waves:
//   * complex64 amplitudes move as 16-byte vectors (two adjacent amplitudes);
//   * target qubit 0 is handled inside a lane (both pair members in one vector);
//   * target qubits 1..6 keep every wave's loads fully contiguous and fetch the
//     partner amplitude from lane ^ 2^(q-1) with a cross-lane shuffle;
//   * higher targets load the two strided 16-byte halves of each pair directly
//     (coalesced: each half is a contiguous 1 KiB run per wave);
//   * controlled gates visit only the control = 1 half (Eq. 4), diagonal and
//     phase gates only the amplitudes they change.
#include <cmath>
#include <cstdlib>

#include "internal.h"

namespace qs {

namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 4;
constexpr uint64_t kMaxGrid = 1u << 20;

__device__ __forceinline__ uint64_t ins0(uint64_t x, int p) {
    const uint64_t lo = x & ((1ull << p) - 1);
    return ((x - lo) << 1) | lo;
}

template <typename R>
struct M2 {
    R ur[4], ui[4];
};

// Each sweep reads and writes every amplitude it touches once: 16-byte
// accesses are issued non-temporal so they do not displace cache contents.
typedef float nt4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld_nt(const float4 *p) {
    const nt4 v = __builtin_nontemporal_load(reinterpret_cast<const nt4 *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st_nt(float4 *p, float4 v) {
    const nt4 w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<nt4 *>(p));
}

// (x, y) = U (a, b) for complex a, b.
template <typename R>
__device__ __forceinline__ void apply2(const M2<R> &m, R ar, R ai, R br, R bi, R &xr, R &xi, R &yr, R &yi) {
    xr = m.ur[0] * ar - m.ui[0] * ai + m.ur[1] * br - m.ui[1] * bi;
    xi = m.ur[0] * ai + m.ui[0] * ar + m.ur[1] * bi + m.ui[1] * br;
    yr = m.ur[2] * ar - m.ui[2] * ai + m.ur[3] * br - m.ui[3] * bi;
    yi = m.ur[2] * ai + m.ui[2] * ar + m.ur[3] * bi + m.ui[3] * br;
}

#define UNIT_LOOP(units)                                                                    \
    for (uint64_t base_ = (uint64_t)blockIdx.x * (kThreads * kUnroll); base_ < (units);    \
         base_ += (uint64_t)gridDim.x * (kThreads * kUnroll))

// ---- one-qubit dense, complex64 ---------------------------------------
// target 0: the pair is one 16-byte vector.
__global__ __launch_bounds__(kThreads) void k_1q_c64_q0(float4 *__restrict__ psi, uint64_t units, M2<float> m) {
    UNIT_LOOP(units) {
        float4 v[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < units) v[j] = ld_nt(psi + u);
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < units) {
                float4 o;
                apply2(m, v[j].x, v[j].y, v[j].z, v[j].w, o.x, o.y, o.z, o.w);
                st_nt(psi + u, o);
            }
        }
    }
}

// target q >= 1: two 16-byte vectors at i and i + 2^q hold two pairs.
__global__ __launch_bounds__(kThreads) void k_1q_c64_pair(float2 *__restrict__ psi, int q, uint64_t units,
                                                          M2<float> m) {
    const uint64_t stride = 1ull << q;
    UNIT_LOOP(units) {
        float4 a[kUnroll], b[kUnroll];
        uint64_t idx[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            idx[j] = ins0(u << 1, q);
            if (u < units) {
                a[j] = ld_nt(reinterpret_cast<const float4 *>(psi + idx[j]));
                b[j] = ld_nt(reinterpret_cast<const float4 *>(psi + idx[j] + stride));
            }
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < units) {
                float4 x, y;
                apply2(m, a[j].x, a[j].y, b[j].x, b[j].y, x.x, x.y, y.x, y.y);
                apply2(m, a[j].z, a[j].w, b[j].z, b[j].w, x.z, x.w, y.z, y.w);
                st_nt(reinterpret_cast<float4 *>(psi + idx[j]), x);
                st_nt(reinterpret_cast<float4 *>(psi + idx[j] + stride), y);
            }
        }
    }
}

// target 1 <= q <= 6: every lane loads the 16-byte vector it owns (fully
// contiguous per wave); the partner vector comes from lane ^ 2^(q-1).
// Requires units to be a multiple of 64 (whole waves).
__global__ __launch_bounds__(kThreads) void k_1q_c64_shfl(float4 *__restrict__ psi, int q, uint64_t units,
                                                          M2<float> m) {
    const int lx = 1 << (q - 1);
    UNIT_LOOP(units) {
        float4 v[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < units) v[j] = ld_nt(psi + u);
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < units) {  // uniform per wave
                float4 p;
                p.x = __shfl_xor(v[j].x, lx);
                p.y = __shfl_xor(v[j].y, lx);
                p.z = __shfl_xor(v[j].z, lx);
                p.w = __shfl_xor(v[j].w, lx);
                const bool upper = (u >> (q - 1)) & 1;  // bit q of the amplitude index
                float4 o;
                float dr, di;
                if (!upper) {
                    apply2(m, v[j].x, v[j].y, p.x, p.y, o.x, o.y, dr, di);
                    apply2(m, v[j].z, v[j].w, p.z, p.w, o.z, o.w, dr, di);
                } else {
                    apply2(m, p.x, p.y, v[j].x, v[j].y, dr, di, o.x, o.y);
                    apply2(m, p.z, p.w, v[j].z, v[j].w, dr, di, o.z, o.w);
                }
                st_nt(psi + u, o);
            }
        }
    }
}

// ---- one-qubit dense, complex128 --------------------------------------
__global__ __launch_bounds__(kThreads) void k_1q_c128(double2 *__restrict__ psi, int q, uint64_t units,
                                                      M2<double> m) {
    const uint64_t stride = 1ull << q;
    UNIT_LOOP(units) {
        double2 a[kUnroll], b[kUnroll];
        uint64_t idx[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            idx[j] = ins0(u, q);
            if (u < units) {
                a[j] = psi[idx[j]];
                b[j] = psi[idx[j] + stride];
            }
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < units) {
                double2 x, y;
                apply2(m, a[j].x, a[j].y, b[j].x, b[j].y, x.x, x.y, y.x, y.y);
                psi[idx[j]] = x;
                psi[idx[j] + stride] = y;
            }
        }
    }
}

// ---- controlled one-qubit (Eq. 4: control = 1 half only) --------------
// complex64, control and target >= 1: vectors of two adjacent pairs.
__global__ __launch_bounds__(kThreads) void k_ctrl_c64_vec(float2 *__restrict__ psi, int c, int t, uint64_t units,
                                                           M2<float> m) {
    const int lo = c < t ? c : t, hi = c < t ? t : c;
    const uint64_t stride = 1ull << t, cm = 1ull << c;
    UNIT_LOOP(units) {
        float4 a[kUnroll], b[kUnroll];
        uint64_t idx[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            idx[j] = ins0(ins0(u << 1, lo), hi) | cm;
            if (u < units) {
                a[j] = ld_nt(reinterpret_cast<const float4 *>(psi + idx[j]));
                b[j] = ld_nt(reinterpret_cast<const float4 *>(psi + idx[j] + stride));
            }
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < units) {
                float4 x, y;
                apply2(m, a[j].x, a[j].y, b[j].x, b[j].y, x.x, x.y, y.x, y.y);
                apply2(m, a[j].z, a[j].w, b[j].z, b[j].w, x.z, x.w, y.z, y.w);
                st_nt(reinterpret_cast<float4 *>(psi + idx[j]), x);
                st_nt(reinterpret_cast<float4 *>(psi + idx[j] + stride), y);
            }
        }
    }
}

// complex64, control c <= 3 and target t >= 1: the control = 1 runs are at
// most 8 amplitudes (64 bytes) long, so touching only them leaves every HBM
// burst half used.  This variant sweeps every pair in whole 16-byte vectors
// (2S bytes, the one-qubit sweep's pattern) and writes the control = 0 pairs
// back unchanged.  Bit 0 of a vector's first index is 0 and bit t is 0 for a,
// 1 for b, so for c >= 1 bit c of idx is the control of all four amplitudes;
// for c = 0 only the second amplitude of each vector has the control set.
__global__ __launch_bounds__(kThreads) void k_ctrl_c64_sweep(float2 *__restrict__ psi, int c, int t, uint64_t units,
                                                             M2<float> m) {
    const uint64_t stride = 1ull << t;
    UNIT_LOOP(units) {
        float4 a[kUnroll], b[kUnroll];
        uint64_t idx[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            idx[j] = ins0(u << 1, t);
            if (u < units) {
                a[j] = ld_nt(reinterpret_cast<const float4 *>(psi + idx[j]));
                b[j] = ld_nt(reinterpret_cast<const float4 *>(psi + idx[j] + stride));
            }
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < units) {
                float4 x = a[j], y = b[j];
                if (c == 0) {
                    apply2(m, a[j].z, a[j].w, b[j].z, b[j].w, x.z, x.w, y.z, y.w);
                } else if ((idx[j] >> c) & 1) {
                    apply2(m, a[j].x, a[j].y, b[j].x, b[j].y, x.x, x.y, y.x, y.y);
                    apply2(m, a[j].z, a[j].w, b[j].z, b[j].w, x.z, x.w, y.z, y.w);
                }
                st_nt(reinterpret_cast<float4 *>(psi + idx[j]), x);
                st_nt(reinterpret_cast<float4 *>(psi + idx[j] + stride), y);
            }
        }
    }
}

// The same sweep for targets 1 <= t <= 6: k_1q_c64_shfl's lane exchange
// (vector u holds amplitudes 2u, 2u + 1), then the control = 0 outputs take
// the loaded values back.  Requires units to be a multiple of 64.
__global__ __launch_bounds__(kThreads) void k_ctrl_c64_shfl(float4 *__restrict__ psi, int c, int t, uint64_t units,
                                                            M2<float> m) {
    const int lx = 1 << (t - 1);
    UNIT_LOOP(units) {
        float4 v[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < units) v[j] = ld_nt(psi + u);
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < units) {  // uniform per wave
                float4 p;
                p.x = __shfl_xor(v[j].x, lx);
                p.y = __shfl_xor(v[j].y, lx);
                p.z = __shfl_xor(v[j].z, lx);
                p.w = __shfl_xor(v[j].w, lx);
                const bool upper = (u >> (t - 1)) & 1;  // bit t of the amplitude index
                float4 o;
                float dr, di;
                if (!upper) {
                    apply2(m, v[j].x, v[j].y, p.x, p.y, o.x, o.y, dr, di);
                    apply2(m, v[j].z, v[j].w, p.z, p.w, o.z, o.w, dr, di);
                } else {
                    apply2(m, p.x, p.y, v[j].x, v[j].y, dr, di, o.x, o.y);
                    apply2(m, p.z, p.w, v[j].z, v[j].w, dr, di, o.z, o.w);
                }
                if (c == 0) {
                    o.x = v[j].x;
                    o.y = v[j].y;
                } else if (!(((u << 1) >> c) & 1)) {
                    o = v[j];
                }
                st_nt(psi + u, o);
            }
        }
    }
}

// any control/target, one pair per unit.
template <typename R, typename A>
__global__ __launch_bounds__(kThreads) void k_ctrl_scalar(A *__restrict__ psi, int c, int t, uint64_t units, M2<R> m) {
    const int lo = c < t ? c : t, hi = c < t ? t : c;
    const uint64_t stride = 1ull << t, cm = 1ull << c;
    UNIT_LOOP(units) {
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < units) {
                uint64_t i = ins0(ins0(u, lo), hi) | cm;
                A a = psi[i], b = psi[i + stride], x, y;
                apply2(m, a.x, a.y, b.x, b.y, x.x, x.y, y.x, y.y);
                psi[i] = x;
                psi[i + stride] = y;
            }
        }
    }
}

// ---- phase on the subspace where every bit of a mask is 1 -------------
// (Z, S, T, P on one qubit; CZ, CP on two.)  np <= 2 positions, ascending.
template <typename R, typename A>
__global__ __launch_bounds__(kThreads) void k_phase(A *__restrict__ psi, int np, int p0, int p1, uint64_t units,
                                                    R pr, R pi) {
    UNIT_LOOP(units) {
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < units) {
                uint64_t i = ins0(u, p0) | (1ull << p0);
                if (np == 2) i = ins0(i, p1) | (1ull << p1);
                A a = psi[i], o;
                o.x = a.x * pr - a.y * pi;
                o.y = a.x * pi + a.y * pr;
                psi[i] = o;
            }
        }
    }
}

// complex64, bit 0 not in the mask: two adjacent amplitudes per vector.
__global__ __launch_bounds__(kThreads) void k_phase_c64_vec(float2 *__restrict__ psi, int np, int p0, int p1,
                                                            uint64_t units, float pr, float pi) {
    UNIT_LOOP(units) {
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < units) {
                uint64_t i = ins0(u << 1, p0) | (1ull << p0);
                if (np == 2) i = ins0(i, p1) | (1ull << p1);
                float4 a = *reinterpret_cast<const float4 *>(psi + i), o;
                o.x = a.x * pr - a.y * pi;
                o.y = a.x * pi + a.y * pr;
                o.z = a.z * pr - a.w * pi;
                o.w = a.z * pi + a.w * pr;
                *reinterpret_cast<float4 *>(psi + i) = o;
            }
        }
    }
}

// ---- general one-qubit diagonal (RZ): every amplitude times d[bit q] ----
template <typename R, typename A>
__global__ __launch_bounds__(kThreads) void k_diag1(A *__restrict__ psi, int q, uint64_t units, R d0r, R d0i, R d1r,
                                                    R d1i) {
    UNIT_LOOP(units) {
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < units) {
                const bool b = (u >> q) & 1;
                const R dr = b ? d1r : d0r, di = b ? d1i : d0i;
                A a = psi[u], o;
                o.x = a.x * dr - a.y * di;
                o.y = a.x * di + a.y * dr;
                psi[u] = o;
            }
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_diag1_c64_vec(float4 *__restrict__ psi, int q, uint64_t units, float d0r,
                                                            float d0i, float d1r, float d1i) {
    UNIT_LOOP(units) {
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < units) {
                // amplitudes 2u (bit q of 2u) and 2u + 1
                const bool b0 = ((u << 1) >> q) & 1, b1 = (((u << 1) | 1) >> q) & 1;
                const float ar = b0 ? d1r : d0r, ai = b0 ? d1i : d0i;
                const float br = b1 ? d1r : d0r, bi = b1 ? d1i : d0i;
                float4 a = psi[u], o;
                o.x = a.x * ar - a.y * ai;
                o.y = a.x * ai + a.y * ar;
                o.z = a.z * br - a.w * bi;
                o.w = a.z * bi + a.w * br;
                psi[u] = o;
            }
        }
    }
}

// ---- SWAP: exchange |..1_a..0_b..> and |..0_a..1_b..> ----------------
template <typename A>
__global__ __launch_bounds__(kThreads) void k_swap(A *__restrict__ psi, int a, int b, uint64_t units) {
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    UNIT_LOOP(units) {
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < units) {
                uint64_t i = ins0(ins0(u, lo), hi) | (1ull << a);
                uint64_t k = i ^ (1ull << a) ^ (1ull << b);
                A x = psi[i], y = psi[k];
                psi[i] = y;
                psi[k] = x;
            }
        }
    }
}

// ---- dense k-qubit gate from global memory (plain DENSE gates) --------
// One group of 2^K amplitudes per thread; U row-major complex (re, im).
template <int K, typename R, typename A>
__global__ __launch_bounds__(kThreads) void k_dense(A *__restrict__ psi, int4 posA, int2 posB, uint64_t units,
                                                    const R *__restrict__ U) {
    constexpr int D = 1 << K;
    const int pos[6] = {posA.x, posA.y, posA.z, posA.w, posB.x, posB.y};
    int sorted[6];
    for (int j = 0; j < K; ++j) sorted[j] = pos[j];
    for (int i = 0; i < K; ++i)
        for (int j = i + 1; j < K; ++j)
            if (sorted[j] < sorted[i]) {
                int tmp = sorted[i];
                sorted[i] = sorted[j];
                sorted[j] = tmp;
            }
    for (uint64_t u = (uint64_t)blockIdx.x * kThreads + threadIdx.x; u < units; u += (uint64_t)gridDim.x * kThreads) {
        uint64_t b = u;
        for (int j = 0; j < K; ++j) b = ins0(b, sorted[j]);
        A v[D];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            uint64_t o = 0;
#pragma unroll
            for (int j = 0; j < K; ++j)
                if ((r >> j) & 1) o |= 1ull << pos[j];
            v[r] = psi[b | o];
        }
#pragma unroll
        for (int r = 0; r < D; ++r) {
            R yr = 0, yi = 0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const R ur = U[2 * (r * D + c)], ui = U[2 * (r * D + c) + 1];
                yr += ur * v[c].x - ui * v[c].y;
                yi += ur * v[c].y + ui * v[c].x;
            }
            uint64_t o = 0;
#pragma unroll
            for (int j = 0; j < K; ++j)
                if ((r >> j) & 1) o |= 1ull << pos[j];
            A y;
            y.x = yr;
            y.y = yi;
            psi[b | o] = y;
        }
    }
}

// ---- whole-state helpers ----------------------------------------------
template <typename R, typename A>
__global__ __launch_bounds__(kThreads) void k_scale(A *__restrict__ psi, uint64_t units, const double *__restrict__ sc) {
    const R s = (R)(*sc);
    UNIT_LOOP(units) {
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < units) {
                A a = psi[u];
                a.x *= s;
                a.y *= s;
                psi[u] = a;
            }
        }
    }
}

// zero 16-byte words, then write 1 at `index`
__global__ __launch_bounds__(kThreads) void k_fill_basis(uint4 *__restrict__ w, uint64_t words, int dtype,
                                                         uint64_t index) {
    UNIT_LOOP(words) {
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < words) {
                uint4 z = make_uint4(0, 0, 0, 0);
                if (dtype == QS_C64) {
                    if ((index >> 1) == u) {
                        if (index & 1) z.z = 0x3f800000u;
                        else z.x = 0x3f800000u;
                    }
                } else if (index == u) {
                    z.y = 0x3ff00000u;  // 1.0 as double (high word)
                }
                w[u] = z;
            }
        }
    }
}

template <bool NT>
__global__ __launch_bounds__(kThreads) void k_copy(float4 *__restrict__ dst, const float4 *__restrict__ src,
                                                   uint64_t words) {
    UNIT_LOOP(words) {
        float4 v[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < words) v[j] = NT ? ld_nt(src + u) : src[u];
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint64_t u = base_ + j * kThreads + threadIdx.x;
            if (u < words) {
                if (NT) st_nt(dst + u, v[j]);
                else dst[u] = v[j];
            }
        }
    }
}

dim3 grid_for(uint64_t units, int per_thread = kUnroll) {
    uint64_t g = (units + (uint64_t)kThreads * per_thread - 1) / ((uint64_t)kThreads * per_thread);
    if (g < 1) g = 1;
    if (g > kMaxGrid) g = kMaxGrid;
    return dim3((unsigned)g);
}

template <typename R>
M2<R> to_m2(const HGate &g, int r0, int r1, int c0, int c1, int d) {
    M2<R> m;
    const int rr[2] = {r0, r1}, cc[2] = {c0, c1};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            cd v = g.m[(size_t)rr[a] * d + cc[b]];
            m.ur[2 * a + b] = (R)v.real();
            m.ui[2 * a + b] = (R)v.imag();
        }
    return m;
}

bool is_zero(cd v) { return v.real() == 0.0 && v.imag() == 0.0; }
bool is_one(cd v) { return v.real() == 1.0 && v.imag() == 0.0; }

bool use_shuffle() {
    static int v = -1;
    if (v < 0) {
        const char *e = getenv("QS_PLAIN_SHUFFLE");
        v = e ? atoi(e) != 0 : 1;
    }
    return v == 1;
}

// complex64 controlled gates with a low control: whole-vector sweep
// (QS_PLAIN_CTRL_SWEEP=0: the control-half kernels)
bool ctrl_sweep_enabled() {
    static int v = -1;
    if (v < 0) {
        const char *e = getenv("QS_PLAIN_CTRL_SWEEP");
        v = e ? atoi(e) != 0 : 1;
    }
    return v == 1;
}

// device copy of a dense matrix for k_dense (kept alive for the process:
// one small cached buffer per (dtype) sized to the largest matrix seen).
struct DenseScratch {
    void *ptr = nullptr;
    size_t cap = 0;
};
DenseScratch g_dense[2];

}  // namespace

qs_status launch_plain(qs_state_s &s, const HGate &g) {
    const int n = s.n;
    const double S = std::ldexp((double)(s.dtype == QS_C64 ? 8 : 16), n);
    hipStream_t st = s.stream;
    const bool c64 = s.dtype == QS_C64;
    if (g.nq == 1 || (g.kind == QS_DENSE && g.nq == 1)) {
        const int q = g.q[0];
        if (is_zero(g.m[1]) && is_zero(g.m[2])) {
            if (is_one(g.m[0])) {  // phase on bit q = 1: half the state, S bytes
                if (is_one(g.m[3])) return QS_OK;
                const double pr = g.m[3].real(), pi = g.m[3].imag();
                prof_begin(st, QS_PROF_PLAIN, S, 6.0 * std::ldexp(1.0, n - 1));
                if (c64 && q >= 1) {
                    uint64_t units = 1ull << (n - 2);
                    hipLaunchKernelGGL(k_phase_c64_vec, grid_for(units), dim3(kThreads), 0, st, (float2 *)s.amp, 1, q,
                                       0, units, (float)pr, (float)pi);
                } else if (c64) {
                    uint64_t units = 1ull << (n - 1);
                    hipLaunchKernelGGL((k_phase<float, float2>), grid_for(units), dim3(kThreads), 0, st,
                                       (float2 *)s.amp, 1, q, 0, units, (float)pr, (float)pi);
                } else {
                    uint64_t units = 1ull << (n - 1);
                    hipLaunchKernelGGL((k_phase<double, double2>), grid_for(units), dim3(kThreads), 0, st,
                                       (double2 *)s.amp, 1, q, 0, units, pr, pi);
                }
                prof_end(st);
                QS_HIP(hipGetLastError());
                return QS_OK;
            }
            // general diagonal (RZ): every amplitude, 2S bytes
            prof_begin(st, QS_PROF_PLAIN, 2 * S, 6.0 * std::ldexp(1.0, n));
            if (c64 && n >= 1) {
                uint64_t units = 1ull << (n - 1);
                hipLaunchKernelGGL(k_diag1_c64_vec, grid_for(units), dim3(kThreads), 0, st, (float4 *)s.amp, q, units,
                                   (float)g.m[0].real(), (float)g.m[0].imag(), (float)g.m[3].real(),
                                   (float)g.m[3].imag());
            } else {
                uint64_t units = 1ull << n;
                hipLaunchKernelGGL((k_diag1<double, double2>), grid_for(units), dim3(kThreads), 0, st,
                                   (double2 *)s.amp, q, units, g.m[0].real(), g.m[0].imag(), g.m[3].real(),
                                   g.m[3].imag());
            }
            prof_end(st);
        } else {
            prof_begin(st, QS_PROF_PLAIN, 2 * S, 14.0 * std::ldexp(1.0, n));
            if (c64) {
                M2<float> m = to_m2<float>(g, 0, 1, 0, 1, 2);
                if (q == 0) {
                    uint64_t units = 1ull << (n - 1);
                    hipLaunchKernelGGL(k_1q_c64_q0, grid_for(units), dim3(kThreads), 0, st, (float4 *)s.amp, units, m);
                } else if (q <= 6 && n >= 7 && use_shuffle()) {
                    uint64_t units = 1ull << (n - 1);
                    hipLaunchKernelGGL(k_1q_c64_shfl, grid_for(units), dim3(kThreads), 0, st, (float4 *)s.amp, q,
                                       units, m);
                } else {
                    uint64_t units = 1ull << (n - 2);
                    hipLaunchKernelGGL(k_1q_c64_pair, grid_for(units), dim3(kThreads), 0, st, (float2 *)s.amp, q,
                                       units, m);
                }
            } else {
                M2<double> m = to_m2<double>(g, 0, 1, 0, 1, 2);
                uint64_t units = 1ull << (n - 1);
                hipLaunchKernelGGL(k_1q_c128, grid_for(units), dim3(kThreads), 0, st, (double2 *)s.amp, q, units, m);
            }
            prof_end(st);
        }
        QS_HIP(hipGetLastError());
        return QS_OK;
    }
    if (g.kind == QS_CNOT || g.kind == QS_CU || g.kind == QS_CZ || g.kind == QS_CP) {
        const int c = g.q[0], t = g.q[1];
        // local index: bit 0 = control, bit 1 = target; control-1 rows are 1 and 3
        if (g.kind == QS_CZ || g.kind == QS_CP) {
            const cd ph = g.m[3 * 4 + 3];
            const int p0 = c < t ? c : t, p1 = c < t ? t : c;
            prof_begin(st, QS_PROF_PLAIN, S / 2, 6.0 * std::ldexp(1.0, n - 2));
            if (c64 && p0 >= 1) {
                uint64_t units = 1ull << (n - 3);
                hipLaunchKernelGGL(k_phase_c64_vec, grid_for(units), dim3(kThreads), 0, st, (float2 *)s.amp, 2, p0,
                                   p1, units, (float)ph.real(), (float)ph.imag());
            } else if (c64) {
                uint64_t units = 1ull << (n - 2);
                hipLaunchKernelGGL((k_phase<float, float2>), grid_for(units), dim3(kThreads), 0, st, (float2 *)s.amp,
                                   2, p0, p1, units, (float)ph.real(), (float)ph.imag());
            } else {
                uint64_t units = 1ull << (n - 2);
                hipLaunchKernelGGL((k_phase<double, double2>), grid_for(units), dim3(kThreads), 0, st,
                                   (double2 *)s.amp, 2, p0, p1, units, ph.real(), ph.imag());
            }
            prof_end(st);
            QS_HIP(hipGetLastError());
            return QS_OK;
        }
        prof_begin(st, QS_PROF_PLAIN, S, 14.0 * std::ldexp(1.0, n - 1));
        if (c64) {
            M2<float> m = to_m2<float>(g, 1, 3, 1, 3, 4);
            if (c <= 3 && t >= 1 && t <= 6 && n >= 7 && use_shuffle() && ctrl_sweep_enabled()) {
                uint64_t units = 1ull << (n - 1);
                hipLaunchKernelGGL(k_ctrl_c64_shfl, grid_for(units), dim3(kThreads), 0, st, (float4 *)s.amp, c, t,
                                   units, m);
            } else if (c <= 3 && t >= 1 && ctrl_sweep_enabled()) {
                uint64_t units = 1ull << (n - 2);
                hipLaunchKernelGGL(k_ctrl_c64_sweep, grid_for(units), dim3(kThreads), 0, st, (float2 *)s.amp, c, t,
                                   units, m);
            } else if (c >= 1 && t >= 1) {
                uint64_t units = 1ull << (n - 3);
                hipLaunchKernelGGL(k_ctrl_c64_vec, grid_for(units), dim3(kThreads), 0, st, (float2 *)s.amp, c, t,
                                   units, m);
            } else {
                uint64_t units = 1ull << (n - 2);
                hipLaunchKernelGGL((k_ctrl_scalar<float, float2>), grid_for(units), dim3(kThreads), 0, st,
                                   (float2 *)s.amp, c, t, units, m);
            }
        } else {
            M2<double> m = to_m2<double>(g, 1, 3, 1, 3, 4);
            uint64_t units = 1ull << (n - 2);
            hipLaunchKernelGGL((k_ctrl_scalar<double, double2>), grid_for(units), dim3(kThreads), 0, st,
                               (double2 *)s.amp, c, t, units, m);
        }
        prof_end(st);
        QS_HIP(hipGetLastError());
        return QS_OK;
    }
    if (g.kind == QS_SWAP) {
        uint64_t units = 1ull << (n - 2);
        prof_begin(st, QS_PROF_PLAIN, S, 0);
        if (c64)
            hipLaunchKernelGGL(k_swap<float2>, grid_for(units), dim3(kThreads), 0, st, (float2 *)s.amp, g.q[0],
                               g.q[1], units);
        else
            hipLaunchKernelGGL(k_swap<double2>, grid_for(units), dim3(kThreads), 0, st, (double2 *)s.amp, g.q[0],
                               g.q[1], units);
        prof_end(st);
        QS_HIP(hipGetLastError());
        return QS_OK;
    }
    // dense k-qubit (k >= 2)
    const int k = g.nq, d = 1 << k;
    DenseScratch &sc = g_dense[c64 ? 0 : 1];
    const size_t need = (size_t)d * d * 2 * (c64 ? sizeof(float) : sizeof(double));
    if (sc.cap < need) {
        if (sc.ptr) {
            QS_HIP(hipStreamSynchronize(st));
            QS_HIP(hipFree(sc.ptr));
        }
        sc.ptr = nullptr;
        sc.cap = 0;
        QS_HIP(hipMalloc(&sc.ptr, need));
        sc.cap = need;
    }
    // the matrix buffer is reused by the next dense gate: stage it synchronously
    QS_HIP(hipStreamSynchronize(st));
    if (c64) {
        std::vector<float> h((size_t)d * d * 2);
        for (size_t i = 0; i < (size_t)d * d; ++i) {
            h[2 * i] = (float)g.m[i].real();
            h[2 * i + 1] = (float)g.m[i].imag();
        }
        QS_HIP(hipMemcpy(sc.ptr, h.data(), need, hipMemcpyHostToDevice));
    } else {
        std::vector<double> h((size_t)d * d * 2);
        for (size_t i = 0; i < (size_t)d * d; ++i) {
            h[2 * i] = g.m[i].real();
            h[2 * i + 1] = g.m[i].imag();
        }
        QS_HIP(hipMemcpy(sc.ptr, h.data(), need, hipMemcpyHostToDevice));
    }
    int pos[6] = {0, 0, 0, 0, 0, 0};
    for (int j = 0; j < k; ++j) pos[j] = g.q[j];
    int4 pa = make_int4(pos[0], pos[1], pos[2], pos[3]);
    int2 pb = make_int2(pos[4], pos[5]);
    uint64_t units = 1ull << (n - k);
    dim3 grid = grid_for(units, 1);
    prof_begin(st, QS_PROF_PLAIN, 2 * S, 8.0 * d * std::ldexp(1.0, n));
#define DENSE_CASE(KK)                                                                                          \
    case KK:                                                                                                    \
        if (c64)                                                                                                \
            hipLaunchKernelGGL((k_dense<KK, float, float2>), grid, dim3(kThreads), 0, st, (float2 *)s.amp, pa, pb, \
                               units, (const float *)sc.ptr);                                                   \
        else                                                                                                    \
            hipLaunchKernelGGL((k_dense<KK, double, double2>), grid, dim3(kThreads), 0, st, (double2 *)s.amp, pa,  \
                               pb, units, (const double *)sc.ptr);                                              \
        break;
    switch (k) {
        DENSE_CASE(2)
        DENSE_CASE(3)
        DENSE_CASE(4)
        DENSE_CASE(5)
        DENSE_CASE(6)
    default:
        prof_end(st);
        set_error("dense width %d unsupported", k);
        return QS_EUNSUPPORTED;
    }
#undef DENSE_CASE
    prof_end(st);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

qs_status launch_scale(qs_state_s &s, const double *d_scale) {
    const uint64_t units = 1ull << s.n;
    const double S = std::ldexp((double)(s.dtype == QS_C64 ? 8 : 16), s.n);
    prof_begin(s.stream, QS_PROF_COPY, 2 * S, 2.0 * units);
    if (s.dtype == QS_C64)
        hipLaunchKernelGGL((k_scale<float, float2>), grid_for(units), dim3(kThreads), 0, s.stream, (float2 *)s.amp,
                           units, d_scale);
    else
        hipLaunchKernelGGL((k_scale<double, double2>), grid_for(units), dim3(kThreads), 0, s.stream,
                           (double2 *)s.amp, units, d_scale);
    prof_end(s.stream);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

qs_status launch_set_basis(qs_state_s &s, uint64_t index) {
    const uint64_t bytes = (uint64_t)(s.dtype == QS_C64 ? 8 : 16) << s.n;
    const uint64_t words = (bytes + 15) / 16;
    if (bytes < 16) {
        // n = 0 is rejected earlier; complex64 with n = 1 is exactly 16 bytes
        set_error("state too small");
        return QS_EINVAL;
    }
    hipLaunchKernelGGL(k_fill_basis, grid_for(words), dim3(kThreads), 0, s.stream, (uint4 *)s.amp, words, (int)s.dtype,
                       index);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

qs_status launch_copy(void *dst, const void *src, uint64_t bytes, hipStream_t st) {
    QS_CHECK(bytes % 16 == 0, QS_EINVAL, "copy size must be a multiple of 16 bytes");
    const uint64_t words = bytes / 16;
    prof_begin(st, QS_PROF_COPY, 2.0 * bytes, 0);
    static int nt = -1;
    if (nt < 0) {
        const char *e = getenv("QS_COPY_TEMPORAL");
        nt = (e && atoi(e) != 0) ? 0 : 1;
    }
    if (nt)
        hipLaunchKernelGGL(k_copy<true>, grid_for(words), dim3(kThreads), 0, st, (float4 *)dst, (const float4 *)src,
                           words);
    else
        hipLaunchKernelGGL(k_copy<false>, grid_for(words), dim3(kThreads), 0, st, (float4 *)dst, (const float4 *)src,
                           words);
    prof_end(st);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

}  // namespace qs
