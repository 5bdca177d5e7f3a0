// Pauli-rotation windows: runs of gates that multiply to exp(-i phi/2 P).
//
// A run C_a * D_q * C_b of Clifford gates around one diagonal one-qubit gate
// D_q = diag(a, b) on qubit q, whose Clifford parts cancel (C_a C_b = e^{i alpha} I),
// equals e^{i alpha} ((a+b)/2 I + (a-b)/2 Q) with Q = C_b^dagger Z_q C_b, a
// Pauli string with sign +-1.  This is how a Pauli exponential is written as
// basis changes, a CNOT ladder, a Z rotation and the ladder and basis changes
// undone.  Such a run acts on a state as
//     y[k] = c psi[k] + d sigma(k xor x) psi[k xor x],   sigma(j) = (-1)^{|j & z|},
// with x, z the X and Z parts of Q: two nonzeros per row, whatever the run's
// length.  Found runs are contracted into one block each (a contraction beyond
// Section 3.4's rule, which only merges gates up to a fixed width).
//
// Cliffords are recognised from the gate matrices themselves: a one- or
// two-qubit gate is Clifford when it maps every X_j and Z_j to a Pauli string
// under conjugation.  Pauli strings are i^e X^x Z^z (bit j of x, z = qubit j).
#include <algorithm>
#include <cmath>
#include <map>

#include "internal.h"

namespace qs {
namespace {

constexpr double kTol = 1e-9;
constexpr int kMaxWindowGates = 96;
constexpr int kMaxWindowWidth = 8;

struct Pauli {
    uint64_t x = 0, z = 0;
    int e = 0;  // phase i^e, mod 4
};

// (i^e1 X^x1 Z^z1)(i^e2 X^x2 Z^z2) = i^(e1+e2) (-1)^|z1 & x2| X^(x1^x2) Z^(z1^z2)
Pauli mul(const Pauli &a, const Pauli &b) {
    Pauli r;
    r.x = a.x ^ b.x;
    r.z = a.z ^ b.z;
    r.e = (a.e + b.e + 2 * __builtin_popcountll(a.z & b.x)) & 3;
    return r;
}

cd ipow(int e) {
    switch (e & 3) {
    case 0: return cd(1, 0);
    case 1: return cd(0, 1);
    case 2: return cd(-1, 0);
    default: return cd(0, -1);
    }
}

// Local Pauli X^a Z^b on nq qubits as a dense D x D matrix (row-major).
std::vector<cd> pauli_matrix(int nq, int a, int b) {
    const int D = 1 << nq;
    std::vector<cd> m((size_t)D * D, cd(0, 0));
    for (int j = 0; j < D; ++j) m[(size_t)(j ^ a) * D + j] = (__builtin_popcount(j & b) & 1) ? -1.0 : 1.0;
    return m;
}

std::vector<cd> matmul(const std::vector<cd> &A, const std::vector<cd> &B, int D) {
    std::vector<cd> C((size_t)D * D, cd(0, 0));
    for (int i = 0; i < D; ++i)
        for (int k = 0; k < D; ++k) {
            const cd v = A[(size_t)i * D + k];
            if (v == cd(0, 0)) continue;
            for (int j = 0; j < D; ++j) C[(size_t)i * D + j] += v * B[(size_t)k * D + j];
        }
    return C;
}

std::vector<cd> dagger(const std::vector<cd> &A, int D) {
    std::vector<cd> B((size_t)D * D);
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) B[(size_t)j * D + i] = std::conj(A[(size_t)i * D + j]);
    return B;
}

// M == i^e X^a Z^b for some (a, b, e)?
bool as_pauli(const std::vector<cd> &M, int nq, Pauli &out) {
    const int D = 1 << nq;
    int a = -1;
    for (int r = 0; r < D; ++r)
        if (std::abs(M[(size_t)r * D]) > 0.5) {
            a = r;
            break;
        }
    if (a < 0) return false;
    const cd ph = M[(size_t)a * D];
    int e = -1;
    for (int k = 0; k < 4; ++k)
        if (std::abs(ph - ipow(k)) < kTol) e = k;
    if (e < 0) return false;
    int b = 0;
    for (int j = 0; j < nq; ++j) {
        const cd v = M[(size_t)((1 << j) ^ a) * D + (1 << j)] / ph;
        if (std::abs(v + 1.0) < kTol) b |= 1 << j;
        else if (std::abs(v - 1.0) >= kTol) return false;
    }
    const std::vector<cd> P = pauli_matrix(nq, a, b);
    for (size_t i = 0; i < M.size(); ++i)
        if (std::abs(M[i] - ph * P[i]) > kTol) return false;
    out.x = (uint64_t)a;
    out.z = (uint64_t)b;
    out.e = e;
    return true;
}

// Conjugation images of X_j, Z_j (local) under a gate: fwd = G P G^dagger,
// back = G^dagger P G.  Valid only when `clifford`.
struct GateTables {
    bool clifford = false;
    Pauli fwd[2][2], back[2][2];  // [X or Z][local qubit]
};

GateTables tables(const HGate &g) {
    GateTables t;
    if (g.nq < 1 || g.nq > 2) return t;
    const int D = 1 << g.nq;
    const std::vector<cd> Gd = dagger(g.m, D);
    for (int which = 0; which < 2; ++which)
        for (int j = 0; j < g.nq; ++j) {
            const std::vector<cd> P = which == 0 ? pauli_matrix(g.nq, 1 << j, 0) : pauli_matrix(g.nq, 0, 1 << j);
            if (!as_pauli(matmul(matmul(g.m, P, D), Gd, D), g.nq, t.fwd[which][j])) return t;
            if (!as_pauli(matmul(matmul(Gd, P, D), g.m, D), g.nq, t.back[which][j])) return t;
        }
    t.clifford = true;
    return t;
}

// Conjugate a global Pauli string by a Clifford gate (tables fwd or back).
Pauli conjugate(const Pauli &p, const HGate &g, const Pauli (&img)[2][2]) {
    uint64_t in = 0;
    for (int j = 0; j < g.nq; ++j) in |= 1ull << g.q[j];
    // i^e X^x Z^z = i^e X^(x out) Z^(z out) * X^(x in) Z^(z in): factors on
    // disjoint qubits commute, so only the local part changes
    Pauli loc;  // image of X^(x in) Z^(z in), in local bits
    for (int j = 0; j < g.nq; ++j)
        if ((p.x >> g.q[j]) & 1) loc = mul(loc, img[0][j]);
    for (int j = 0; j < g.nq; ++j)
        if ((p.z >> g.q[j]) & 1) loc = mul(loc, img[1][j]);
    Pauli r;
    r.x = p.x & ~in;
    r.z = p.z & ~in;
    r.e = (p.e + loc.e) & 3;
    for (int j = 0; j < g.nq; ++j) {
        if ((loc.x >> j) & 1) r.x |= 1ull << g.q[j];
        if ((loc.z >> j) & 1) r.z |= 1ull << g.q[j];
    }
    return r;
}

bool diagonal_1q(const HGate &g) {
    return g.nq == 1 && std::abs(g.m[1]) < kTol && std::abs(g.m[2]) < kTol;
}

// Clifford part of a window applied to |0..0> of its support: e^{i alpha}|0..0>.
bool clifford_phase(const std::vector<HGate> &gates, int64_t i0, int64_t i1, int64_t skip,
                    const std::vector<int> &support, cd &phase) {
    const int w = (int)support.size();
    const int D = 1 << w;
    std::vector<cd> v(D, cd(0, 0)), t(D);
    v[0] = 1;
    for (int64_t gi = i0; gi <= i1; ++gi) {
        if (gi == skip) continue;
        const HGate &g = gates[gi];
        int lp[2];
        for (int j = 0; j < g.nq; ++j)
            lp[j] = (int)(std::find(support.begin(), support.end(), g.q[j]) - support.begin());
        const int gd = 1 << g.nq;
        std::fill(t.begin(), t.end(), cd(0, 0));
        for (int s = 0; s < D; ++s) {
            if (v[s] == cd(0, 0)) continue;
            int a = 0;
            for (int j = 0; j < g.nq; ++j) a |= ((s >> lp[j]) & 1) << j;
            int base = s;
            for (int j = 0; j < g.nq; ++j) base &= ~(1 << lp[j]);
            for (int r = 0; r < gd; ++r) {
                const cd m = g.m[(size_t)r * gd + a];
                if (m == cd(0, 0)) continue;
                int o = base;
                for (int j = 0; j < g.nq; ++j)
                    if ((r >> j) & 1) o |= 1 << lp[j];
                t[o] += m * v[s];
            }
        }
        v.swap(t);
    }
    for (int s = 1; s < D; ++s)
        if (std::abs(v[s]) > kTol) return false;
    if (std::abs(std::abs(v[0]) - 1.0) > kTol) return false;
    phase = v[0];
    return true;
}

}  // namespace

std::vector<PauliWindow> find_pauli_windows(const std::vector<HGate> &gates, int max_x_weight) {
    std::vector<PauliWindow> out;
    std::vector<GateTables> tab(gates.size());
    std::vector<char> have(gates.size(), 0);
    auto tables_of = [&](size_t gi) -> const GateTables & {
        if (!have[gi]) {
            tab[gi] = tables(gates[gi]);
            have[gi] = 1;
        }
        return tab[gi];
    };
    size_t i = 0;
    while (i < gates.size()) {
        // images of X_q, Z_q under the window's Clifford gates (rotation left out)
        std::map<int, std::pair<Pauli, Pauli>> img;
        uint64_t support = 0;
        int64_t rot = -1, end = -1;
        for (size_t j = i; j < gates.size() && j < i + kMaxWindowGates; ++j) {
            const HGate &g = gates[j];
            if (g.nq < 1 || g.nq > 2) break;
            for (int a = 0; a < g.nq; ++a) support |= 1ull << g.q[a];
            if (__builtin_popcountll(support) > kMaxWindowWidth) break;
            const GateTables &T = tables_of(j);
            if (!T.clifford) {
                if (rot >= 0 || !diagonal_1q(g)) break;
                rot = (int64_t)j;
                continue;
            }
            for (int a = 0; a < g.nq; ++a)
                if (!img.count(g.q[a])) {
                    Pauli X, Z;
                    X.x = 1ull << g.q[a];
                    Z.z = 1ull << g.q[a];
                    img[g.q[a]] = {X, Z};
                }
            for (auto &kv : img) {
                kv.second.first = conjugate(kv.second.first, g, T.fwd);
                kv.second.second = conjugate(kv.second.second, g, T.fwd);
            }
            if (rot < 0) continue;
            bool ident = true;
            for (auto &kv : img) {
                const Pauli &X = kv.second.first, &Z = kv.second.second;
                if (X.x != (1ull << kv.first) || X.z || X.e || Z.z != (1ull << kv.first) || Z.x || Z.e) {
                    ident = false;
                    break;
                }
            }
            if (ident) {
                end = (int64_t)j;
                break;
            }
        }
        if (end < 0) {
            ++i;
            continue;
        }
        // Q = C_b^dagger Z_q C_b, C_b = the gates before the rotation
        const HGate &R = gates[rot];
        Pauli Q;
        Q.z = 1ull << R.q[0];
        for (int64_t gi = rot - 1; gi >= (int64_t)i; --gi) Q = conjugate(Q, gates[gi], tables_of(gi).back);
        const int xz = __builtin_popcountll(Q.x & Q.z);
        // Q = i^(e - |x&z|) P with P = i^|x&z| X^x Z^z Hermitian; the sign must be real
        const int lam_e = (Q.e - xz) & 3;
        std::vector<int> sup;
        for (int q = 0; q < 64; ++q)
            if ((support >> q) & 1) sup.push_back(q);
        cd phase;
        if ((lam_e & 1) || __builtin_popcountll(Q.x) > max_x_weight ||
            !clifford_phase(gates, (int64_t)i, end, rot, sup, phase)) {
            ++i;
            continue;
        }
        const cd a = R.m[0], b = R.m[3];
        PauliWindow w;
        w.begin = (int64_t)i;
        w.end = end + 1;
        w.x = Q.x;
        w.z = Q.z;
        w.support = sup;
        w.c = phase * (a + b) * 0.5;
        w.d = phase * (a - b) * 0.5 * (lam_e == 2 ? -1.0 : 1.0) * ipow(xz);
        out.push_back(std::move(w));
        i = (size_t)(end + 1);
    }
    return out;
}

// Dense FP64 action of a window's block on its support (tests, qs_plan_block):
// y[k] = c psi[k] + d sigma(k ^ x) psi[k ^ x] in the block's local bits.
void pauli_block_matrix(HBlock &b) {
    const int k = (int)b.qubits.size();
    const int D = 1 << k;
    uint64_t lx = 0, lz = 0;
    for (int j = 0; j < k; ++j) {
        if ((b.px >> b.qubits[j]) & 1) lx |= 1ull << j;
        if ((b.pz >> b.qubits[j]) & 1) lz |= 1ull << j;
    }
    b.U.assign((size_t)D * D, cd(0, 0));
    for (int r = 0; r < D; ++r) {
        b.U[(size_t)r * D + r] += b.pc;
        const int c = r ^ (int)lx;
        const double s = (__builtin_popcountll((uint64_t)c & lz) & 1) ? -1.0 : 1.0;
        b.U[(size_t)r * D + c] += s * b.pd;
    }
}

}  // namespace qs
