/*
 * FP64 reference state-vector simulator.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the GPU library, and it must never be used as a fallback for it.
 *
 * Everything here is deliberately plain: one loop per gate over the whole
 * amplitude array, std C99 double complex, no blocking, no fusion.
 *
 * Conventions (paper, Section 2.1, Eq. 1 and Eq. 2):
 *   - the state holds 2^n amplitudes; amplitude i is the coefficient of the
 *     basis state whose binary expansion is i;
 *   - qubit q is bit q of the index (little-endian): a single-qubit gate on
 *     qubit k acts as I^(n-k-1) (x) U (x) I^(k)  (Eq. 2).
 *
 * Parallelism: the sweeps carry an OpenMP "parallel for" over independent
 * amplitude pairs.  Reductions use fixed blocks summed in a fixed order, so
 * results do not depend on the thread count.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* threads                                                              */
/* ------------------------------------------------------------------ */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Gate table.  The paper names gates but never writes their matrices;  */
/* these are the OpenQASM-2.0 style textbook forms.  Matrices are       */
/* row-major: m[2*r + c] = <r|U|c>.                                      */
/* ------------------------------------------------------------------ */
enum {
    OR_H = 0, OR_X, OR_Y, OR_Z, OR_S, OR_SDG, OR_T, OR_TDG,
    OR_RX, OR_RY, OR_RZ, OR_U3, OR_P,
    OR_CNOT, OR_CZ, OR_CP, OR_CU, OR_SWAP, OR_DENSE
};

/* 2x2 matrix of a single-qubit kind (also the target part of the
 * controlled kinds).  Returns 0 on success, -1 for an unknown kind. */
int or_gate_2x2(int kind, const double *p, cplx *m)
{
    const double r2 = 1.0 / sqrt(2.0);
    double c, s;
    switch (kind) {
    case OR_H:   m[0] = r2; m[1] = r2; m[2] = r2; m[3] = -r2; return 0;
    case OR_X:
    case OR_CNOT: m[0] = 0; m[1] = 1; m[2] = 1; m[3] = 0; return 0;
    case OR_Y:   m[0] = 0; m[1] = -I; m[2] = I; m[3] = 0; return 0;
    case OR_Z:
    case OR_CZ:  m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -1; return 0;
    case OR_S:   m[0] = 1; m[1] = 0; m[2] = 0; m[3] = I; return 0;
    case OR_SDG: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -I; return 0;
    case OR_T:   m[0] = 1; m[1] = 0; m[2] = 0; m[3] = cexp(I * M_PI / 4); return 0;
    case OR_TDG: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = cexp(-I * M_PI / 4); return 0;
    case OR_RX:
        c = cos(p[0] / 2); s = sin(p[0] / 2);
        m[0] = c; m[1] = -I * s; m[2] = -I * s; m[3] = c; return 0;
    case OR_RY:
        c = cos(p[0] / 2); s = sin(p[0] / 2);
        m[0] = c; m[1] = -s; m[2] = s; m[3] = c; return 0;
    case OR_RZ:
        m[0] = cexp(-I * p[0] / 2); m[1] = 0; m[2] = 0; m[3] = cexp(I * p[0] / 2); return 0;
    case OR_U3:
    case OR_CU:
        c = cos(p[0] / 2); s = sin(p[0] / 2);
        m[0] = c;
        m[1] = -cexp(I * p[2]) * s;
        m[2] = cexp(I * p[1]) * s;
        m[3] = cexp(I * (p[1] + p[2])) * c;
        return 0;
    case OR_P:
    case OR_CP:
        m[0] = 1; m[1] = 0; m[2] = 0; m[3] = cexp(I * p[0]); return 0;
    default:
        return -1;
    }
}

/* ------------------------------------------------------------------ */
/* Index helper: the m-th index (in increasing order) whose bit p is 0,  */
/* i.e. m with a zero bit inserted at position p.                        */
/* ------------------------------------------------------------------ */
static int64_t with_zero_bit(int64_t m, int p)
{
    const int64_t low = m & (((int64_t)1 << p) - 1);
    return ((m - low) << 1) | low;
}

/* ------------------------------------------------------------------ */
/* Single-qubit gate, Eq. 3 (Section 2.2): U on qubit k couples exactly  */
/* the amplitude pairs (i, i + 2^k) with bit k of i equal to 0; every    */
/* such pair is replaced by U applied to it.  The 2^(n-1) lower members  */
/* are enumerated directly as m with a zero bit inserted at k.           */
/* ------------------------------------------------------------------ */
void or_apply_1q(cplx *psi, int n, int k, const cplx *u)
{
    const int64_t npairs = (int64_t)1 << (n - 1);
    const int64_t step = (int64_t)1 << k;
    #pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < npairs; ++m) {
        const int64_t lo = with_zero_bit(m, k), hi = lo + step;
        const cplx a0 = psi[lo], a1 = psi[hi];
        psi[lo] = u[0] * a0 + u[1] * a1;
        psi[hi] = u[2] * a0 + u[3] * a1;
    }
}

/* ------------------------------------------------------------------ */
/* Controlled gate, Eq. 4 (Section 2.1): |0><0| (x) I + |1><1| (x) U on  */
/* (control, target), generalised to a set of control bits.  The pairs   */
/* it couples are the target pairs of Eq. 3 restricted to the set        */
/* { i : (i & ctrl_mask) == ctrl_mask }; the others are left unchanged.  */
/* ------------------------------------------------------------------ */
void or_apply_controlled(cplx *psi, int n, uint64_t ctrl_mask, int t, const cplx *u)
{
    const int64_t npairs = (int64_t)1 << (n - 1);
    const int64_t step = (int64_t)1 << t;
    const int64_t cm = (int64_t)ctrl_mask;
    #pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < npairs; ++m) {
        const int64_t lo = with_zero_bit(m, t), hi = lo + step;
        if ((lo & cm) != cm) continue;
        const cplx a0 = psi[lo], a1 = psi[hi];
        psi[lo] = u[0] * a0 + u[1] * a1;
        psi[hi] = u[2] * a0 + u[3] * a1;
    }
}

/* ------------------------------------------------------------------ */
/* Dense k-qubit gate (Eq. 6 for k = 2, generalised).                   */
/* Local bit j of the 2^k sub-index corresponds to qubits[j].  For      */
/* every base index with all those bits 0, the 2^k amplitudes are       */
/* gathered, multiplied by U (row-major 2^k x 2^k) and scattered back.  */
/* ------------------------------------------------------------------ */
int or_apply_dense(cplx *psi, int n, const int *qubits, int k, const cplx *u)
{
    if (k < 1 || k > 12) return -1;
    const int64_t dim = (int64_t)1 << n;
    const int d = 1 << k;
    int64_t allmask = 0;
    for (int j = 0; j < k; ++j) allmask |= (int64_t)1 << qubits[j];
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * d);
    if (!off) return -2;
    for (int r = 0; r < d; ++r) {
        int64_t o = 0;
        for (int j = 0; j < k; ++j)
            if ((r >> j) & 1) o |= (int64_t)1 << qubits[j];
        off[r] = o;
    }
    #pragma omp parallel
    {
        cplx *v = (cplx *)malloc(sizeof(cplx) * d);
        cplx *w = (cplx *)malloc(sizeof(cplx) * d);
        #pragma omp for schedule(static)
        for (int64_t i = 0; i < dim; ++i) {
            if ((i & allmask) != 0) continue;
            for (int r = 0; r < d; ++r) v[r] = psi[i | off[r]];
            for (int r = 0; r < d; ++r) {
                cplx acc = 0;
                for (int c = 0; c < d; ++c) acc += u[(int64_t)r * d + c] * v[c];
                w[r] = acc;
            }
            for (int r = 0; r < d; ++r) psi[i | off[r]] = w[r];
        }
        free(v);
        free(w);
    }
    free(off);
    return 0;
}

/* SWAP exchanges the amplitudes whose two bits read 01 and 10. */
void or_apply_swap(cplx *psi, int n, int a, int b)
{
    const int64_t dim = (int64_t)1 << n;
    const int64_t ma = (int64_t)1 << a, mb = (int64_t)1 << b;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; ++i) {
        if ((i & ma) != 0 && (i & mb) == 0) {
            cplx tmp = psi[i];
            psi[i] = psi[i - ma + mb];
            psi[i - ma + mb] = tmp;
        }
    }
}

/* ------------------------------------------------------------------ */
/* One gate of a circuit.  qubits: for controlled kinds the control     */
/* comes first, then the target.  dense: 2^nq x 2^nq row-major matrix   */
/* for OR_DENSE (local bit j <-> qubits[j]).                            */
/* ------------------------------------------------------------------ */
int or_apply_gate(cplx *psi, int n, int kind, const int *qubits, int nq,
                  const double *params, const cplx *dense)
{
    cplx m[4];
    for (int j = 0; j < nq; ++j)
        if (qubits[j] < 0 || qubits[j] >= n) return -1;
    switch (kind) {
    case OR_CNOT: case OR_CZ: case OR_CP: case OR_CU:
        if (nq != 2 || qubits[0] == qubits[1]) return -1;
        or_gate_2x2(kind, params, m);
        or_apply_controlled(psi, n, (uint64_t)1 << qubits[0], qubits[1], m);
        return 0;
    case OR_SWAP:
        if (nq != 2 || qubits[0] == qubits[1]) return -1;
        or_apply_swap(psi, n, qubits[0], qubits[1]);
        return 0;
    case OR_DENSE:
        if (!dense) return -1;
        return or_apply_dense(psi, n, qubits, nq, dense);
    default:
        if (nq != 1) return -1;
        if (or_gate_2x2(kind, params, m) != 0) return -1;
        or_apply_1q(psi, n, qubits[0], m);
        return 0;
    }
}

/* ------------------------------------------------------------------ */
/* Reductions: fixed 4096-amplitude blocks, each summed sequentially,   */
/* then the block sums added in index order.                            */
/* ------------------------------------------------------------------ */
#define OR_RED_BLOCK 4096

double or_norm2(const cplx *psi, int n)
{
    const int64_t dim = (int64_t)1 << n;
    const int64_t nb = (dim + OR_RED_BLOCK - 1) / OR_RED_BLOCK;
    double *part = (double *)malloc(sizeof(double) * nb);
    #pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b) {
        double s = 0;
        int64_t e = (b + 1) * OR_RED_BLOCK;
        if (e > dim) e = dim;
        for (int64_t i = b * OR_RED_BLOCK; i < e; ++i)
            s += creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
        part[b] = s;
    }
    double tot = 0;
    for (int64_t b = 0; b < nb; ++b) tot += part[b];
    free(part);
    return tot;
}

/* Pauli string P given by bit masks: x = positions holding X or Y,
 * z = positions holding Z or Y.  Per qubit X|b> = |b^1>, Z|b> = (-1)^b|b>,
 * Y|b> = i(-1)^b |b^1>, hence
 *   P|j> = i^{|x&z|} (-1)^{popcount(j & z)} |j ^ x>.
 * <psi|P|psi> = sum_j conj(psi[j^x]) i^{|x&z|} (-1)^{popcount(j&z)} psi[j]. */
static cplx ipow(int e)
{
    switch (e & 3) {
    case 0: return 1;
    case 1: return I;
    case 2: return -1;
    default: return -I;
    }
}

cplx or_expect_pauli_c(const cplx *psi, int n, uint64_t x, uint64_t z)
{
    const int64_t dim = (int64_t)1 << n;
    const int64_t nb = (dim + OR_RED_BLOCK - 1) / OR_RED_BLOCK;
    double *pr = (double *)malloc(sizeof(double) * nb);
    double *pi = (double *)malloc(sizeof(double) * nb);
    #pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b) {
        cplx s = 0;
        int64_t e = (b + 1) * OR_RED_BLOCK;
        if (e > dim) e = dim;
        for (int64_t j = b * OR_RED_BLOCK; j < e; ++j) {
            int par = __builtin_popcountll((uint64_t)j & z) & 1;
            cplx term = conj(psi[(uint64_t)j ^ x]) * psi[j];
            s += par ? -term : term;
        }
        pr[b] = creal(s);
        pi[b] = cimag(s);
    }
    cplx tot = 0;
    for (int64_t b = 0; b < nb; ++b) tot += pr[b] + I * pi[b];
    free(pr);
    free(pi);
    return tot * ipow(__builtin_popcountll(x & z));
}

/* Real and imaginary parts of <psi|P|psi> (the imaginary part is zero up
 * to rounding for a Hermitian P; it is returned so tests can check it). */
void or_expect_pauli(const cplx *psi, int n, uint64_t x, uint64_t z, double *re, double *im)
{
    cplx v = or_expect_pauli_c(psi, n, x, z);
    *re = creal(v);
    *im = cimag(v);
}

/* Pauli-sum energy: sum_k c_k <psi|P_k|psi>, terms added in order. */
double or_expect_pauli_sum(const cplx *psi, int n, const uint64_t *x, const uint64_t *z,
                           const double *coeff, int nterms)
{
    double e = 0;
    for (int k = 0; k < nterms; ++k)
        e += coeff[k] * creal(or_expect_pauli_c(psi, n, x[k], z[k]));
    return e;
}

/* Closed form of a Pauli rotation: since P^2 = I,
 *   exp(-i theta P) psi = cos(theta) psi - i sin(theta) P psi.
 * P maps the pair (j, j^x) onto itself, so the update is done pairwise in
 * place; x = 0 (a pure Z string) is diagonal. */
void or_pauli_rotation(cplx *psi, int n, uint64_t x, uint64_t z, double theta)
{
    const int64_t dim = (int64_t)1 << n;
    const double c = cos(theta), s = sin(theta);
    const cplx ph = ipow(__builtin_popcountll(x & z));
    if (x == 0) {
        #pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < dim; ++j) {
            int par = __builtin_popcountll((uint64_t)j & z) & 1;
            cplx pj = (par ? -ph : ph) * psi[j];
            psi[j] = c * psi[j] - I * s * pj;
        }
        return;
    }
    const uint64_t hi = (uint64_t)1 << (63 - __builtin_clzll(x));
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < dim; ++j) {
        if (((uint64_t)j & hi) != 0) continue;
        int64_t jp = (int64_t)((uint64_t)j ^ x);
        cplx a = psi[j], b = psi[jp];
        /* (P psi)[j^x] = phase(j) psi[j], (P psi)[j] = phase(j^x) psi[j^x] */
        int pj = __builtin_popcountll((uint64_t)j & z) & 1;
        int pjp = __builtin_popcountll((uint64_t)jp & z) & 1;
        cplx Pa_at_jp = (pj ? -ph : ph) * a;
        cplx Pb_at_j = (pjp ? -ph : ph) * b;
        psi[j] = c * a - I * s * Pb_at_j;
        psi[jp] = c * b - I * s * Pa_at_jp;
    }
}

/* ------------------------------------------------------------------ */
/* The lower members of the pairs a gate on target t couples, from the  */
/* definitions of Eq. 3 and Eq. 4: { i : bit t of i is 0 and            */
/* (i & ctrl_mask) == ctrl_mask }, in increasing order (ctrl_mask = 0:  */
/* a one-qubit gate).  Written to out (capacity cap); returns the count. */
/* Tests compare this set with the grouped traversal of Section 2.2.    */
/* ------------------------------------------------------------------ */
int64_t or_pair_lows(int n, int t, uint64_t ctrl_mask, int64_t *out, int64_t cap)
{
    int64_t cnt = 0;
    const int64_t cm = (int64_t)ctrl_mask;
    for (int64_t m = 0; m < ((int64_t)1 << (n - 1)); ++m) {
        const int64_t lo = with_zero_bit(m, t);
        if ((lo & cm) != cm) continue;
        if (cnt < cap) out[cnt] = lo;
        ++cnt;
    }
    return cnt;
}

/* Operation-count model of Section 3.4: a 2^k x 2^k matrix-vector product
 * on each of the 2^(n-k) groups costs 4^k multiplications, 4^k - 2^k
 * additions and 2*2^k data copies (k = 1: 4 + 2 + 4 = 10 per pair;
 * k = 2: 16 + 12 + 8 = 36 per group of four). */
double or_opcount(int n, int k)
{
    double d = ldexp(1.0, k);
    return ldexp(1.0, n - k) * (d * d + (d * d - d) + 2 * d);
}
