// Gate ingest: validation and FP64 matrices of every gate kind.
//
// The paper names its gates (Section 2.1: one-qubit U_1 on a target, Eq. 3;
// controlled CU = |0><0| (x) I + |1><1| (x) U, Eq. 4) and reads them from
// OpenQASM-2.0 style circuit files (Section 4.1); the matrices below are the
// usual OpenQASM forms.  Every gate becomes a full 2^nq x 2^nq matrix whose
// local bit j corresponds to qubits[j] (controls first).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "internal.h"

namespace qs {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

qs_status hip_fail(hipError_t e, const char *what) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? QS_ENOMEM : QS_EDEVICE;
}

const char *last_error() { return g_err.c_str(); }

namespace {

const cd kI(0.0, 1.0);

// 2x2 target matrix of a one-qubit kind (or of a controlled kind's U).
bool two_by_two(int kind, const double *p, cd m[4]) {
    const double r2 = 1.0 / std::sqrt(2.0);
    switch (kind) {
    case QS_H: m[0] = r2; m[1] = r2; m[2] = r2; m[3] = -r2; return true;
    case QS_X: case QS_CNOT: m[0] = 0; m[1] = 1; m[2] = 1; m[3] = 0; return true;
    case QS_Y: m[0] = 0; m[1] = -kI; m[2] = kI; m[3] = 0; return true;
    case QS_Z: case QS_CZ: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -1; return true;
    case QS_S: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = kI; return true;
    case QS_SDG: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -kI; return true;
    case QS_T: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = std::polar(1.0, M_PI / 4); return true;
    case QS_TDG: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = std::polar(1.0, -M_PI / 4); return true;
    case QS_RX: {
        double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
        m[0] = c; m[1] = cd(0, -s); m[2] = cd(0, -s); m[3] = c;
        return true;
    }
    case QS_RY: {
        double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
        m[0] = c; m[1] = -s; m[2] = s; m[3] = c;
        return true;
    }
    case QS_RZ:
        m[0] = std::polar(1.0, -p[0] / 2); m[1] = 0; m[2] = 0; m[3] = std::polar(1.0, p[0] / 2);
        return true;
    case QS_P: case QS_CP:
        m[0] = 1; m[1] = 0; m[2] = 0; m[3] = std::polar(1.0, p[0]);
        return true;
    case QS_U3: case QS_CU: {
        double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
        m[0] = c;
        m[1] = -std::polar(s, p[2]);
        m[2] = std::polar(s, p[1]);
        m[3] = std::polar(c, p[1] + p[2]);
        return true;
    }
    default:
        return false;
    }
}

}  // namespace

qs_status make_gate(const qs_gate &g, int n, HGate &out) {
    QS_CHECK(g.kind >= 0 && g.kind < QS_NUM_KINDS, QS_EINVAL, "unknown gate kind %d", g.kind);
    int want = 1;
    if (g.kind >= QS_CNOT && g.kind <= QS_SWAP) want = 2;
    if (g.kind == QS_DENSE) {
        QS_CHECK(g.nq >= 1 && g.nq <= kMaxK, QS_EINVAL, "dense gate width %d outside 1..%d", g.nq, kMaxK);
        QS_CHECK(g.matrix != nullptr, QS_EINVAL, "dense gate without matrix");
        want = g.nq;
    }
    QS_CHECK(g.nq == want, QS_EINVAL, "gate kind %d needs %d qubits, got %d", g.kind, want, g.nq);
    for (int j = 0; j < g.nq; ++j) {
        QS_CHECK(g.qubits[j] >= 0 && g.qubits[j] < n, QS_EINVAL, "qubit %d out of range for n=%d",
                 g.qubits[j], n);
        for (int i = 0; i < j; ++i)
            QS_CHECK(g.qubits[i] != g.qubits[j], QS_EINVAL, "duplicate qubit %d in gate", g.qubits[j]);
    }
    out.kind = g.kind;
    out.nq = g.nq;
    for (int j = 0; j < 8; ++j) out.q[j] = j < g.nq ? g.qubits[j] : 0;
    for (int j = 0; j < 4; ++j) out.p[j] = g.params[j];
    const int d = 1 << g.nq;
    out.m.assign((size_t)d * d, cd(0, 0));
    if (g.kind == QS_DENSE) {
        for (int i = 0; i < d * d; ++i) out.m[i] = cd(g.matrix[2 * i], g.matrix[2 * i + 1]);
        return QS_OK;
    }
    if (g.kind == QS_SWAP) {
        // local index r = b0 + 2 b1; SWAP maps |b0 b1> to |b1 b0>
        for (int c = 0; c < 4; ++c) {
            int r = ((c & 1) << 1) | ((c >> 1) & 1);
            out.m[r * 4 + c] = 1;
        }
        return QS_OK;
    }
    cd u[4];
    two_by_two(g.kind, g.params, u);
    if (want == 1) {
        for (int i = 0; i < 4; ++i) out.m[i] = u[i];
        return QS_OK;
    }
    // controlled: local bit 0 = control, bit 1 = target (Eq. 4)
    out.m[0 * 4 + 0] = 1;
    out.m[2 * 4 + 2] = 1;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) out.m[(1 + 2 * a) * 4 + (1 + 2 * b)] = u[2 * a + b];
    return QS_OK;
}

}  // namespace qs
