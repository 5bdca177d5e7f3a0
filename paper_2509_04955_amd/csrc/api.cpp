// C ABI entry points (include/qsim.h): states, plain gate lists, plans,
// expectation values and profiling.  Argument checking and marshalling
// happen here; every sweep over amplitudes runs in the HIP kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "internal.h"

namespace qs {
const char *last_error();

// ------------------------------------------------------------ profiling
namespace {
struct ProfRec {
    int cls;
    hipEvent_t a, b;
    double bytes, flops;
};
std::mutex g_prof_mu;
bool g_prof = false;
std::vector<ProfRec> g_recs;
std::vector<hipEvent_t> g_free_events;
thread_local int g_open = -1;

hipEvent_t get_event() {
    if (!g_free_events.empty()) {
        hipEvent_t e = g_free_events.back();
        g_free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    hipEventCreate(&e);
    return e;
}
}  // namespace

bool prof_on() { return g_prof; }

void prof_begin(hipStream_t st, int cls, double bytes, double flops) {
    if (!g_prof) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    ProfRec r{cls, get_event(), get_event(), bytes, flops};
    hipEventRecord(r.a, st);
    g_recs.push_back(r);
    g_open = (int)g_recs.size() - 1;
}

void prof_end(hipStream_t st) {
    if (!g_prof || g_open < 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    hipEventRecord(g_recs[g_open].b, st);
    g_open = -1;
}

}  // namespace qs

using namespace qs;

qs_plan_s::~qs_plan_s() {
    for (int i = 0; i < 2; ++i) {
        if (d_blocks[i]) hipFree(d_blocks[i]);
        if (d_pool[i]) hipFree(d_pool[i]);
    }
}

namespace {

qs_status check_device() {
    int cnt = 0;
    hipError_t e = hipGetDeviceCount(&cnt);
    if (e != hipSuccess || cnt < 1) {
        set_error("no HIP device available (%s)", e == hipSuccess ? "count 0" : hipGetErrorString(e));
        return QS_EDEVICE;
    }
    return QS_OK;
}

size_t amp_bytes(qs_dtype d) { return d == QS_C64 ? 8 : 16; }

// If a pass left its renormalisation pending, bake it into the amplitudes.
qs_status materialize(qs_state_s &s) {
    if (!s.scale_pending) return QS_OK;
    qs_status st = launch_scale(s, s.d_slots + 1);
    if (st != QS_OK) return st;
    s.scale_pending = false;
    return QS_OK;
}

qs_status convert_gates(int n, const qs_gate *gates, size_t ng, std::vector<HGate> &out) {
    QS_CHECK(gates != nullptr || ng == 0, QS_EINVAL, "null gate list");
    out.resize(ng);
    for (size_t i = 0; i < ng; ++i) {
        qs_status st = make_gate(gates[i], n, out[i]);
        if (st != QS_OK) {
            std::string m = last_error();
            set_error("gate %zu: %s", i, m.c_str());
            return st;
        }
    }
    return QS_OK;
}

qs_status check_expect_args(qs_state s, const uint64_t *x, const uint64_t *z, const double *coeff, size_t n_terms,
                            const double *out) {
    QS_CHECK(s && x && z && coeff && out, QS_EINVAL, "null argument");
    QS_CHECK(n_terms >= 1 && n_terms <= (1u << 20), QS_ERANGE, "n_terms %zu outside 1..2^20", n_terms);
    const uint64_t lim = s->n >= 64 ? ~0ull : ((1ull << s->n) - 1);
    for (size_t k = 0; k < n_terms; ++k)
        QS_CHECK((x[k] & ~lim) == 0 && (z[k] & ~lim) == 0, QS_EINVAL, "term %zu acts outside the %d qubits", k, s->n);
    return QS_OK;
}

// one expectation launch into d_scr; res (plan.terms.size()) receives the
// unnormalised terms, res[0] the squared norm.  Synchronises the stream.
qs_status run_expect(qs_state_s &s, const ExpectPlan &plan, void *d_scr, std::vector<double> &res) {
    double *d_res = nullptr;
    qs_status st = launch_expect(s, plan, d_scr, &d_res);
    if (st != QS_OK) return st;
    QS_HIP(hipMemcpyAsync(res.data(), d_res, res.size() * sizeof(double), hipMemcpyDeviceToHost, s.stream));
    QS_HIP(hipStreamSynchronize(s.stream));
    return QS_OK;
}

qs_status finish_expect(std::vector<double> &terms, double nrm, const double *coeff, double *out, double *out_terms) {
    QS_CHECK(nrm > 0, QS_EINVAL, "state has zero norm");
    double E = 0;
    for (size_t k = 0; k < terms.size(); ++k) {
        terms[k] /= nrm;
        E += coeff[k] * terms[k];
        if (out_terms) out_terms[k] = terms[k];
    }
    *out = E;
    return QS_OK;
}

}  // namespace

extern "C" {

const char *qs_last_error(void) { return qs::last_error(); }
const char *qs_version(void) { return "qsim-gfx950 0.1"; }

qs_status qs_device_query(int *cu_count, int *lds_bytes, char *arch, size_t arch_len) {
    qs_status st = check_device();
    if (st != QS_OK) return st;
    int dev = 0;
    QS_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    QS_HIP(hipGetDeviceProperties(&prop, dev));
    if (cu_count) *cu_count = prop.multiProcessorCount;
    if (lds_bytes) *lds_bytes = (int)prop.sharedMemPerBlock;
    if (arch && arch_len) {
        std::strncpy(arch, prop.gcnArchName, arch_len - 1);
        arch[arch_len - 1] = 0;
    }
    return QS_OK;
}

qs_status qs_state_create(int n, qs_dtype dtype, void *dev_ptr, void *stream, qs_state *out) {
    QS_CHECK(out != nullptr, QS_EINVAL, "null output handle");
    QS_CHECK(n >= 1 && n <= kMaxQubits, QS_EINVAL, "n=%d outside 1..%d", n, kMaxQubits);
    QS_CHECK(dtype == QS_C64 || dtype == QS_C128, QS_EINVAL, "bad dtype %d", (int)dtype);
    QS_CHECK(dev_ptr == nullptr || ((uintptr_t)dev_ptr % 16) == 0, QS_EINVAL, "state buffer must be 16-byte aligned");
    qs_status st = check_device();
    if (st != QS_OK) return st;
    qs_state_s *s = new (std::nothrow) qs_state_s();
    QS_CHECK(s != nullptr, QS_ENOMEM, "host allocation failed");
    s->n = n;
    s->dtype = dtype;
    s->stream = (hipStream_t)stream;
    hipGetDevice(&s->device);
    hipError_t e = hipMalloc(&s->d_slots, kNumSlots * sizeof(double));
    if (e == hipSuccess) e = hipMemset(s->d_slots, 0, kNumSlots * sizeof(double));   // ticket counter at 0
    if (e != hipSuccess) {
        if (s->d_slots) hipFree(s->d_slots);
        delete s;
        return hip_fail(e, "hipMalloc(slots)");
    }
    if (dev_ptr) {
        s->amp = dev_ptr;
    } else {
        e = hipMalloc(&s->amp, amp_bytes(dtype) << n);
        if (e != hipSuccess) {
            hipFree(s->d_slots);
            delete s;
            return hip_fail(e, "hipMalloc(state)");
        }
        s->owned = true;
    }
    *out = s;
    return QS_OK;
}

qs_status qs_state_destroy(qs_state s) {
    if (!s) return QS_OK;
    hipStreamSynchronize(s->stream);
    if (s->owned && s->amp) hipFree(s->amp);
    if (s->d_slots) hipFree(s->d_slots);
    if (s->d_partials) hipFree(s->d_partials);
    delete s;
    return QS_OK;
}

qs_status qs_state_data(qs_state s, void **dev_ptr) {
    QS_CHECK(s && dev_ptr, QS_EINVAL, "null argument");
    *dev_ptr = s->amp;
    return QS_OK;
}

qs_status qs_state_set_basis(qs_state s, uint64_t index) {
    QS_CHECK(s != nullptr, QS_EINVAL, "null state");
    QS_CHECK(index < (1ull << s->n), QS_EINVAL, "basis index out of range");
    s->scale_pending = false;
    return launch_set_basis(*s, index);
}

qs_status qs_state_normalize(qs_state s) {
    QS_CHECK(s != nullptr, QS_EINVAL, "null state");
    return materialize(*s);
}

qs_status qs_state_copy_out(qs_state s, uint64_t offset, uint64_t count, double *host) {
    QS_CHECK(s && host, QS_EINVAL, "null argument");
    QS_CHECK(offset <= (1ull << s->n) && count <= (1ull << s->n) - offset, QS_EINVAL, "range outside state");
    double scale = 1.0;
    if (s->scale_pending) QS_HIP(hipMemcpyAsync(&scale, s->d_slots + 1, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    QS_HIP(hipStreamSynchronize(s->stream));
    const size_t ab = amp_bytes(s->dtype);
    const size_t chunk = 1u << 22;
    std::vector<unsigned char> buf(std::min<uint64_t>(count, chunk) * ab);
    for (uint64_t done = 0; done < count; done += chunk) {
        const uint64_t m = std::min<uint64_t>(chunk, count - done);
        QS_HIP(hipMemcpy(buf.data(), (unsigned char *)s->amp + (offset + done) * ab, m * ab, hipMemcpyDeviceToHost));
        if (s->dtype == QS_C64) {
            const float *f = (const float *)buf.data();
            for (uint64_t i = 0; i < 2 * m; ++i) host[2 * done + i] = (double)f[i] * scale;
        } else {
            const double *f = (const double *)buf.data();
            for (uint64_t i = 0; i < 2 * m; ++i) host[2 * done + i] = f[i] * scale;
        }
    }
    return QS_OK;
}

qs_status qs_state_copy_in(qs_state s, uint64_t offset, uint64_t count, const double *host) {
    QS_CHECK(s && host, QS_EINVAL, "null argument");
    QS_CHECK(offset <= (1ull << s->n) && count <= (1ull << s->n) - offset, QS_EINVAL, "range outside state");
    qs_status st = materialize(*s);
    if (st != QS_OK) return st;
    QS_HIP(hipStreamSynchronize(s->stream));
    const size_t ab = amp_bytes(s->dtype);
    if (s->dtype == QS_C64) {
        std::vector<float> f(2 * count);
        for (uint64_t i = 0; i < 2 * count; ++i) f[i] = (float)host[i];
        QS_HIP(hipMemcpy((unsigned char *)s->amp + offset * ab, f.data(), count * ab, hipMemcpyHostToDevice));
    } else {
        QS_HIP(hipMemcpy((unsigned char *)s->amp + offset * ab, host, count * ab, hipMemcpyHostToDevice));
    }
    return QS_OK;
}

qs_status qs_norm(qs_state s, double *out) {
    QS_CHECK(s && out, QS_EINVAL, "null argument");
    double *slot = s->d_slots + 2;  // slots 2/3: scratch norm (slot 1 keeps the pending scale)
    qs_status st = launch_norm_full(*s, slot);
    if (st != QS_OK) return st;
    double v[2] = {0, 1};
    QS_HIP(hipMemcpyAsync(&v[0], slot, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    if (s->scale_pending) QS_HIP(hipMemcpyAsync(&v[1], s->d_slots + 1, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    QS_HIP(hipStreamSynchronize(s->stream));
    *out = v[0] * v[1] * v[1];
    return QS_OK;
}

qs_status qs_apply_gates(qs_state s, const qs_gate *gates, size_t n_gates) {
    QS_ABI_TRY
    QS_CHECK(s != nullptr, QS_EINVAL, "null state");
    std::vector<HGate> hg;
    qs_status st = convert_gates(s->n, gates, n_gates, hg);
    if (st != QS_OK) return st;
    st = materialize(*s);
    if (st != QS_OK) return st;
    for (const HGate &g : hg) {
        st = launch_plain(*s, g);
        if (st != QS_OK) return st;
    }
    return QS_OK;
    QS_ABI_CATCH
}

qs_status qs_apply_gates_smgp(qs_state s, const qs_gate *gates, size_t n_gates) {
    QS_ABI_TRY
    QS_CHECK(s != nullptr, QS_EINVAL, "null state");
    std::vector<HGate> hg;
    qs_status st = convert_gates(s->n, gates, n_gates, hg);
    if (st != QS_OK) return st;
    st = materialize(*s);
    if (st != QS_OK) return st;
    return launch_smgp(*s, hg);
    QS_ABI_CATCH
}

qs_status qs_contract(int n, const qs_gate *gates, size_t n_gates, const qs_contract_opts *opts, qs_plan *out) {
    QS_CHECK(out != nullptr, QS_EINVAL, "null output handle");
    QS_CHECK(n >= 1 && n <= kMaxQubits, QS_EINVAL, "n=%d outside 1..%d", n, kMaxQubits);
    qs_plan_s *p = new (std::nothrow) qs_plan_s();
    QS_CHECK(p != nullptr, QS_ENOMEM, "host allocation failed");
    p->n = n;
    std::memset(&p->opts, 0, sizeof p->opts);
    if (opts) p->opts = *opts;
    else {
        p->opts.strategy = QS_STRATEGY_GREEDY;
        p->opts.renorm = 1;
    }
    qs_status st = QS_OK;
    {
        try {
            st = convert_gates(n, gates, n_gates, p->gates);
            if (st == QS_OK) st = build_plan(*p);
        } catch (const std::bad_alloc &) {
            set_error("host allocation failed while planning");
            st = QS_ENOMEM;
        } catch (const std::exception &e) {
            set_error("planner error: %s", e.what());
            st = QS_EINVAL;
        }
    }
    if (st != QS_OK) {
        delete p;
        return st;
    }
    *out = p;
    return QS_OK;
}

qs_status qs_plan_destroy(qs_plan p) {
    delete p;
    return QS_OK;
}

qs_status qs_plan_info_get(qs_plan p, qs_plan_info *info) {
    QS_CHECK(p && info, QS_EINVAL, "null argument");
    std::memset(info, 0, sizeof *info);
    info->n = p->n;
    info->n_gates = p->gates.size();
    info->n_blocks = p->blocks.size();
    info->n_passes = p->passes.size();
    for (const HBlock &b : p->blocks) {
        const int k = (int)b.qubits.size();
        info->max_k = std::max(info->max_k, k);
        if (k < 8) info->blocks_by_k[k]++;
        info->flops_per_amp += 8.0 * std::ldexp(1.0, k);
    }
    return QS_OK;
}

qs_status qs_plan_block(qs_plan p, uint64_t b, int *k, int *qubits, double *matrix, uint64_t *members,
                        uint64_t member_cap, uint64_t *n_members) {
    QS_ABI_TRY
    QS_CHECK(p != nullptr, QS_EINVAL, "null plan");
    QS_CHECK(b < p->blocks.size(), QS_EINVAL, "block index out of range");
    const HBlock &B = p->blocks[b];
    const int kk = (int)B.qubits.size();
    if (k) *k = kk;
    if (qubits)
        for (int j = 0; j < kk; ++j) qubits[j] = B.qubits[j];
    if (matrix) {
        const std::vector<cd> *U = &B.U;
        HBlock dense;
        if (B.pauli) {   // Pauli blocks keep (x, z, c, d); the dense form is built on request
            QS_CHECK(kk <= 10, QS_EUNSUPPORTED, "dense matrix of a %d-qubit Pauli block not available", kk);
            dense = B;
            pauli_block_matrix(dense);
            U = &dense.U;
        }
        for (size_t i = 0; i < U->size(); ++i) {
            matrix[2 * i] = (*U)[i].real();
            matrix[2 * i + 1] = (*U)[i].imag();
        }
    }
    if (members)
        for (uint64_t i = 0; i < std::min<uint64_t>(member_cap, B.members.size()); ++i) members[i] = B.members[i];
    if (n_members) *n_members = B.members.size();
    return QS_OK;
    QS_ABI_CATCH
}

qs_status qs_plan_pass(qs_plan p, uint64_t i, int *t, int *tile_qubits, uint64_t *first_block, uint64_t *n_blocks) {
    QS_CHECK(p != nullptr, QS_EINVAL, "null plan");
    QS_CHECK(i < p->passes.size(), QS_EINVAL, "pass index out of range");
    const HPass &ps = p->passes[i];
    if (t) *t = ps.t;
    if (tile_qubits)
        for (int j = 0; j < ps.t; ++j) tile_qubits[j] = ps.tile[j];
    if (first_block) *first_block = (uint64_t)ps.block0;
    if (n_blocks) *n_blocks = (uint64_t)ps.nblocks;
    return QS_OK;
}

qs_status qs_apply_plan(qs_state s, qs_plan p) {
    QS_CHECK(s && p, QS_EINVAL, "null argument");
    QS_CHECK(s->n == p->n, QS_EINVAL, "plan is for %d qubits, state has %d", p->n, s->n);
    const int tcap = s->dtype == QS_C128 ? kMaxTile128 : kMaxTile;
    for (const HPass &ps : p->passes)
        QS_CHECK(ps.t <= tcap, QS_EINVAL, "plan tile %d too large for this dtype", ps.t);
    qs_status st = plan_upload(*p, s->dtype);
    if (st != QS_OK) return st;
    const bool renorm = p->opts.renorm != 0;
    for (size_t i = 0; i < p->passes.size(); ++i) {
        const HPass &ps = p->passes[i];
        uint64_t nparts = 0;
        st = launch_pass(*s, *p, ps, (int64_t)i, s->scale_pending, renorm, &nparts);
        if (st != QS_OK) return st;
        s->scale_pending = false;
        if (renorm) {
            st = launch_norm_reduce(*s, nparts, s->d_slots);
            if (st != QS_OK) return st;
            s->scale_pending = true;
        }
    }
    return QS_OK;
}

qs_status qs_expect_pauli_sum(qs_state s, const uint64_t *x, const uint64_t *z, const double *coeff, size_t n_terms,
                              double *out, double *out_terms) {
    QS_ABI_TRY
    qs_status st = check_expect_args(s, x, z, coeff, n_terms, out);
    if (st != QS_OK) return st;
    std::vector<double> terms(n_terms);
    double nrm = 0;
    // launches of at most kExpTermsPerLaunch terms, each with its own scratch
    for (size_t k0 = 0; k0 < n_terms; k0 += kExpTermsPerLaunch) {
        const size_t cnt = std::min(kExpTermsPerLaunch, n_terms - k0);
        ExpectPlan plan;
        st = expect_plan(s->n, s->dtype, x + k0, z + k0, cnt, plan);
        if (st != QS_OK) return st;
        void *d_scr = nullptr;
        QS_HIP(hipMalloc(&d_scr, expect_scratch_bytes(plan)));
        std::vector<double> res(plan.terms.size());
        st = run_expect(*s, plan, d_scr, res);
        hipFree(d_scr);
        if (st != QS_OK) return st;
        if (k0 == 0) nrm = res[0];   // squared norm of the stored amplitudes (a pending scale cancels)
        std::copy(res.begin() + 1, res.end(), terms.begin() + k0);
    }
    return finish_expect(terms, nrm, coeff, out, out_terms);
    QS_ABI_CATCH
}

qs_status qs_expect_pauli_sum_noalloc(qs_state s, const uint64_t *x, const uint64_t *z, const double *coeff,
                                      size_t n_terms, double *out, double *out_terms) {
    QS_ABI_TRY
    qs_status st = check_expect_args(s, x, z, coeff, n_terms, out);
    if (st != QS_OK) return st;
    QS_CHECK(n_terms <= kNoAllocMaxTerms, QS_ERANGE, "n_terms %zu above the %zu this call holds scratch for",
             n_terms, kNoAllocMaxTerms);
    ExpectPlan plan;
    st = expect_plan(s->n, s->dtype, x, z, n_terms, plan, kNoAllocMaxGrid);
    if (st != QS_OK) return st;
    std::vector<double> res(plan.terms.size());
    {
        // one user of the device's scratch at a time in this process
        std::lock_guard<std::mutex> lk(noalloc_lock());
        void *d_scr = nullptr;
        st = noalloc_scratch(expect_scratch_bytes(plan), &d_scr);
        if (st != QS_OK) return st;
        st = run_expect(*s, plan, d_scr, res);
        if (st != QS_OK) return st;
    }
    std::vector<double> terms(res.begin() + 1, res.end());
    return finish_expect(terms, res[0], coeff, out, out_terms);
    QS_ABI_CATCH
}

qs_status qs_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof = on != 0;
    return QS_OK;
}

qs_status qs_profile_collect(qs_profile *out) {
    QS_CHECK(out != nullptr, QS_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    std::memset(out, 0, sizeof *out);
    for (ProfRec &r : g_recs) {
        hipEventSynchronize(r.b);
        float ms = 0;
        hipEventElapsedTime(&ms, r.a, r.b);
        if (r.cls >= 0 && r.cls < QS_PROF_CLASSES) {
            out->launches[r.cls]++;
            out->ms[r.cls] += ms;
            out->bytes[r.cls] += r.bytes;
            out->flops[r.cls] += r.flops;
        }
        g_free_events.push_back(r.a);
        g_free_events.push_back(r.b);
    }
    g_recs.clear();
    return QS_OK;
}

qs_status qs_copy(void *dst, const void *src, uint64_t bytes, void *stream) {
    QS_CHECK(dst && src, QS_EINVAL, "null pointer");
    return launch_copy(dst, src, bytes, (hipStream_t)stream);
}

}  // extern "C"
