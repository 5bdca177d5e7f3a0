// Cost-model MLP: hand-written forward, backward and Adam kernels, device
// inference for the planner, and the pass timing harness that produces its
// training data.
//
// Network: x (kNumFeatures) -> ReLU(W1 x + b1) (kH1) -> ReLU(W2 h1 + b2) (kH2)
// -> y = W3 h2 + b3, trained on log-microseconds with the mean squared error.
// Weights are one flat FP32 array W1 (kH1 x F, row-major), b1, W2 (kH2 x kH1),
// b2, W3 (kH2), b3.  Gradient reductions over the batch are done one weight
// per thread in sample order, so training is deterministic.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

namespace qs {
namespace {

constexpr int F = kNumFeatures, H1 = kH1, H2 = kH2;
constexpr int OW1 = 0, OB1 = OW1 + H1 * F, OW2 = OB1 + H1, OB2 = OW2 + H2 * H1, OW3 = OB2 + H2, OB3 = OW3 + H2;
static_assert(OB3 + 1 == kNumWeights, "weight layout");

// one thread per sample; h1/h2 may be null (inference)
__global__ __launch_bounds__(256) void k_mlp_fwd(const float *__restrict__ w, const float *__restrict__ X, int B,
                                                 float *__restrict__ h1o, float *__restrict__ h2o,
                                                 float *__restrict__ y) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float x[F], h1[H1];
    for (int j = 0; j < F; ++j) x[j] = X[(size_t)b * F + j];
    for (int i = 0; i < H1; ++i) {
        float z = w[OB1 + i];
        for (int j = 0; j < F; ++j) z = fmaf(w[OW1 + i * F + j], x[j], z);
        h1[i] = z > 0.f ? z : 0.f;
        if (h1o) h1o[(size_t)b * H1 + i] = h1[i];
    }
    float out = w[OB3];
    for (int i = 0; i < H2; ++i) {
        float z = w[OB2 + i];
        for (int j = 0; j < H1; ++j) z = fmaf(w[OW2 + i * H1 + j], h1[j], z);
        const float h = z > 0.f ? z : 0.f;
        if (h2o) h2o[(size_t)b * H2 + i] = h;
        out = fmaf(w[OW3 + i], h, out);
    }
    y[b] = out;
}

// single workgroup: dy = 2 (y - t) / B and the mean squared error (fixed order)
__global__ __launch_bounds__(256) void k_mlp_loss(const float *__restrict__ y, const float *__restrict__ t, int B,
                                                  float *__restrict__ dy, float *__restrict__ loss) {
    __shared__ float sh[256];
    float s = 0;
    for (int b = threadIdx.x; b < B; b += 256) {
        const float d = y[b] - t[b];
        dy[b] = 2.f * d / (float)B;
        s += d * d;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = sh[0] / (float)B;
}

// one thread per sample: dz2 = (dy W3) . [h2 > 0], dz1 = (W2^T dz2) . [h1 > 0]
__global__ __launch_bounds__(256) void k_mlp_delta(const float *__restrict__ w, int B, const float *__restrict__ h1,
                                                   const float *__restrict__ h2, const float *__restrict__ dy,
                                                   float *__restrict__ dz1, float *__restrict__ dz2) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float d2[H2];
    for (int i = 0; i < H2; ++i) {
        d2[i] = h2[(size_t)b * H2 + i] > 0.f ? dy[b] * w[OW3 + i] : 0.f;
        dz2[(size_t)b * H2 + i] = d2[i];
    }
    for (int j = 0; j < H1; ++j) {
        float s = 0;
        for (int i = 0; i < H2; ++i) s = fmaf(w[OW2 + i * H1 + j], d2[i], s);
        dz1[(size_t)b * H1 + j] = h1[(size_t)b * H1 + j] > 0.f ? s : 0.f;
    }
}

// one thread per weight: sum over samples in order
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ X, const float *__restrict__ h1,
                                                  const float *__restrict__ h2, const float *__restrict__ dz1,
                                                  const float *__restrict__ dz2, const float *__restrict__ dy, int B,
                                                  float *__restrict__ g) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kNumWeights) return;
    float s = 0;
    if (idx < OB1) {
        const int i = idx / F, j = idx % F;
        for (int b = 0; b < B; ++b) s = fmaf(dz1[(size_t)b * H1 + i], X[(size_t)b * F + j], s);
    } else if (idx < OW2) {
        const int i = idx - OB1;
        for (int b = 0; b < B; ++b) s += dz1[(size_t)b * H1 + i];
    } else if (idx < OB2) {
        const int i = (idx - OW2) / H1, j = (idx - OW2) % H1;
        for (int b = 0; b < B; ++b) s = fmaf(dz2[(size_t)b * H2 + i], h1[(size_t)b * H1 + j], s);
    } else if (idx < OW3) {
        const int i = idx - OB2;
        for (int b = 0; b < B; ++b) s += dz2[(size_t)b * H2 + i];
    } else if (idx < OB3) {
        const int j = idx - OW3;
        for (int b = 0; b < B; ++b) s = fmaf(dy[b], h2[(size_t)b * H2 + j], s);
    } else {
        for (int b = 0; b < B; ++b) s += dy[b];
    }
    g[idx] = s;
}

__global__ __launch_bounds__(256) void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                                              float *__restrict__ v, float lr, float b1, float b2, float eps, float bc1,
                                              float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNumWeights) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

unsigned blocks_for(int n) { return (unsigned)std::max(1, (n + 255) / 256); }

struct Model {
    std::mutex mu;
    bool loaded = false;
    std::vector<float> w = std::vector<float>(kNumWeights, 0.f);
};
Model g_model;

// device scratch for one forward/backward over B rows
struct Work {
    float *w = nullptr, *X = nullptr, *t = nullptr, *h1 = nullptr, *h2 = nullptr, *y = nullptr, *dy = nullptr,
          *dz1 = nullptr, *dz2 = nullptr, *g = nullptr, *m = nullptr, *v = nullptr, *loss = nullptr;
    int cap = 0;
    ~Work() {
        float *all[] = {w, X, t, h1, h2, y, dy, dz1, dz2, g, m, v, loss};
        for (float *p : all)
            if (p) hipFree(p);
    }
    qs_status alloc(int B) {
        cap = B;
        struct {
            float **p;
            size_t n;
        } req[] = {{&w, (size_t)kNumWeights}, {&X, (size_t)B * F}, {&t, (size_t)B},       {&h1, (size_t)B * H1},
                   {&h2, (size_t)B * H2},      {&y, (size_t)B},     {&dy, (size_t)B},     {&dz1, (size_t)B * H1},
                   {&dz2, (size_t)B * H2},     {&g, (size_t)kNumWeights}, {&m, (size_t)kNumWeights},
                   {&v, (size_t)kNumWeights},  {&loss, (size_t)1}};
        for (auto &r : req) QS_HIP(hipMalloc((void **)r.p, std::max<size_t>(1, r.n) * sizeof(float)));
        return QS_OK;
    }
};

qs_status fwd_bwd(Work &wk, int B) {
    hipLaunchKernelGGL(k_mlp_fwd, dim3(blocks_for(B)), dim3(256), 0, nullptr, wk.w, wk.X, B, wk.h1, wk.h2, wk.y);
    hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, nullptr, wk.y, wk.t, B, wk.dy, wk.loss);
    hipLaunchKernelGGL(k_mlp_delta, dim3(blocks_for(B)), dim3(256), 0, nullptr, wk.w, B, wk.h1, wk.h2, wk.dy, wk.dz1,
                       wk.dz2);
    hipLaunchKernelGGL(k_mlp_grad, dim3(blocks_for(kNumWeights)), dim3(256), 0, nullptr, wk.X, wk.h1, wk.h2, wk.dz1,
                       wk.dz2, wk.dy, B, wk.g);
    QS_HIP(hipGetLastError());
    return QS_OK;
}

// splitmix64 and Box-Muller for the seeded He initialisation
uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
double uniform01(uint64_t &s) { return ((splitmix(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
double normal(uint64_t &s) { return std::sqrt(-2.0 * std::log(uniform01(s))) * std::cos(2 * M_PI * uniform01(s)); }

void he_init(std::vector<float> &w, uint64_t seed) {
    uint64_t s = seed;
    std::fill(w.begin(), w.end(), 0.f);
    for (int i = 0; i < H1 * F; ++i) w[OW1 + i] = (float)(normal(s) * std::sqrt(2.0 / F));
    for (int i = 0; i < H2 * H1; ++i) w[OW2 + i] = (float)(normal(s) * std::sqrt(2.0 / H1));
    for (int i = 0; i < H2; ++i) w[OW3 + i] = (float)(normal(s) * std::sqrt(1.0 / H2));
}

}  // namespace

bool costmodel_loaded() {
    std::lock_guard<std::mutex> lk(g_model.mu);
    return g_model.loaded;
}

qs_status costmodel_predict_device(const float *features, int n_rows, float *out) {
    QS_CHECK(n_rows >= 0, QS_EINVAL, "negative row count");
    if (n_rows == 0) return QS_OK;
    std::vector<float> w;
    {
        std::lock_guard<std::mutex> lk(g_model.mu);
        QS_CHECK(g_model.loaded, QS_EINVAL, "no cost model loaded");
        w = g_model.w;
    }
    float *dw = nullptr, *dX = nullptr, *dy = nullptr;
    QS_HIP(hipMalloc(&dw, kNumWeights * sizeof(float)));
    hipError_t e = hipMalloc(&dX, (size_t)n_rows * F * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&dy, (size_t)n_rows * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(dw, w.data(), kNumWeights * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dX, features, (size_t)n_rows * F * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_mlp_fwd, dim3(blocks_for(n_rows)), dim3(256), 0, nullptr, dw, dX, n_rows, nullptr, nullptr,
                           dy);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out, dy, (size_t)n_rows * sizeof(float), hipMemcpyDeviceToHost);
    hipFree(dw);
    if (dX) hipFree(dX);
    if (dy) hipFree(dy);
    if (e != hipSuccess) return hip_fail(e, "cost-model inference");
    return QS_OK;
}

}  // namespace qs

using namespace qs;

extern "C" {

int qs_costmodel_num_features(void) { return kNumFeatures; }
int qs_costmodel_num_weights(void) { return kNumWeights; }

qs_status qs_costmodel_set_weights(const float *w) {
    std::lock_guard<std::mutex> lk(g_model.mu);
    if (!w) {
        g_model.loaded = false;  // unload: the learned strategy falls back to greedy
        return QS_OK;
    }
    for (int i = 0; i < kNumWeights; ++i)
        QS_CHECK(std::isfinite(w[i]), QS_EINVAL, "non-finite weight %d", i);
    std::copy(w, w + kNumWeights, g_model.w.begin());
    g_model.loaded = true;
    return QS_OK;
}

qs_status qs_costmodel_get_weights(float *w) {
    QS_CHECK(w != nullptr, QS_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(g_model.mu);
    QS_CHECK(g_model.loaded, QS_EINVAL, "no cost model loaded");
    std::copy(g_model.w.begin(), g_model.w.end(), w);
    return QS_OK;
}

qs_status qs_costmodel_predict(const float *features, int n_rows, float *out) {
    QS_CHECK(features && out, QS_EINVAL, "null argument");
    return costmodel_predict_device(features, n_rows, out);
}

qs_status qs_costmodel_grad(const float *weights, const float *features, const float *targets, int n_rows,
                            float *grad_out, float *loss_out) {
    QS_CHECK(weights && features && targets && grad_out && loss_out, QS_EINVAL, "null argument");
    QS_CHECK(n_rows >= 1 && n_rows <= (1 << 20), QS_EINVAL, "n_rows outside 1..2^20");
    Work wk;
    qs_status st = wk.alloc(n_rows);
    if (st != QS_OK) return st;
    QS_HIP(hipMemcpy(wk.w, weights, kNumWeights * sizeof(float), hipMemcpyHostToDevice));
    QS_HIP(hipMemcpy(wk.X, features, (size_t)n_rows * F * sizeof(float), hipMemcpyHostToDevice));
    QS_HIP(hipMemcpy(wk.t, targets, (size_t)n_rows * sizeof(float), hipMemcpyHostToDevice));
    st = fwd_bwd(wk, n_rows);
    if (st != QS_OK) return st;
    QS_HIP(hipMemcpy(grad_out, wk.g, kNumWeights * sizeof(float), hipMemcpyDeviceToHost));
    QS_HIP(hipMemcpy(loss_out, wk.loss, sizeof(float), hipMemcpyDeviceToHost));
    return QS_OK;
}

qs_status qs_costmodel_train(const float *features, const float *targets, int n_rows, int epochs, int batch, float lr,
                             uint64_t seed, const float *init_weights, float *loss_out) {
    QS_CHECK(features && targets, QS_EINVAL, "null argument");
    QS_CHECK(n_rows >= 1 && n_rows <= (1 << 20), QS_EINVAL, "n_rows outside 1..2^20");
    QS_CHECK(epochs >= 1 && batch >= 1 && lr > 0, QS_EINVAL, "bad training hyper-parameters");
    batch = std::min(batch, n_rows);
    std::vector<float> w(kNumWeights);
    if (init_weights) std::copy(init_weights, init_weights + kNumWeights, w.begin());
    else he_init(w, seed);
    Work wk;
    qs_status st = wk.alloc(batch);
    if (st != QS_OK) return st;
    QS_HIP(hipMemcpy(wk.w, w.data(), kNumWeights * sizeof(float), hipMemcpyHostToDevice));
    QS_HIP(hipMemset(wk.m, 0, kNumWeights * sizeof(float)));
    QS_HIP(hipMemset(wk.v, 0, kNumWeights * sizeof(float)));
    std::vector<int> perm(n_rows);
    std::vector<float> bx((size_t)batch * F), bt(batch);
    uint64_t rs = seed ^ 0x5bd1e995ull;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    int step = 0;
    float last = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int i = 0; i < n_rows; ++i) perm[i] = i;
        for (int i = n_rows - 1; i > 0; --i) std::swap(perm[i], perm[splitmix(rs) % (uint64_t)(i + 1)]);
        double ep_loss = 0;
        int nb = 0;
        for (int s = 0; s + batch <= n_rows; s += batch) {
            for (int r = 0; r < batch; ++r) {
                std::memcpy(&bx[(size_t)r * F], features + (size_t)perm[s + r] * F, F * sizeof(float));
                bt[r] = targets[perm[s + r]];
            }
            QS_HIP(hipMemcpy(wk.X, bx.data(), bx.size() * sizeof(float), hipMemcpyHostToDevice));
            QS_HIP(hipMemcpy(wk.t, bt.data(), bt.size() * sizeof(float), hipMemcpyHostToDevice));
            st = fwd_bwd(wk, batch);
            if (st != QS_OK) return st;
            ++step;
            const float bc1 = 1.f - std::pow(b1, (float)step), bc2 = 1.f - std::pow(b2, (float)step);
            hipLaunchKernelGGL(k_adam, dim3(blocks_for(kNumWeights)), dim3(256), 0, nullptr, wk.w, wk.g, wk.m, wk.v, lr,
                               b1, b2, eps, bc1, bc2);
            QS_HIP(hipGetLastError());
            float l = 0;
            QS_HIP(hipMemcpy(&l, wk.loss, sizeof(float), hipMemcpyDeviceToHost));
            ep_loss += l;
            ++nb;
        }
        last = nb ? (float)(ep_loss / nb) : 0.f;
    }
    QS_HIP(hipMemcpy(w.data(), wk.w, kNumWeights * sizeof(float), hipMemcpyDeviceToHost));
    if (loss_out) *loss_out = last;
    return qs_costmodel_set_weights(w.data());
}

qs_status qs_plan_pass_features(qs_plan p, float *out, uint64_t cap_rows) {
    QS_ABI_TRY
    QS_CHECK(p && out, QS_EINVAL, "null argument");
    QS_CHECK(cap_rows >= p->passes.size(), QS_ERANGE, "need %zu rows", p->passes.size());
    const qs_dtype dt = p->opts.dtype == QS_C128 ? QS_C128 : QS_C64;
    for (size_t i = 0; i < p->passes.size(); ++i) pass_features(p->n, dt, p->passes[i], p->blocks, out + i * kNumFeatures);
    return QS_OK;
    QS_ABI_CATCH
}

qs_status qs_plan_time_passes(qs_plan p, qs_dtype dtype, int reps, double *us_out) {
    QS_ABI_TRY
    QS_CHECK(p && us_out, QS_EINVAL, "null argument");
    QS_CHECK(reps >= 1 && reps <= 100, QS_EINVAL, "reps outside 1..100");
    qs_state s = nullptr;
    qs_status st = qs_state_create(p->n, dtype, nullptr, nullptr, &s);
    if (st != QS_OK) return st;
    st = qs_state_set_basis(s, 0);
    if (st == QS_OK) st = plan_upload(*p, dtype);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    std::vector<float> t(reps);
    for (size_t i = 0; st == QS_OK && i < p->passes.size(); ++i) {
        st = launch_pass(*s, *p, p->passes[i], (int64_t)i, false, false);  // warm
        for (int r = 0; st == QS_OK && r < reps; ++r) {
            hipEventRecord(e0, nullptr);
            st = launch_pass(*s, *p, p->passes[i], (int64_t)i, false, false);
            hipEventRecord(e1, nullptr);
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t[r], e0, e1) != hipSuccess) {
                set_error("pass timing failed");
                st = QS_EDEVICE;
            }
        }
        std::sort(t.begin(), t.end());
        us_out[i] = 1000.0 * t[reps / 2];
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    qs_state_destroy(s);
    return st;
    QS_ABI_CATCH
}

}  // extern "C"
