// C ABI of the schedule selector: features of a request, the perceptron's training steps and
// the AUTO choice between the three schedules.
#include "../../include/qsd_select.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "plan.h"
#include "select_kernels.h"

namespace qsd {
qsd_status desc_status(const qsd_desc* d);
}

using namespace qsd;

struct qsd_model_s {
    float* params = nullptr;  // device
    float margin = 0.f;
    int64_t min_nnz = 0;
};

namespace {

constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// selector workspace: counts | features | outputs
constexpr size_t kWsCounts = 0;
constexpr size_t kWsFeat = 256;
constexpr size_t kWsOut = 512;
constexpr size_t kWsBytes = 1024;

uint64_t splitmix_next(uint64_t& state) {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint32_t mode_mask(const std::vector<int>& modes) {
    uint32_t m = 0;
    for (int x : modes) m |= 1u << x;
    return m;
}

// Pass and key-bit counts of the three schedules (minimal, Top-K, full LSD) and the mode
// sets whose joint changes size their buckets.
struct PlanTerms {
    int s1_plain_calls = 0, s1_bucket_calls = 0, s1_plain_bits = 0, s1_bucket_bits = 0;
    int s2_plain_bits = 0, s2_bucket_bits = 0, s3_bits = 0;
    uint32_t prefix1 = 0, prefix2 = 0;
};

PlanTerms plan_terms(int r, const int* bits, const int* in_order, const int* out_order) {
    PlanTerms t;
    for (const Call& c : quesadilla_calls(r, in_order, out_order)) {
        if (c.prefix.empty()) {
            ++t.s1_plain_calls;
            t.s1_plain_bits += bits[c.mode];
        } else {
            if (!t.s1_bucket_calls) t.prefix1 = mode_mask(c.prefix);
            ++t.s1_bucket_calls;
            t.s1_bucket_bits += bits[c.mode];
        }
    }
    const int K = std::max(0, std::min(2, r - 2));
    int target[kMaxR], n = 0;
    for (int i = 0; i < K; ++i) target[n++] = out_order[i];
    for (int i = 0; i < r; ++i) {
        bool head = false;
        for (int j = 0; j < K; ++j) head |= out_order[j] == in_order[i];
        if (!head) target[n++] = in_order[i];
    }
    for (const Call& c : quesadilla_calls(r, in_order, target)) {
        if (c.prefix.empty())
            t.s2_plain_bits += bits[c.mode];
        else
            t.s2_bucket_bits += bits[c.mode];
    }
    if (K > 0) {
        for (int i = K; i < r; ++i) t.s2_bucket_bits += bits[out_order[i]];
        t.prefix2 = mode_mask(std::vector<int>(out_order, out_order + K));
    }
    for (int m = 0; m < r; ++m) t.s3_bits += bits[m];
    return t;
}

double linear_count(uint32_t zero) {
    const double M = (double)kFeatMapBits;
    return zero == 0 ? M * std::log(M) : -M * std::log((double)zero / M);
}

void finish_features(const qsd_desc* d, const PlanTerms& t, const int* bits, const uint32_t* counts, uint32_t S,
                     uint32_t pairs, float* out) {
    const int r = d->order;
    const double n = (double)d->nnz;
    double f[kNFeat] = {};
    f[0] = d->nnz > 0 ? std::log2(n) / 32.0 : 0.0;
    f[1] = r / 8.0;
    for (int i = 0; i < std::min(r, 5); ++i) {
        const int m = d->out_order[i];
        const uint32_t zero = counts[3 * m], top = counts[3 * m + 1], change = counts[3 * m + 2];
        f[2 + 4 * i] = bits[m] / 32.0;
        f[3 + 4 * i] = S ? std::log2(1.0 + linear_count(zero)) / 24.0 : 0.0;
        f[4 + 4 * i] = pairs ? (double)change / pairs : 0.0;
        f[5 + 4 * i] = S ? (double)top / S : 0.0;
    }
    f[22] = t.s1_plain_calls / 8.0;
    f[23] = t.s1_bucket_calls / 8.0;
    f[24] = t.s1_plain_bits / 64.0;
    f[25] = t.s1_bucket_bits / 64.0;
    f[26] = t.s2_plain_bits / 64.0;
    f[27] = t.s2_bucket_bits / 64.0;
    f[28] = t.s3_bits / 64.0;
    f[29] = (pairs && t.prefix1) ? (double)counts[3 * r] / pairs : 0.0;
    f[30] = (pairs && t.prefix2) ? (double)counts[3 * (r + 1)] / pairs : 0.0;
    f[31] = std::log2(1.0 + f[29] * n) / 32.0;
    for (int i = 0; i < kNFeat; ++i) out[i] = (float)f[i];
}

qsd_status counts_impl(const qsd_desc* d, const void* const* in_crd, void* ws, size_t ws_bytes, hipStream_t s,
                       const PlanTerms& t, uint32_t* counts, uint32_t* S_out, uint32_t* pairs_out) {
    std::memset(counts, 0, sizeof(uint32_t) * QSD_FEAT_COUNTS);
    const uint64_t n = (uint64_t)d->nnz;
    const uint32_t S = (uint32_t)std::min<uint64_t>(n, kFeatSample);
    uint32_t pairs = 0;
    for (uint32_t k = 0; k < S; ++k)
        if ((uint64_t)k * n / S + 1 < n) ++pairs;
    *S_out = S;
    *pairs_out = pairs;
    if (n == 0) return QSD_OK;
    if (!in_crd) return QSD_ERR_NULL;
    for (int m = 0; m < d->order; ++m)
        if (!in_crd[m]) return QSD_ERR_NULL;
    if (!ws || ws_bytes < kWsBytes) return QSD_ERR_WORKSPACE;
    FeatArgs a{};
    for (int m = 0; m < d->order; ++m) a.crd[m] = in_crd[m];
    a.r = d->order;
    a.S = S;
    a.n = n;
    a.mask[0] = t.prefix1;
    a.mask[1] = t.prefix2;
    uint32_t* dev = (uint32_t*)((char*)ws + kWsCounts);
    a.out = dev;
    if (launch_feat(a, d->crd_type == QSD_I64 ? 8 : 4, s) != hipSuccess) return QSD_ERR_HIP;
    if (hipMemcpyAsync(counts, dev, sizeof(uint32_t) * 3 * (d->order + 2), hipMemcpyDeviceToHost, s) != hipSuccess)
        return QSD_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return QSD_ERR_HIP;
    return QSD_OK;
}

void desc_bits(const qsd_desc* d, int* bits) {
    for (int m = 0; m < d->order; ++m) bits[m] = bits_for_extent(d->extents[m]);
}

}  // namespace

extern "C" {

qsd_status qsd_select_workspace(size_t* bytes) {
    if (!bytes) return QSD_ERR_NULL;
    *bytes = kWsBytes;
    return QSD_OK;
}

qsd_status qsd_feature_counts(const qsd_desc* desc, const void* const* in_crd, void* ws, size_t ws_bytes,
                              hipStream_t stream, uint32_t* counts_host, uint32_t* sample, uint32_t* pairs) {
    if (!counts_host || !sample || !pairs) return QSD_ERR_NULL;
    const qsd_status st = desc_status(desc);
    if (st != QSD_OK) return st;
    int bits[kMaxR];
    desc_bits(desc, bits);
    const PlanTerms t = plan_terms(desc->order, bits, desc->in_order, desc->out_order);
    return counts_impl(desc, in_crd, ws, ws_bytes, stream, t, counts_host, sample, pairs);
}

qsd_status qsd_features(const qsd_desc* desc, const void* const* in_crd, void* ws, size_t ws_bytes,
                        hipStream_t stream, float* feat_host) {
    if (!feat_host) return QSD_ERR_NULL;
    qsd_status st = desc_status(desc);
    if (st != QSD_OK) return st;
    int bits[kMaxR];
    desc_bits(desc, bits);
    const PlanTerms t = plan_terms(desc->order, bits, desc->in_order, desc->out_order);
    uint32_t counts[QSD_FEAT_COUNTS], S = 0, pairs = 0;
    if ((st = counts_impl(desc, in_crd, ws, ws_bytes, stream, t, counts, &S, &pairs)) != QSD_OK) return st;
    finish_features(desc, t, bits, counts, S, pairs, feat_host);
    return QSD_OK;
}

qsd_status qsd_mlp_init(uint64_t seed, float* params_host) {
    if (!params_host) return QSD_ERR_NULL;
    uint64_t state = seed;
    std::fill(params_host, params_host + kNParam, 0.f);
    const int fan_in[3] = {kNFeat, kH1, kH2}, fan_out[3] = {kH1, kH2, kNOut}, off[3] = {kOffW1, kOffW2, kOffW3};
    for (int l = 0; l < 3; ++l) {
        const double a = std::sqrt(6.0 / fan_in[l]);
        for (int k = 0; k < fan_in[l] * fan_out[l]; ++k) {
            const double u = (double)(splitmix_next(state) >> 11) * (1.0 / 9007199254740992.0);
            params_host[off[l] + k] = (float)((2.0 * u - 1.0) * a);
        }
    }
    return QSD_OK;
}

qsd_status qsd_mlp_forward(const float* params_dev, const float* x_dev, int32_t n, float* h1_dev, float* h2_dev,
                           float* y_dev, hipStream_t stream) {
    if (n < 0) return QSD_ERR_TOO_LARGE;
    if (n == 0) return QSD_OK;
    if (!params_dev || !x_dev || !y_dev) return QSD_ERR_NULL;
    return launch_mlp_fwd(params_dev, x_dev, n, h1_dev, h2_dev, y_dev, stream) == hipSuccess ? QSD_OK : QSD_ERR_HIP;
}

qsd_status qsd_mlp_backward_workspace(int32_t n, size_t* bytes) {
    if (!bytes) return QSD_ERR_NULL;
    if (n < 0) return QSD_ERR_TOO_LARGE;
    const size_t N = (size_t)std::max(n, 1);
    *bytes = up(N * kH1 * 4) + up(N * kH2 * 4) + up(N * kNOut * 4) + up(N * 4);
    return QSD_OK;
}

qsd_status qsd_mlp_backward(const float* params_dev, const float* x_dev, const float* h1_dev, const float* h2_dev,
                            const float* y_dev, const float* t_dev, int32_t n, float* grad_dev, float* loss_dev,
                            void* ws, size_t ws_bytes, hipStream_t stream) {
    if (n <= 0) return QSD_ERR_TOO_LARGE;
    if (!params_dev || !x_dev || !h1_dev || !h2_dev || !y_dev || !t_dev || !grad_dev || !loss_dev || !ws)
        return QSD_ERR_NULL;
    size_t need = 0;
    qsd_mlp_backward_workspace(n, &need);
    if (ws_bytes < need) return QSD_ERR_WORKSPACE;
    char* w = (char*)ws;
    const size_t N = (size_t)n;
    float* D1 = (float*)w;
    float* D2 = (float*)(w + up(N * kH1 * 4));
    float* D3 = (float*)(w + up(N * kH1 * 4) + up(N * kH2 * 4));
    float* RL = (float*)(w + up(N * kH1 * 4) + up(N * kH2 * 4) + up(N * kNOut * 4));
    if (launch_mlp_delta(params_dev, h1_dev, h2_dev, y_dev, t_dev, n, D1, D2, D3, RL, stream) != hipSuccess ||
        launch_mlp_grad(x_dev, h1_dev, h2_dev, D1, D2, D3, n, grad_dev, stream) != hipSuccess ||
        launch_sum(RL, n, 1.0f / ((float)n * (float)kNOut), loss_dev, stream) != hipSuccess)
        return QSD_ERR_HIP;
    return QSD_OK;
}

qsd_status qsd_mlp_adam(float* params_dev, const float* grad_dev, float* m_dev, float* v_dev, int32_t step,
                        float lr, float beta1, float beta2, float eps, hipStream_t stream) {
    if (!params_dev || !grad_dev || !m_dev || !v_dev) return QSD_ERR_NULL;
    if (step < 1) return QSD_ERR_UNSUPPORTED;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, step)));
    return launch_adam(params_dev, grad_dev, m_dev, v_dev, lr, beta1, beta2, eps, c1, c2, stream) == hipSuccess
               ? QSD_OK
               : QSD_ERR_HIP;
}

namespace {
struct TrainLayout {
    size_t order, xb, tb, h1, h2, y, bw, grad, m, v, loss, total;
};
TrainLayout train_layout(int32_t n, int32_t batch) {
    TrainLayout L{};
    const size_t B = (size_t)std::max(batch, 1);
    size_t at = 0;
    L.order = at;
    at = up(at + (size_t)std::max(n, 1) * 4);
    L.xb = at;
    at = up(at + B * kNFeat * 4);
    L.tb = at;
    at = up(at + B * kNOut * 4);
    L.h1 = at;
    at = up(at + B * kH1 * 4);
    L.h2 = at;
    at = up(at + B * kH2 * 4);
    L.y = at;
    at = up(at + B * kNOut * 4);
    L.bw = at;
    size_t bw = 0;
    qsd_mlp_backward_workspace((int32_t)B, &bw);
    at = up(at + bw);
    L.grad = at;
    at = up(at + kNParam * 4);
    L.m = at;
    at = up(at + kNParam * 4);
    L.v = at;
    at = up(at + kNParam * 4);
    L.loss = at;
    at = up(at + 4);
    L.total = at;
    return L;
}
}  // namespace

qsd_status qsd_mlp_train_workspace(int32_t n, int32_t batch, size_t* bytes) {
    if (!bytes) return QSD_ERR_NULL;
    if (n < 0 || batch < 1) return QSD_ERR_TOO_LARGE;
    *bytes = train_layout(n, batch).total;
    return QSD_OK;
}

qsd_status qsd_mlp_train(float* params_dev, const float* x_dev, const float* t_dev, int32_t n, int32_t epochs,
                         int32_t batch, float lr, uint64_t seed, void* ws, size_t ws_bytes, hipStream_t stream,
                         float* last_loss) {
    if (!params_dev || !x_dev || !t_dev || !ws || !last_loss) return QSD_ERR_NULL;
    if (n < 1 || batch < 1 || epochs < 0) return QSD_ERR_TOO_LARGE;
    const TrainLayout L = train_layout(n, batch);
    if (ws_bytes < L.total) return QSD_ERR_WORKSPACE;
    char* W = (char*)ws;
    uint32_t* order_dev = (uint32_t*)(W + L.order);
    float *Xb = (float*)(W + L.xb), *Tb = (float*)(W + L.tb), *H1 = (float*)(W + L.h1), *H2 = (float*)(W + L.h2);
    float *Y = (float*)(W + L.y), *G = (float*)(W + L.grad), *M = (float*)(W + L.m), *V = (float*)(W + L.v);
    float* loss = (float*)(W + L.loss);
    size_t bw = 0;
    qsd_mlp_backward_workspace(batch, &bw);
    if (hipMemsetAsync(M, 0, kNParam * 4, stream) != hipSuccess || hipMemsetAsync(V, 0, kNParam * 4, stream) != hipSuccess ||
        hipMemsetAsync(loss, 0, 4, stream) != hipSuccess)
        return QSD_ERR_HIP;
    uint64_t state = seed;
    std::vector<uint32_t> order(n);
    int32_t step = 0;
    qsd_status st = QSD_OK;
    for (int e = 0; e < epochs; ++e) {
        for (int32_t i = 0; i < n; ++i) order[i] = (uint32_t)i;
        for (int32_t i = n - 1; i > 0; --i) {
            const uint64_t j = splitmix_next(state) % (uint64_t)(i + 1);
            std::swap(order[i], order[j]);
        }
        // the previous epoch's batches read order_dev: wait before replacing it
        if (hipStreamSynchronize(stream) != hipSuccess ||
            hipMemcpyAsync(order_dev, order.data(), (size_t)n * 4, hipMemcpyHostToDevice, stream) != hipSuccess)
            return QSD_ERR_HIP;
        for (int32_t s = 0; s < n; s += batch) {
            const int32_t nb = std::min(batch, n - s);
            if (launch_gather_rows(x_dev, t_dev, order_dev + s, nb, Xb, Tb, stream) != hipSuccess) return QSD_ERR_HIP;
            if ((st = qsd_mlp_forward(params_dev, Xb, nb, H1, H2, Y, stream)) != QSD_OK) return st;
            if ((st = qsd_mlp_backward(params_dev, Xb, H1, H2, Y, Tb, nb, G, loss, W + L.bw, bw, stream)) != QSD_OK)
                return st;
            if ((st = qsd_mlp_adam(params_dev, G, M, V, ++step, lr, 0.9f, 0.999f, 1e-8f, stream)) != QSD_OK) return st;
        }
    }
    if (hipMemcpyAsync(last_loss, loss, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return QSD_ERR_HIP;
    return QSD_OK;
}

qsd_status qsd_model_create(const float* params_host, float margin, int64_t min_nnz, qsd_model_t* out) {
    if (!params_host || !out) return QSD_ERR_NULL;
    *out = nullptr;
    if (!std::isfinite(margin) || margin < 0.f || min_nnz < 0) return QSD_ERR_UNSUPPORTED;
    for (int i = 0; i < kNParam; ++i)
        if (!std::isfinite(params_host[i])) return QSD_ERR_UNSUPPORTED;
    auto* m = new qsd_model_s();
    m->margin = margin;
    m->min_nnz = min_nnz;
    if (hipMalloc(&m->params, kNParam * sizeof(float)) != hipSuccess) {
        delete m;
        return QSD_ERR_HIP;
    }
    if (hipMemcpy(m->params, params_host, kNParam * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(m->params);
        delete m;
        return QSD_ERR_HIP;
    }
    *out = m;
    return QSD_OK;
}

qsd_status qsd_model_load(const char* path, qsd_model_t* out) {
    if (!path || !out) return QSD_ERR_NULL;
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return QSD_ERR_NULL;
    char magic[8];
    int32_t np = 0;
    float margin = 0.f;
    int64_t min_nnz = 0;
    std::vector<float> p(kNParam);
    const bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "QSDMLP1", 8) == 0 &&
                    std::fread(&np, 4, 1, f) == 1 && np == kNParam && std::fread(&margin, 4, 1, f) == 1 &&
                    std::fread(&min_nnz, 8, 1, f) == 1 && std::fread(p.data(), 4, kNParam, f) == (size_t)kNParam;
    std::fclose(f);
    if (!ok) return QSD_ERR_UNSUPPORTED;
    return qsd_model_create(p.data(), margin, min_nnz, out);
}

void qsd_model_destroy(qsd_model_t m) {
    if (!m) return;
    if (m->params) hipFree(m->params);
    delete m;
}

qsd_status qsd_select(qsd_model_t model, const qsd_desc* desc, const void* const* in_crd, void* ws, size_t ws_bytes,
                      hipStream_t stream, qsd_sched_t* chosen, float* predicted_host) {
    if (!model || !chosen) return QSD_ERR_NULL;
    qsd_status st = desc_status(desc);
    if (st != QSD_OK) return st;
    *chosen = QSD_SCHED_MINIMAL;
    if (desc->nnz < model->min_nnz) return QSD_OK;  // too small for the choice to pay for itself
    float feat[kNFeat];
    if ((st = qsd_features(desc, in_crd, ws, ws_bytes, stream, feat)) != QSD_OK) return st;
    for (float v : feat)
        if (!std::isfinite(v) || v < 0.f || v > 4.f) return QSD_OK;  // outside the trained range
    if (!ws || ws_bytes < kWsBytes) return QSD_ERR_WORKSPACE;
    float* fdev = (float*)((char*)ws + kWsFeat);
    float* ydev = (float*)((char*)ws + kWsOut);
    float y[kNOut];
    if (hipMemcpyAsync(fdev, feat, sizeof(feat), hipMemcpyHostToDevice, stream) != hipSuccess ||
        launch_mlp_fwd(model->params, fdev, 1, nullptr, nullptr, ydev, stream) != hipSuccess ||
        hipMemcpyAsync(y, ydev, sizeof(y), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return QSD_ERR_HIP;
    if (predicted_host) std::copy(y, y + kNOut, predicted_host);
    int best = 0;
    for (int s = 1; s < kNOut; ++s)
        if (y[s] < y[0] - model->margin && y[s] < y[best]) best = s;
    *chosen = (qsd_sched_t)(QSD_SCHED_MINIMAL + best);
    return QSD_OK;
}

qsd_status qsd_plan_auto(qsd_model_t model, const qsd_desc* desc, const void* const* in_crd, void* ws,
                         size_t ws_bytes, hipStream_t stream, qsd_plan_t* out, qsd_sched_t* chosen) {
    if (!out) return QSD_ERR_NULL;
    qsd_sched_t s = QSD_SCHED_MINIMAL;
    const qsd_status st = qsd_select(model, desc, in_crd, ws, ws_bytes, stream, &s, nullptr);
    if (st != QSD_OK) return st;
    if (chosen) *chosen = s;
    return qsd_plan(desc, s, out);
}

}  // extern "C"
