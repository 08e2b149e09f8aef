// C ABI of the schedule selector: features of a request, the perceptron's training steps and
// the AUTO choice between the candidate schedules.
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

// selector workspace: sampled counts | result of k_select (candidate, predictions, features)
constexpr size_t kWsCounts = 0;
constexpr size_t kWsOut = 512;
constexpr size_t kWsBytes = 1024;
static_assert(QSD_FEAT_COUNTS * 4 <= kWsOut && kWsOut + kSelectOutFloats * 4 <= kWsBytes, "selector workspace");

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

// The candidate schedules of the selector and, for each valid one, the plan terms of its
// groups as the library runs them; the mode sets whose joint changes size their buckets.
struct PlanTerms {
    int valid[kNOut] = {};
    int gp[kNOut] = {}, sb[kNOut] = {};
    uint32_t set[kNSets] = {};
};

constexpr int kCandSched[kNOut] = {kSchedMinimal, kSchedMinimal, kSchedTopK + 1, kSchedTopK + 2, kSchedTopK + 3,
                                   kSchedLsd};
constexpr uint32_t kCandFlags[kNOut] = {0u, kKeepBuckets, 0u, 0u, 0u, 0u};

PlanTerms plan_terms(const qsd_desc* d, const int* bits) {
    PlanTerms t;
    const int r = d->order;
    int segmented[2] = {0, 0};
    for (int c = 0; c < kNOut; ++c) {
        const int sched = kCandSched[c];
        if (sched >= kSchedTopK && sched - kSchedTopK > r - 2) continue;  // K = r - 1 is MINIMAL
        if (sched == kSchedLsd && r < 2) continue;
        PlanData p;
        p.r = r;
        p.nnz = d->nnz;
        p.flags = kCandFlags[c];
        for (int m = 0; m < r; ++m) {
            p.ext[m] = d->extents[m];
            p.bits[m] = bits[m];
            p.in_order[m] = d->in_order[m];
            p.out_order[m] = d->out_order[m];
        }
        if (!build_plan(p, sched)) continue;
        t.valid[c] = 1;
        for (const Group& g : p.groups) {
            int passes = 0;
            for (const auto& sk : g.subs) passes += (int)sk.passes.size();
            if (g.segmented) {
                t.sb[c] += g.key_bits;
                if (c < 2) ++segmented[c];
            } else {
                t.gp[c] += passes;
            }
        }
    }
    // keeping the buckets is a candidate of its own only where the minimal plan flattens some
    if (t.valid[1] && segmented[1] == segmented[0]) t.valid[1] = 0;
    for (const Call& c : quesadilla_calls(r, d->in_order, d->out_order))
        if (!c.prefix.empty()) {
            t.set[0] = mode_mask(c.prefix);
            break;
        }
    for (int K = 1; K <= 3; ++K)
        if (K <= r - 2) t.set[K] = mode_mask(std::vector<int>(d->out_order, d->out_order + K));
    return t;
}

uint32_t sample_size(uint64_t n) { return (uint32_t)std::min<uint64_t>(n, kFeatSample); }

uint32_t sample_pairs(uint64_t n) {
    const uint32_t S = sample_size(n);
    uint32_t pairs = 0;
    for (uint32_t k = 0; k < S; ++k)
        if ((uint64_t)k * n / S + 1 < n) ++pairs;
    return pairs;
}

// k_feat for a request: its counts land at the start of the workspace (no host copy).
qsd_status launch_counts(const qsd_desc* d, const void* const* in_crd, void* ws, size_t ws_bytes, hipStream_t s,
                         const PlanTerms& t) {
    const uint64_t n = (uint64_t)d->nnz;
    if (n > 0) {
        if (!in_crd) return QSD_ERR_NULL;
        for (int m = 0; m < d->order; ++m)
            if (!in_crd[m]) return QSD_ERR_NULL;
    }
    if (!ws || ws_bytes < kWsBytes) return QSD_ERR_WORKSPACE;
    FeatArgs a{};
    for (int m = 0; m < d->order; ++m) a.crd[m] = n ? in_crd[m] : nullptr;
    a.r = d->order;
    a.S = sample_size(n);
    a.n = n;
    for (int q = 0; q < kNSets; ++q) a.mask[q] = t.set[q];
    a.out = (uint32_t*)((char*)ws + kWsCounts);
    return launch_feat(a, d->crd_type == QSD_I64 ? 8 : 4, s) == hipSuccess ? QSD_OK : QSD_ERR_HIP;
}

void desc_bits(const qsd_desc* d, int* bits) {
    for (int m = 0; m < d->order; ++m) bits[m] = bits_for_extent(d->extents[m]);
}

// Sampling, features and (with params) the forward pass and the choice, on the device; one
// copy of the result back and one synchronisation.  out: kSelectOutFloats floats.
qsd_status select_impl(const qsd_desc* d, const void* const* in_crd, void* ws, size_t ws_bytes, hipStream_t s,
                       const float* params, float margin, float* out) {
    int bits[kMaxR];
    desc_bits(d, bits);
    const PlanTerms t = plan_terms(d, bits);
    qsd_status st = launch_counts(d, in_crd, ws, ws_bytes, s, t);
    if (st != QSD_OK) return st;
    SelectArgs a{};
    a.counts = (const uint32_t*)((char*)ws + kWsCounts);
    a.r = d->order;
    a.n = (double)d->nnz;
    a.S = sample_size((uint64_t)d->nnz);
    a.pairs = sample_pairs((uint64_t)d->nnz);
    for (int i = 0; i < 5 && i < d->order; ++i) a.slot_mode[i] = d->out_order[i];
    for (int m = 0; m < d->order; ++m) a.bits[m] = bits[m];
    a.crd_bytes = d->crd_type == QSD_I64 ? 8 : 4;
    a.val_bytes = d->val_type == QSD_F64 ? 8 : 4;
    for (int c = 0; c < kNOut; ++c) {
        a.valid[c] = t.valid[c];
        a.gp[c] = t.gp[c];
        a.sb[c] = t.sb[c];
    }
    for (int q = 0; q < kNSets; ++q) a.set_nonempty[q] = t.set[q] != 0;
    a.params = params;
    a.margin = margin;
    a.out = (float*)((char*)ws + kWsOut);
    if (launch_select(a, s) != hipSuccess ||
        hipMemcpyAsync(out, a.out, kSelectOutFloats * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return QSD_ERR_HIP;
    return QSD_OK;
}

}  // namespace

extern "C" {

qsd_status qsd_select_workspace(size_t* bytes) {
    if (!bytes) return QSD_ERR_NULL;
    *bytes = kWsBytes;
    return QSD_OK;
}

qsd_status qsd_candidate(int32_t candidate, qsd_sched_t* sched, uint32_t* flags) {
    if (!sched || !flags) return QSD_ERR_NULL;
    if (candidate < 0 || candidate >= kNOut) return QSD_ERR_UNSUPPORTED;
    *sched = (qsd_sched_t)kCandSched[candidate];
    *flags = kCandFlags[candidate];
    return QSD_OK;
}

qsd_status qsd_candidate_terms(const qsd_desc* desc, int32_t* valid_host, int32_t* passes_host,
                               int32_t* bucket_bits_host) {
    if (!valid_host) return QSD_ERR_NULL;
    const qsd_status st = desc_status(desc);
    if (st != QSD_OK) return st;
    int bits[kMaxR];
    desc_bits(desc, bits);
    const PlanTerms t = plan_terms(desc, bits);
    for (int c = 0; c < kNOut; ++c) {
        valid_host[c] = t.valid[c];
        if (passes_host) passes_host[c] = t.valid[c] ? t.gp[c] : 0;
        if (bucket_bits_host) bucket_bits_host[c] = t.valid[c] ? t.sb[c] : 0;
    }
    return QSD_OK;
}

qsd_status qsd_feature_counts(const qsd_desc* desc, const void* const* in_crd, void* ws, size_t ws_bytes,
                              hipStream_t stream, uint32_t* counts_host, uint32_t* sample, uint32_t* pairs) {
    if (!counts_host || !sample || !pairs) return QSD_ERR_NULL;
    qsd_status st = desc_status(desc);
    if (st != QSD_OK) return st;
    int bits[kMaxR];
    desc_bits(desc, bits);
    const PlanTerms t = plan_terms(desc, bits);
    std::memset(counts_host, 0, sizeof(uint32_t) * QSD_FEAT_COUNTS);
    *sample = sample_size((uint64_t)desc->nnz);
    *pairs = sample_pairs((uint64_t)desc->nnz);
    if (desc->nnz == 0) return QSD_OK;
    if ((st = launch_counts(desc, in_crd, ws, ws_bytes, stream, t)) != QSD_OK) return st;
    if (hipMemcpyAsync(counts_host, (char*)ws + kWsCounts, sizeof(uint32_t) * 3 * (desc->order + kNSets),
                       hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return QSD_ERR_HIP;
    return QSD_OK;
}

qsd_status qsd_features(const qsd_desc* desc, const void* const* in_crd, void* ws, size_t ws_bytes,
                        hipStream_t stream, float* feat_host) {
    if (!feat_host) return QSD_ERR_NULL;
    qsd_status st = desc_status(desc);
    if (st != QSD_OK) return st;
    float out[kSelectOutFloats];
    if ((st = select_impl(desc, in_crd, ws, ws_bytes, stream, nullptr, 0.f, out)) != QSD_OK) return st;
    std::copy(out + 8, out + 8 + kNFeat, feat_host);
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
        (void)hipFree(m->params);
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
    const bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "QSDMLP2", 8) == 0 &&
                    std::fread(&np, 4, 1, f) == 1 && np == kNParam && std::fread(&margin, 4, 1, f) == 1 &&
                    std::fread(&min_nnz, 8, 1, f) == 1 && std::fread(p.data(), 4, kNParam, f) == (size_t)kNParam;
    std::fclose(f);
    if (!ok) return QSD_ERR_UNSUPPORTED;
    return qsd_model_create(p.data(), margin, min_nnz, out);
}

void qsd_model_destroy(qsd_model_t m) {
    if (!m) return;
    if (m->params) (void)hipFree(m->params);
    delete m;
}

qsd_status qsd_select(qsd_model_t model, const qsd_desc* desc, const void* const* in_crd, void* ws, size_t ws_bytes,
                      hipStream_t stream, int32_t* candidate, float* predicted_host) {
    if (!model || !candidate) return QSD_ERR_NULL;
    qsd_status st = desc_status(desc);
    if (st != QSD_OK) return st;
    *candidate = 0;
    if (desc->nnz < model->min_nnz) return QSD_OK;  // too small for the choice to pay for itself
    float out[kSelectOutFloats];
    if ((st = select_impl(desc, in_crd, ws, ws_bytes, stream, model->params, model->margin, out)) != QSD_OK)
        return st;
    int32_t c = 0;
    std::memcpy(&c, &out[0], 4);
    if (c < 0 || c >= kNOut) return QSD_ERR_DEVICE;
    if (predicted_host) std::copy(out + 1, out + 1 + kNOut, predicted_host);
    *candidate = c;
    return QSD_OK;
}

qsd_status qsd_plan_auto(qsd_model_t model, const qsd_desc* desc, const void* const* in_crd, void* ws,
                         size_t ws_bytes, hipStream_t stream, qsd_plan_t* out, int32_t* candidate) {
    if (!out) return QSD_ERR_NULL;
    int32_t c = 0;
    const qsd_status st = qsd_select(model, desc, in_crd, ws, ws_bytes, stream, &c, nullptr);
    if (st != QSD_OK) return st;
    if (candidate) *candidate = c;
    qsd_desc d = *desc;
    d.flags |= kCandFlags[c];
    return qsd_plan(&d, (qsd_sched_t)kCandSched[c], out);
}

}  // extern "C"
