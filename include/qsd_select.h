/* libqsd schedule selector: the true-cost model the paper proposes in place of counting
 * passes (Sec. 5; Sec. 4.2 shows that the fewest passes are not always the fastest, e.g. with
 * large extents).  A small network predicts the run time of each of the three schedules of
 * qsd_plan from 32 features of the request, and AUTO takes the fastest prediction.
 *
 * Features (all sampled on the device from the input, then finished on the host):
 *   With N nonzeros and S = min(N, QSD_FEAT_SAMPLE), positions j_k = floor(k N / S),
 *   k = 0..S-1; a pair (j_k, j_k + 1) is counted when j_k + 1 < N.  Coordinates are hashed
 *   with SplitMix64's output function (Steele, Lea and Flood, OOPSLA 2014) applied to the
 *   coordinate as a signed 64-bit integer.
 *   Per mode m: zero_m = zero bits of a 65536-bit map after setting bit (h mod 2^16) of every
 *   sampled coordinate; top_m = the largest of 1024 bucket counts ((h >> 16) mod 1024);
 *   change_m = pairs whose coordinates in m differ.  For the prefix of the minimal plan's
 *   first bucketed call and for (sigma_1..sigma_K) of the Top-K plan: pairs differing in at
 *   least one mode of the set.
 *   Feature i: 0 log2(N)/32; 1 r/8; per slot s = 0..4 (mode sigma_{s+1}, zero past r):
 *   2+4s bits/32, 3+4s log2(1 + D)/24 with the linear-counting estimate
 *   D = -65536 ln(zero/65536) (65536 ln 65536 when zero = 0), 4+4s change/pairs, 5+4s top/S;
 *   22/23 minimal plan plain/bucketed calls / 8; 24/25 their key bits / 64; 26/27 Top-K plan
 *   plain key bits / 64 and bucketed key bits plus the bits of sigma_{K+1..r} (K > 0) / 64;
 *   28 all key bits / 64; 29 minimal-plan bucket prefix change/pairs; 30 Top-K prefix
 *   change/pairs; 31 log2(1 + f29 N)/32.  (K = min(2, r - 2).)
 *
 * Network: 32 -> 64 -> 64 -> 3, ReLU after both hidden layers, float32.  Output s is the
 * predicted log2 of the run time in ms of schedule s + 1 (MINIMAL, TOP2, LSD).  Parameters are
 * one float array of QSD_MLP_NPARAM entries: W1 (64 x 32, row-major W1[o][i]), b1 (64),
 * W2 (64 x 64), b2 (64), W3 (3 x 64), b3 (3).  Training minimises the mean over rows and
 * outputs of the squared error with Adam (Kingma and Ba, ICLR 2015).
 *
 * Ownership: every pointer named *_dev is device memory owned by the caller; *_host is host
 * memory.  Functions returning a model allocate it (qsd_model_destroy frees it).  Errors as in
 * qsd.h; the training and selection calls synchronise their stream.
 */
#ifndef QSD_SELECT_H
#define QSD_SELECT_H

#include "qsd.h"

#ifdef __cplusplus
extern "C" {
#endif

#define QSD_NFEAT 32
#define QSD_NSCHED 3
#define QSD_FEAT_SAMPLE 16384
#define QSD_MLP_NPARAM 6467
/* counts per mode (zero, top, change) for r modes, then (change, 0, 0) for the two prefixes */
#define QSD_FEAT_COUNTS (3 * (QSD_MAX_ORDER + 2))

/* Device workspace of qsd_feature_counts / qsd_features / qsd_select. */
qsd_status qsd_select_workspace(size_t* bytes);

/* Raw sampled counts of a request (desc->nnz nonzeros at in_crd, device pointers).  counts_host
 * receives QSD_FEAT_COUNTS words; *sample and *pairs receive S and the number of pairs. */
qsd_status qsd_feature_counts(const qsd_desc* desc, const void* const* in_crd, void* ws, size_t ws_bytes,
                              hipStream_t stream, uint32_t* counts_host, uint32_t* sample, uint32_t* pairs);

/* The QSD_NFEAT features of a request (as in the header comment) into feat_host. */
qsd_status qsd_features(const qsd_desc* desc, const void* const* in_crd, void* ws, size_t ws_bytes,
                        hipStream_t stream, float* feat_host);

/* He-uniform initial parameters from a SplitMix64 stream seeded with `seed`: weights
 * (2u - 1) sqrt(6 / fan_in) with u from the top 53 bits of each output, in layout order;
 * biases zero.  Host only. */
qsd_status qsd_mlp_init(uint64_t seed, float* params_host);

/* Forward pass over n rows: x_dev (n x 32), h1_dev and h2_dev (n x 64, post-ReLU),
 * y_dev (n x 3).  h1_dev / h2_dev may be NULL when not needed. */
qsd_status qsd_mlp_forward(const float* params_dev, const float* x_dev, int32_t n, float* h1_dev,
                           float* h2_dev, float* y_dev, hipStream_t stream);

/* Device workspace of qsd_mlp_backward for n rows. */
qsd_status qsd_mlp_backward_workspace(int32_t n, size_t* bytes);

/* Loss (mean squared error against t_dev, n x 3) and its gradient (QSD_MLP_NPARAM floats)
 * for the activations of a forward pass of the same rows.  loss_dev: one float. */
qsd_status qsd_mlp_backward(const float* params_dev, const float* x_dev, const float* h1_dev,
                            const float* h2_dev, const float* y_dev, const float* t_dev, int32_t n,
                            float* grad_dev, float* loss_dev, void* ws, size_t ws_bytes, hipStream_t stream);

/* One Adam update of every parameter; step counts from 1. */
qsd_status qsd_mlp_adam(float* params_dev, const float* grad_dev, float* m_dev, float* v_dev, int32_t step,
                        float lr, float beta1, float beta2, float eps, hipStream_t stream);

/* Minibatch training: `epochs` passes over the n rows (x_dev n x 32, t_dev n x 3), each in a
 * fresh order drawn by Fisher-Yates from a SplitMix64 stream seeded with `seed` (swap index
 * = next() mod (i + 1), i from n - 1 down to 1), in batches of `batch` rows (the last may be
 * shorter), one Adam step per batch (beta1 0.9, beta2 0.999, eps 1e-8).  Updates params_dev in
 * place; *last_loss receives the loss of the last batch.  Synchronises the stream. */
qsd_status qsd_mlp_train_workspace(int32_t n, int32_t batch, size_t* bytes);
qsd_status qsd_mlp_train(float* params_dev, const float* x_dev, const float* t_dev, int32_t n, int32_t epochs,
                         int32_t batch, float lr, uint64_t seed, void* ws, size_t ws_bytes, hipStream_t stream,
                         float* last_loss);

/* A trained selector.  params_host: QSD_MLP_NPARAM floats (copied to the device).  margin:
 * another schedule is chosen only when its predicted log2 time is below MINIMAL's by more
 * than margin (>= 0).  min_nnz: requests with fewer nonzeros take MINIMAL without sampling
 * (the choice cannot pay for itself there).  qsd_model_load reads the file format written by
 * the training tool (little endian): 8 bytes "QSDMLP1\0", int32 nparam, float32 margin,
 * int64 min_nnz, float32 params[nparam]. */
typedef struct qsd_model_s* qsd_model_t;
qsd_status qsd_model_create(const float* params_host, float margin, int64_t min_nnz, qsd_model_t* out);
qsd_status qsd_model_load(const char* path, qsd_model_t* out);
void qsd_model_destroy(qsd_model_t model);

/* Features + forward pass on the device, then the choice: MINIMAL unless another schedule is
 * predicted faster by more than the margin; MINIMAL too below the model's min_nnz (no device
 * work then) and when a feature is not finite or outside [0, 4].  predicted_host (3 floats)
 * may be NULL; it is left untouched when no prediction is made.  Synchronises the stream. */
qsd_status qsd_select(qsd_model_t model, const qsd_desc* desc, const void* const* in_crd, void* ws,
                      size_t ws_bytes, hipStream_t stream, qsd_sched_t* chosen, float* predicted_host);

/* qsd_select, then qsd_plan with the chosen schedule. */
qsd_status qsd_plan_auto(qsd_model_t model, const qsd_desc* desc, const void* const* in_crd, void* ws,
                         size_t ws_bytes, hipStream_t stream, qsd_plan_t* out, qsd_sched_t* chosen);

#ifdef __cplusplus
}
#endif
#endif /* QSD_SELECT_H */
