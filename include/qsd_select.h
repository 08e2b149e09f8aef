/* libqsd schedule selector: the true-cost model the paper proposes in place of counting
 * passes (Sec. 5; Sec. 4.2 shows that the fewest passes are not always the fastest, e.g. with
 * large extents).  A small network predicts the run time of each candidate schedule from 40
 * features of the request, and AUTO takes the fastest prediction.
 *
 * Candidates (every one gives the identical output):
 *   0  MINIMAL, flags 0 (a bucketed group runs as one global sort where that is cheaper)
 *   1  MINIMAL, QSD_KEEP_BUCKETS            valid when some bucketed group of 0 is flattened
 *   2  QSD_SCHED_TOPK + 1                   valid when r >= 3   (Top-K-sadilla, Sec. 3.6)
 *   3  QSD_SCHED_TOPK + 2                   valid when r >= 4
 *   4  QSD_SCHED_TOPK + 3                   valid when r >= 5
 *   5  LSD                                  valid when r >= 2
 * (K = r - 1 plans exactly what MINIMAL plans, so Top-K stops at K = r - 2.)
 *
 * Features (sampled on the device from the input; plan terms from the host planner):
 *   With N nonzeros and S = min(N, QSD_FEAT_SAMPLE), positions j_k = floor(k N / S),
 *   k = 0..S-1; a pair (j_k, j_k + 1) is counted when j_k + 1 < N.  Coordinates are hashed
 *   with SplitMix64's output function (Steele, Lea and Flood, OOPSLA 2014) applied to the
 *   coordinate as a signed 64-bit integer.
 *   Per mode m: zero_m = zero bits of a 65536-bit map after setting bit (h mod 2^16) of every
 *   sampled coordinate; top_m = the largest of 1024 bucket counts ((h >> 16) mod 1024);
 *   change_m = pairs whose coordinates in m differ.  Mode sets Q0 = the kept prefix of the
 *   minimal plan's first bucketed call, Q1..Q3 = (sigma_1..sigma_K) for K = 1..3 (a set is empty
 *   when it does not exist); change_Q = pairs differing in at least one mode of Q.
 *   Plan terms of a valid candidate, for its groups as the library runs them (8-bit digits,
 *   modes of extent 1 dropped, bucketed groups flattened by the rule of QSD_KEEP_BUCKETS): gp =
 *   digit passes of global groups, sb = key bits of bucketed groups.
 *   Feature i: 0 log2(N)/32; 1 r/8; per slot s = 0..4 (mode sigma_{s+1}, zero past r):
 *   2+4s bits/32, 3+4s log2(1 + D)/24 with the linear-counting estimate
 *   D = -65536 ln(zero/65536) (65536 ln 65536 when zero = 0), 4+4s change/pairs, 5+4s top/S;
 *   22 coordinate bytes/8; 23 value bytes/8; 24+2c gp/16 and 25+2c sb/64 of candidate c (zero
 *   when not valid); 36+q change_Qq/pairs (zero for an empty set).
 *
 * Network: 40 -> 64 -> 64 -> 6, ReLU after both hidden layers, float32.  Output c is the
 * predicted log2 of the run time in ms of candidate c.  Parameters are one float array of
 * QSD_MLP_NPARAM entries: W1 (64 x 40, row-major W1[o][i]), b1 (64), W2 (64 x 64), b2 (64),
 * W3 (6 x 64), b3 (6).  Training minimises the mean over rows and outputs of the squared
 * error, where a target that is not a number (a candidate not valid for that row) contributes
 * zero, with Adam (Kingma and Ba, ICLR 2015).
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

#define QSD_NFEAT 40
#define QSD_NCAND 6
#define QSD_FEAT_SAMPLE 16384
#define QSD_MLP_NPARAM 7174
/* counts per mode (zero, top, change) for r modes, then (change, 0, 0) for the sets Q0..Q3 */
#define QSD_FEAT_COUNTS (3 * (QSD_MAX_ORDER + 4))

/* Schedule and extra plan flags of candidate c (0 <= c < QSD_NCAND). */
qsd_status qsd_candidate(int32_t candidate, qsd_sched_t* sched, uint32_t* flags);
/* The candidates of a request (host only; QSD_NCAND entries each): valid_host[c] = 0 or 1, and
 * the plan terms gp (digit passes of global groups) and sb (key bits of bucketed groups) of the
 * valid ones (0 for the others).  passes_host / bucket_bits_host may be NULL. */
qsd_status qsd_candidate_terms(const qsd_desc* desc, int32_t* valid_host, int32_t* passes_host,
                               int32_t* bucket_bits_host);

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

/* Forward pass over n rows: x_dev (n x 40), h1_dev and h2_dev (n x 64, post-ReLU),
 * y_dev (n x 6).  h1_dev / h2_dev may be NULL when not needed. */
qsd_status qsd_mlp_forward(const float* params_dev, const float* x_dev, int32_t n, float* h1_dev,
                           float* h2_dev, float* y_dev, hipStream_t stream);

/* Device workspace of qsd_mlp_backward for n rows. */
qsd_status qsd_mlp_backward_workspace(int32_t n, size_t* bytes);

/* Loss (mean squared error against t_dev, n x 6; NaN targets contribute zero) and its gradient
 * (QSD_MLP_NPARAM floats) for the activations of a forward pass of the same rows.  loss_dev:
 * one float. */
qsd_status qsd_mlp_backward(const float* params_dev, const float* x_dev, const float* h1_dev,
                            const float* h2_dev, const float* y_dev, const float* t_dev, int32_t n,
                            float* grad_dev, float* loss_dev, void* ws, size_t ws_bytes, hipStream_t stream);

/* One Adam update of every parameter; step counts from 1. */
qsd_status qsd_mlp_adam(float* params_dev, const float* grad_dev, float* m_dev, float* v_dev, int32_t step,
                        float lr, float beta1, float beta2, float eps, hipStream_t stream);

/* Minibatch training: `epochs` passes over the n rows (x_dev n x 40, t_dev n x 6), each in a
 * fresh order drawn by Fisher-Yates from a SplitMix64 stream seeded with `seed` (swap index
 * = next() mod (i + 1), i from n - 1 down to 1), in batches of `batch` rows (the last may be
 * shorter), one Adam step per batch (beta1 0.9, beta2 0.999, eps 1e-8).  Updates params_dev in
 * place; *last_loss receives the loss of the last batch.  Synchronises the stream. */
qsd_status qsd_mlp_train_workspace(int32_t n, int32_t batch, size_t* bytes);
qsd_status qsd_mlp_train(float* params_dev, const float* x_dev, const float* t_dev, int32_t n, int32_t epochs,
                         int32_t batch, float lr, uint64_t seed, void* ws, size_t ws_bytes, hipStream_t stream,
                         float* last_loss);

/* A trained selector.  params_host: QSD_MLP_NPARAM floats (copied to the device).  margin:
 * another candidate is chosen only when its predicted log2 time is below candidate 0's by more
 * than margin (>= 0).  min_nnz: requests with fewer nonzeros take candidate 0 without sampling
 * (the choice cannot pay for itself there).  qsd_model_load reads the file format written by
 * the training tool (little endian): 8 bytes "QSDMLP2\0", int32 nparam, float32 margin,
 * int64 min_nnz, float32 params[nparam]. */
typedef struct qsd_model_s* qsd_model_t;
qsd_status qsd_model_create(const float* params_host, float margin, int64_t min_nnz, qsd_model_t* out);
qsd_status qsd_model_load(const char* path, qsd_model_t* out);
void qsd_model_destroy(qsd_model_t model);

/* Sampling, features, forward pass and the choice, all on the device (two kernel launches,
 * one copy of the result back, one stream synchronisation): candidate 0 unless another valid
 * candidate is predicted faster by more than the margin; candidate 0 too below the model's
 * min_nnz (no device work then) and when a feature is not finite or outside [0, 4].
 * predicted_host (QSD_NCAND floats) may be NULL; it is left untouched when no prediction is
 * made.  Synchronises the stream. */
qsd_status qsd_select(qsd_model_t model, const qsd_desc* desc, const void* const* in_crd, void* ws,
                      size_t ws_bytes, hipStream_t stream, int32_t* candidate, float* predicted_host);

/* qsd_select, then qsd_plan with the chosen candidate's schedule and flags (added to the
 * descriptor's). */
qsd_status qsd_plan_auto(qsd_model_t model, const qsd_desc* desc, const void* const* in_crd, void* ws,
                         size_t ws_bytes, hipStream_t stream, qsd_plan_t* out, int32_t* candidate);

#ifdef __cplusplus
}
#endif
#endif /* QSD_SELECT_H */
