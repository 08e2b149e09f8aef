/*
 * qsd.h -- C ABI of libqsd: sparse-tensor transposition on one AMD Instinct MI355X (gfx950).
 *
 * The operation (Mueller et al., "Sparse Tensor Transpositions", Sec. 2.2): a tensor in
 * coordinate (COO) format is stored as N nonzeros listed in the lexicographic order of a
 * complete mode order `in_order` (the paper's tau, most significant mode first, Sec. 2).
 * Transposing it to `out_order` (sigma) lists the same nonzeros in sigma's lexicographic
 * order.  Nonzeros whose coordinates tie keep their input order (the paper's partial sorts
 * are stable, Sec. 3.1), so the result is unique and reproducible bit for bit.
 *
 * Layout: structure of arrays.  Coordinates are r separate device arrays, one per mode,
 * indexed by the ORIGINAL mode number (crd[m][j] is mode m of nonzero j), of int32 or
 * int64; values are one device array of fp32 or fp64 moved as raw bits (no arithmetic:
 * signed zeros and NaN payloads survive).  Coordinates are 0-based: 0 <= crd[m][j] < n_m.
 *
 * Ownership: the caller owns every device buffer (inputs, outputs, workspace).  The library
 * allocates no device memory in qsd_transpose / qsd_pack_csf / qsd_batch_transpose; it
 * only launches kernels on the caller's stream, without host synchronisation (except when
 * QSD_VALIDATE is set), so these calls may be captured into a HIP graph.
 *
 * Errors: argument errors are returned synchronously before anything is launched.
 * A failed HIP launch returns QSD_ERR_HIP.  Plans and batches are immutable after
 * creation and may be used from several streams if each call has its own workspace.
 */
#ifndef QSD_H
#define QSD_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QSD_MAX_ORDER 8              /* modes per tensor */
#define QSD_MAX_NNZ ((int64_t)1 << 30) /* nnz must be below this */

typedef enum qsd_status {
    QSD_OK = 0,
    QSD_ERR_NULL = 1,          /* a required pointer is NULL */
    QSD_ERR_BAD_ORDER = 2,     /* an order is not a permutation of 0..r-1, or r out of range */
    QSD_ERR_BAD_EXTENT = 3,    /* an extent is < 1 or does not fit the coordinate type */
    QSD_ERR_TOO_LARGE = 4,     /* nnz < 0, nnz >= QSD_MAX_NNZ, or nnz above the planned nnz */
    QSD_ERR_UNSORTED = 5,      /* QSD_VALIDATE: input not sorted under in_order */
    QSD_ERR_COORD_RANGE = 6,   /* QSD_VALIDATE: a coordinate outside [0, n_m) */
    QSD_ERR_WORKSPACE = 7,     /* workspace NULL or smaller than the plan requires */
    QSD_ERR_UNSUPPORTED = 8,   /* combination not supported (e.g. bad type enum) */
    QSD_ERR_HIP = 9,           /* a HIP runtime call or kernel launch failed */
    QSD_ERR_DEVICE = 10        /* a kernel reported an internal failure (see qsd_device_status) */
} qsd_status;

typedef enum qsd_index_t { QSD_I32 = 0, QSD_I64 = 1 } qsd_index_t;
typedef enum qsd_value_t { QSD_F32 = 0, QSD_F64 = 1 } qsd_value_t;

/* Pass schedules; every schedule produces the identical output.
 * MINIMAL: QuesadillaSort (Alg. 3, Sec. 3.5) -- the provably minimal number of partial
 *          sorts, bucketed ones only where necessary (Thm 3.4, Thm 3.5).
 * TOPK + K (1 <= K <= r-1): Top-K-sadilla (Sec. 3.6): MINIMAL towards
 *          (sigma_1..sigma_K, remaining modes in input order), then every bucket of equal
 *          (sigma_1..sigma_K) sorted completely on the rest of sigma.  K = r-1 plans exactly
 *          what MINIMAL plans (the last mode never needs a sort of its own).
 * TOP2:    TOPK with K = min(2, r-2): Top-1 for 3 modes, Top-2 from 4 modes on.
 * LSD:     full least-significant-digit radix sort over all r modes (the paper's "radix").
 * AUTO:    a learned cost model picks among the candidates of qsd_select.h (MINIMAL when no
 *          model is loaded). */
typedef enum qsd_sched_t {
    QSD_SCHED_AUTO = 0,
    QSD_SCHED_MINIMAL = 1,
    QSD_SCHED_TOP2 = 2,
    QSD_SCHED_LSD = 3,
    QSD_SCHED_TOPK = 16         /* QSD_SCHED_TOPK + K selects Top-K-sadilla with that K */
} qsd_sched_t;

#define QSD_VALIDATE 1u   /* qsd_transpose checks ranges and input order first (synchronises) */
/* Bucketed groups (PartialSort calls that keep a prefix, Alg. 2) always run as bucket
 * discovery plus segment-local sorts.  Without this flag, a bucketed group whose nonzeros pack
 * into one 64-bit word is run as one global sort on (prefix, keys) with packed records when
 * that adds at most one digit pass: the same stable result (the input is sorted on the
 * prefix), usually cheaper. */
#define QSD_KEEP_BUCKETS 2u

typedef struct qsd_desc {
    int32_t order;              /* r, 1..QSD_MAX_ORDER */
    int64_t nnz;                /* largest nnz the plan will be used with */
    const int64_t* extents;     /* host, r entries n_m >= 1 */
    qsd_index_t crd_type;
    qsd_value_t val_type;
    const int32_t* in_order;    /* host, r entries, permutation of 0..r-1 (tau) */
    const int32_t* out_order;   /* host, r entries, permutation of 0..r-1 (sigma) */
    uint32_t flags;             /* QSD_VALIDATE | QSD_KEEP_BUCKETS */
} qsd_desc;

typedef struct qsd_plan_s* qsd_plan_t;

/* Build a plan on the host (Alg. 3 and its variants; digit splitting).  All inputs are
 * copied.  *out receives a plan to release with qsd_plan_destroy. */
qsd_status qsd_plan(const qsd_desc* desc, qsd_sched_t sched, qsd_plan_t* out);
void qsd_plan_destroy(qsd_plan_t plan);

/* Bytes of device workspace qsd_transpose needs for this plan (its planned nnz). */
qsd_status qsd_plan_workspace(qsd_plan_t plan, size_t* bytes);

/* Human-readable plan (schedule, PartialSort calls, groups, digit passes) into buf
 * (NUL-terminated, truncated to len).  Format, one item per line:
 *   sched=<MINIMAL|TOP2|LSD> K=<k>
 *   call prefix=<modes comma-separated or empty> mode=<m>      (QuesadillaSort calls)
 *   group prefix=<...> keys=<modes, most significant first> bits=<b> passes=<d>
 */
qsd_status qsd_plan_describe(qsd_plan_t plan, char* buf, size_t len);

/* Transpose (Sec. 2.2: the same nonzeros re-listed in sigma's lexicographic order; carried
 * out as the plan's partial sorts, Alg. 1 and Alg. 2, in the order Alg. 3 gives).
 * in_crd / out_crd: host arrays of r DEVICE pointers (mode order);
 * in_val / out_val: device pointers.  nnz <= planned nnz.  Inputs are read only; outputs
 * must not overlap the inputs or the workspace.  ws: device workspace of ws_bytes >=
 * qsd_plan_workspace.  Asynchronous on `stream`. */
qsd_status qsd_transpose(qsd_plan_t plan, int64_t nnz,
                         const void* const* in_crd, const void* in_val,
                         void* const* out_crd, void* out_val,
                         void* ws, size_t ws_bytes, hipStream_t stream);

/* qsd_transpose without a workspace argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).  The
 * workspace is a fixed array of QSD_NOALLOC_MAX_WORKSPACE bytes in device memory that the
 * library holds on every GPU it runs on until the process ends; the call allocates nothing.
 * Plans whose qsd_plan_workspace exceeds that size are rejected with QSD_ERR_WORKSPACE before
 * anything is launched (for 3-mode int32/fp64 tensors about 1.8M planned nonzeros fit).
 * `stream` must belong to the GPU to run on (NULL: the current device).  All calls on one GPU
 * share its array, which keeps the last call's contents (each call clears what must start at
 * zero): calls that overlap on one GPU race and must not be issued.  The device status bits of
 * these calls cannot be read back (qsd_device_status needs a workspace pointer).  Other
 * arguments, errors and semantics as qsd_transpose. */
#define QSD_NOALLOC_MAX_WORKSPACE ((size_t)64 << 20)
qsd_status qsd_transpose_noalloc(qsd_plan_t plan, int64_t nnz,
                                 const void* const* in_crd, const void* in_val,
                                 void* const* out_crd, void* out_val, hipStream_t stream);

/* Compressed sparse fiber (CSF) pack of a tensor already sorted under the plan's out_order
 * (e.g. qsd_transpose's output): the compressed, level-by-level format of Sec. 1-2, whose
 * level order is the mode order the tensor is sorted in (the reason a transposition is needed
 * before building it).  Levels d = 1..r store mode sigma_d.  Every level is
 * compressed: level d has F_d fibers (maximal runs sharing sigma_1..sigma_d; at d = r
 * every nonzero is its own leaf, F_r = nnz).
 *   crd[d-1]: device array (crd type) with room for nnz entries; receives F_d coordinates.
 *   pos[d-1]: device array (int32 for QSD_I32 plans, int64 for QSD_I64) with room for
 *             nnz + 1 entries (2 for d = 1); receives F_{d-1} + 1 offsets: the children of
 *             level-(d-1) fiber p are level-d fibers pos[d-1][p] .. pos[d-1][p+1]-1.
 *   fiber_counts: device int64[r + 1] receiving F_0 = 1, F_1, ..., F_r.
 * ws: device workspace of qsd_csf_workspace bytes. */
qsd_status qsd_csf_workspace(qsd_plan_t plan, size_t* bytes);
qsd_status qsd_pack_csf(qsd_plan_t plan, int64_t nnz, const void* const* sorted_crd,
                        void* const* pos, void* const* crd, int64_t* fiber_counts,
                        void* ws, size_t ws_bytes, hipStream_t stream);

/* CSF -> CSF transposition (Sec. 5's proposal of transposing the compressed format without a
 * separate conversion step).  Input: a tensor of nnz leaves in the CSF layout above for the
 * plan's in_order (level d stores mode in_order[d-1]; in_pos[d-1] / in_crd[d-1] as pos / crd
 * of qsd_pack_csf, in_val in leaf order), well formed as qsd_pack_csf writes it (reads are
 * bounded by the fiber counts that the arrays themselves give).  Output: the same tensor in
 * the CSF layout for the plan's out_order (out_pos / out_crd / fiber_counts as qsd_pack_csf,
 * out_val in leaf order).  The expansion to coordinates is one scan per level over the
 * leaves (each leaf's ancestor at level d is the number of level-d fibers whose first leaf is
 * at or before it, minus one); the leaf level is used as it is; then the plan's passes and the
 * pack run on the workspace.  ws: device workspace of qsd_csf_transpose_workspace bytes; its
 * device status is read with qsd_device_status(ws).  Asynchronous on `stream` (the pack's
 * empty-input path synchronises, as qsd_pack_csf's). */
qsd_status qsd_csf_transpose_workspace(qsd_plan_t plan, size_t* bytes);
qsd_status qsd_csf_transpose(qsd_plan_t plan, int64_t nnz, const void* const* in_pos,
                             const void* const* in_crd, const void* in_val, void* const* out_pos,
                             void* const* out_crd, void* out_val, int64_t* fiber_counts,
                             void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------------------
 * Batched transposition: many independent tensors (uneven nnz, orders and mode orders) in a
 * handful of kernel launches that can be captured into one HIP graph.  All tensors of a batch
 * share the coordinate and value types.  Each tensor is sorted stably by its flattened key
 * (sigma_1..sigma_q, where sigma_{q+1}..sigma_r is the longest tail already in input order),
 * which yields the same output as every schedule of qsd_plan.  Tensors with at most
 * `small_cap` nonzeros are sorted whole in LDS by one workgroup; the others take global
 * digit passes, launch p running the p-th pass of every tensor that has one.
 *
 * Use: qsd_batch_plan -> qsd_batch_workspace -> qsd_batch_bind (uploads the per-tensor
 * pointer tables into the workspace; synchronises the stream) -> qsd_batch_transpose (kernel
 * launches only: no allocation, no host synchronisation, graph-capturable) any number of
 * times.  Re-bind after changing buffers or tuning.  qsd_batch_tune times candidate settings
 * (items per thread, digit width, small-tensor cutoff) on the bound buffers and keeps the
 * fastest; it overwrites the outputs.
 * --------------------------------------------------------------------------------------- */
typedef struct qsd_batch_s* qsd_batch_t;

typedef struct qsd_batch_io {
    const void* in_crd[QSD_MAX_ORDER];  /* device pointers, mode order */
    const void* in_val;
    void* out_crd[QSD_MAX_ORDER];
    void* out_val;
} qsd_batch_io;

typedef struct qsd_tuning {
    int32_t items;       /* records per thread in a digit pass: 8 or 16 (0 = automatic) */
    int32_t radix_bits;  /* digit width of a pass: 4..8 */
    int32_t small_cap;   /* tensors with nnz <= small_cap are sorted in LDS: 0..4096 */
} qsd_tuning;

/* descs: count descriptors (flags ignored).  Returns QSD_ERR_UNSUPPORTED for mixed types, a
 * flattened key wider than 128 bits, or more than 16 digit passes for one tensor. */
qsd_status qsd_batch_plan(const qsd_desc* descs, int32_t count, qsd_batch_t* out);
void qsd_batch_destroy(qsd_batch_t batch);
qsd_status qsd_batch_set_tuning(qsd_batch_t batch, const qsd_tuning* tuning);
qsd_status qsd_batch_get_tuning(qsd_batch_t batch, qsd_tuning* tuning);
qsd_status qsd_batch_workspace(qsd_batch_t batch, size_t* bytes);
/* io: host array of `count` entries (device pointers).  Copies the tables into ws. */
qsd_status qsd_batch_bind(qsd_batch_t batch, const qsd_batch_io* io, void* ws, size_t ws_bytes,
                          hipStream_t stream);
qsd_status qsd_batch_transpose(qsd_batch_t batch, void* ws, size_t ws_bytes, hipStream_t stream);
/* Autotuner: tries items {8, 16} x radix bits {6, 7, 8} x small_cap {0, 1024, 4096}, `reps`
 * timed runs each (best of), on the bound buffers; applies and returns the fastest setting and
 * its time.  qsd_batch_workspace_max: bytes enough for every tuning qsd_batch_set_tuning
 * accepts (hence for every candidate of the autotuner). */
qsd_status qsd_batch_workspace_max(qsd_batch_t batch, size_t* bytes);
qsd_status qsd_batch_tune(qsd_batch_t batch, const qsd_batch_io* io, void* ws, size_t ws_bytes,
                          hipStream_t stream, int32_t reps, qsd_tuning* best, float* best_ms);

/* Autotune cache.  The key of a batch names the device architecture, the coordinate and value
 * widths, the largest order and the size class (floor(log2(total nonzeros + 1)) and
 * floor(log2(tensors))), e.g. "gfx950/c4/v8/r4/n29/t12"; key_bytes >= 64 is enough.
 * qsd_batch_tune_cached looks the key up in the text file at cache_path (one entry per line:
 * key items radix_bits small_cap ms); on a hit it applies and binds that tuning without timing
 * (*from_cache = 1, *best_ms = the recorded time; the first matching line is used), otherwise it
 * runs qsd_batch_tune and appends the result (*from_cache = 0).  A missing file is a miss, lines
 * that do not parse are skipped, an entry that qsd_batch_set_tuning rejects or whose workspace
 * exceeds ws_bytes is tuned afresh, and a file that cannot be written leaves the result uncached
 * (not an error).  Concurrent writers to one file are not coordinated. */
qsd_status qsd_batch_tune_key(qsd_batch_t batch, char* key, size_t key_bytes);
qsd_status qsd_batch_tune_cached(qsd_batch_t batch, const qsd_batch_io* io, void* ws, size_t ws_bytes,
                                 hipStream_t stream, int32_t reps, const char* cache_path, qsd_tuning* best,
                                 float* best_ms, int32_t* from_cache);

/* HIP graph of qsd_batch_transpose on the bound workspace: captured on an internal stream and
 * instantiated; launch it on any stream.  The graph holds the buffer addresses bound now. */
typedef struct qsd_graph_s* qsd_graph_t;
qsd_status qsd_batch_graph(qsd_batch_t batch, void* ws, size_t ws_bytes, qsd_graph_t* out);
qsd_status qsd_graph_launch(qsd_graph_t graph, hipStream_t stream);
void qsd_graph_destroy(qsd_graph_t graph);

/* Device-side status of every call that used this workspace since the previous
 * qsd_device_status on it (or since its first use): 0 when every kernel ran normally,
 * otherwise the OR of the bits the kernels set (1: a bounded wait in a scan timed out, and the
 * output of that call is not valid).  Synchronises `stream`, reads 4 bytes and clears them.
 * Validation results are returned by qsd_transpose itself. */
qsd_status qsd_device_status(void* ws, hipStream_t stream, uint32_t* code);

const char* qsd_status_str(qsd_status s);

/* Kernel timing.  Between qsd_profile_start and qsd_profile_stop every kernel the library
 * launches (from any thread, on any stream) is bracketed by two hipEvents recorded on the
 * stream it is launched on.  qsd_profile_stop synchronises those events and returns one
 * entry per kernel kind: launches, summed event durations, and the algorithmic bytes the
 * launches had to move (the data-movement model of the kind; 0 where none is modelled).
 * Kinds: zero, copy, validate, hist, digit, boundary, classify, small, hist_seg,
 * digit_seg, csf, hist_batch, small_batch, digit_batch.  Launches made while the stream is
 * being captured into a graph are not recorded.  Recording adds two event records per launch; it is off by default. */
typedef struct qsd_kernel_stat {
    char name[24];
    int64_t launches;
    double total_ms;
    double bytes;
} qsd_kernel_stat;
qsd_status qsd_profile_start(void);
qsd_status qsd_profile_stop(qsd_kernel_stat* out, int32_t max, int32_t* count);

#ifdef __cplusplus
}
#endif
#endif /* QSD_H */
