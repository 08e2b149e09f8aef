// C ABI of libqsd: argument checks, workspace layout, and the launch sequence of a plan.
#include "../../include/qsd.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "csf_kernels.h"
#include "kernels.h"
#include "plan.h"

using namespace qsd;

namespace {

constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }
uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

struct Layout {
    size_t ctl = 0;
    size_t rec_crd[kMaxR] = {};
    size_t rec_val = 0;
    size_t hist = 0;          // global-group histograms, one block per sub-key
    size_t hist_words = 0;
    size_t status[2] = {};
    size_t status_words = 0;  // per array
    size_t seg_start = 0, region_seg = 0, bstatus = 0, bstatus_words = 0, geo = 0, large = 0, seg_hist = 0;
    size_t tile_map = 0;
    size_t pk[2] = {};        // packed-record ping-pong buffers (64-bit words)
    size_t seg_bits = 0;      // segment starts as one bit per record (bucket reuse)
    uint32_t max_large = 0, max_med = 0, max_tiles_large = 0;
    size_t total = 0;
};

struct HopPlan {
    int total = 0;
};

}  // namespace

struct qsd_plan_s {
    PlanData p;
    Layout L;
    std::vector<char> reuse;           // per group: derives its segment starts from the previous group's
    int tile = 0;
    int items = 16;
    bool pack = true;                  // pack records inside global groups when they fit
    std::vector<size_t> sub_hist_off;  // word offset of each global sub-key's histograms
    int nseg_groups = 0;
};

namespace {

// A global group of two or more digit passes moves packed records when every coordinate of a
// nonzero fits in one 64-bit word: the first pass packs, the last unpacks (Sec. 5's bit
// packing).  The group's composite key occupies the low bits of the word.
bool packable_key(const qsd_plan_s* q, const Group& g) {
    if (!q->pack || g.subs.size() != 1 || g.subs[0].passes.size() < 2) return false;
    int total = 0;
    for (int m = 0; m < q->p.r; ++m) total += q->p.bits[m];
    if (total > 64) return false;
    const KeySpec& k = g.subs[0].key;
    for (int m = 0; m < q->p.r; ++m)
        if (k.width[m] && (k.src_lo[m] != 0 || k.width[m] != q->p.bits[m])) return false;
    return true;
}
bool packable(const qsd_plan_s* q, const Group& g) { return !g.segmented && packable_key(q, g); }
// The large segments of a segmented group take the same packed passes (kernels for 16 records
// per thread only); the LDS segment sorts move the records as they are.
bool packable_seg(const qsd_plan_s* q, const Group& g) { return g.segmented && q->items == 16 && packable_key(q, g); }

// Word layout of packed records: key modes at their place in the composite key (low bits),
// the other modes above it.
void pack_layout(int r, const int* bits, const KeySpec& k, int32_t* pos, uint64_t* mask) {
    int at = k.bits;
    for (int m = 0; m < r; ++m) {
        const int b = bits[m];
        mask[m] = b ? ((b >= 64) ? ~0ull : ((1ull << b) - 1)) : 0;
        if (k.width[m]) {
            pos[m] = k.dst[m];
        } else {
            pos[m] = b ? at : 0;
            at += b;
        }
    }
}

void pack_spec(const PlanData& p, const KeySpec& k, DigitArgs& da) { pack_layout(p.r, p.bits, k, da.pk_pos, da.pk_mask); }

void make_layout(qsd_plan_s* q) {
    const PlanData& p = q->p;
    Layout& L = q->L;
    const uint64_t N = (uint64_t)std::max<int64_t>(p.nnz, 1);
    q->items = digit_items(p.r, p.crd_bytes, p.val_bytes);
    q->tile = kBlock * q->items;
    const uint64_t T = (uint64_t)q->tile;
    size_t at = 0;
    L.ctl = at;
    at = up(at + kCtlWords * 4);
    for (int m = 0; m < p.r; ++m) {
        L.rec_crd[m] = at;
        at = up(at + N * p.crd_bytes);
    }
    L.rec_val = at;
    at = up(at + N * p.val_bytes);
    // histograms of global groups
    q->sub_hist_off.clear();
    size_t hw = 0;
    int max_seg_passes = 0;
    bool any_seg = false;
    for (const auto& g : p.groups) {
        if (g.segmented) {
            any_seg = true;
            for (const auto& s : g.subs) max_seg_passes = std::max(max_seg_passes, (int)s.passes.size());
            continue;
        }
        for (const auto& s : g.subs) {
            q->sub_hist_off.push_back(hw);
            hw += s.passes.size() * kBins;
        }
    }
    q->nseg_groups = 0;
    for (const auto& g : p.groups) q->nseg_groups += g.segmented ? 1 : 0;
    L.hist = at;
    L.hist_words = hw;
    at = up(at + hw * 4);
    // look-back status (two arrays used alternately)
    uint64_t tiles = cdiv(N, T);
    L.max_large = (uint32_t)(N / (kSmallCap + 1) + 1);
    L.max_med = (uint32_t)(N / (kTinyLen + 1) + 1);
    L.max_tiles_large = (uint32_t)(tiles + L.max_large);
    if (any_seg) tiles = std::max<uint64_t>(tiles, L.max_tiles_large);
    L.status_words = tiles * kBins;
    for (int i = 0; i < 2; ++i) {
        L.status[i] = at;
        at = up(at + L.status_words * 4);
    }
    if (any_seg) {
        L.seg_start = at;
        at = up(at + (N + 2) * 4);
        L.region_seg = at;
        at = up(at + (cdiv(N, kRegion) + 2) * 4);
        L.tile_map = at;
        at = up(at + (size_t)L.max_tiles_large * 16);
        L.large = at;
        at = up(at + (size_t)L.max_large * 16);
        L.bstatus_words = cdiv(N, kDiscTile);
        L.bstatus = at;
        at = up(at + L.bstatus_words * 4 * q->nseg_groups);
        L.geo = at;
        at = up(at + (cdiv(N, kRegion) + L.max_med) * 16);
        L.seg_hist = at;
        at = up(at + (size_t)L.max_large * max_seg_passes * kBins * 4);
    }
    // bucket reuse (Sec. 5): a segmented group right after a segmented group whose kept prefix
    // its own extends finds its segment starts from the previous ones plus the added modes
    q->reuse.assign(p.groups.size(), 0);
    bool any_reuse = false;
    for (size_t i = 1; i < p.groups.size(); ++i) {
        const Group &a = p.groups[i - 1], &b = p.groups[i];
        if (a.segmented && b.segmented && a.prefix.size() < b.prefix.size() &&
            std::equal(a.prefix.begin(), a.prefix.end(), b.prefix.begin())) {
            q->reuse[i] = 1;
            any_reuse = true;
        }
    }
    if (any_reuse) {
        L.seg_bits = at;
        at = up(at + cdiv(N, 64) * 8);
    }
    bool any_pack = false;
    for (const auto& g : p.groups) any_pack |= packable(q, g) || packable_seg(q, g);
    if (any_pack)
        for (int i = 0; i < 2; ++i) {
            L.pk[i] = at;
            at = up(at + N * 8);
        }
    L.total = at;
}

// Histogram workgroups per CU (loads in flight).  Measured per CU: one key of 2 modes over 1e8
// records: 4 -> 385 us, 8 -> 341, 12 -> 326, 16 -> 319; 4096 tensors, 608M records: 4 -> 3.69 ms,
// 8 -> 3.13, 12 -> 2.97, 16 -> 2.85.
int hist_blocks_per_cu() { return 16; }

bool is_perm(const int32_t* o, int r) {
    bool seen[kMaxR] = {};
    for (int i = 0; i < r; ++i) {
        if (o[i] < 0 || o[i] >= r || seen[o[i]]) return false;
        seen[o[i]] = true;
    }
    return true;
}

qsd_status check_desc(const qsd_desc* d) {
    if (!d || !d->extents || !d->in_order || !d->out_order) return QSD_ERR_NULL;
    if (d->order < 1 || d->order > QSD_MAX_ORDER) return QSD_ERR_BAD_ORDER;
    if (!is_perm(d->in_order, d->order) || !is_perm(d->out_order, d->order)) return QSD_ERR_BAD_ORDER;
    if (d->crd_type != QSD_I32 && d->crd_type != QSD_I64) return QSD_ERR_UNSUPPORTED;
    if (d->val_type != QSD_F32 && d->val_type != QSD_F64) return QSD_ERR_UNSUPPORTED;
    const int64_t lim = d->crd_type == QSD_I32 ? (int64_t)1 << 31 : INT64_MAX;
    for (int m = 0; m < d->order; ++m)
        if (d->extents[m] < 1 || d->extents[m] > lim) return QSD_ERR_BAD_EXTENT;
    if (d->nnz < 0 || d->nnz >= QSD_MAX_NNZ) return QSD_ERR_TOO_LARGE;
    return QSD_OK;
}

}  // namespace

static_assert(QSD_KEEP_BUCKETS == kKeepBuckets, "plan flag values differ");

// Argument check shared with the selector's entry points.
namespace qsd {
qsd_status desc_status(const qsd_desc* d) { return check_desc(d); }
}  // namespace qsd

namespace {

struct Bufs {
    const void* crd[kMaxR];
    const void* val;
};

// ---- launch timing (qsd_profile_*)
enum Kind { kZero, kCopy, kValidate, kHist, kDigit, kBoundary, kClassify, kSmall, kHistSeg, kDigitSeg, kCsf,
            kHistBatch, kSmallBatch, kDigitBatch, kCsfExpand, kNumKinds };
const char* kKindName[kNumKinds] = {"zero", "copy", "validate", "hist", "digit", "boundary",
                                    "classify", "small", "hist_seg", "digit_seg", "csf",
                                    "hist_batch", "small_batch", "digit_batch", "csf_expand"};
struct ProfRec {
    int kind;
    hipEvent_t a, b;
    double bytes;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_pool;

hipEvent_t pool_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

template <typename F>
hipError_t timed(int kind, double bytes, hipStream_t s, F&& fn) {
    if (!g_prof_on) return fn();
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return fn();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    ProfRec r{kind, pool_event(), pool_event(), bytes};
    const bool ra = r.a && hipEventRecord(r.a, s) == hipSuccess;
    const hipError_t e = fn();
    const bool rb = r.b && hipEventRecord(r.b, s) == hipSuccess;
    if (ra && rb) {
        g_prof.push_back(r);
    } else {  // a launch whose events did not record is left out of the profile
        if (r.a) (void)hipEventDestroy(r.a);
        if (r.b) (void)hipEventDestroy(r.b);
    }
    return e;
}

}  // namespace

extern "C" {

const char* qsd_status_str(qsd_status s) {
    switch (s) {
        case QSD_OK: return "ok";
        case QSD_ERR_NULL: return "null pointer";
        case QSD_ERR_BAD_ORDER: return "bad mode order";
        case QSD_ERR_BAD_EXTENT: return "bad extent";
        case QSD_ERR_TOO_LARGE: return "nnz too large";
        case QSD_ERR_UNSORTED: return "input not sorted under in_order";
        case QSD_ERR_COORD_RANGE: return "coordinate out of range";
        case QSD_ERR_WORKSPACE: return "workspace missing or too small";
        case QSD_ERR_UNSUPPORTED: return "unsupported";
        case QSD_ERR_HIP: return "HIP error";
        case QSD_ERR_DEVICE: return "device-side failure";
    }
    return "unknown status";
}

qsd_status qsd_plan(const qsd_desc* desc, qsd_sched_t sched, qsd_plan_t* out) {
    if (!out) return QSD_ERR_NULL;
    *out = nullptr;
    const qsd_status st = check_desc(desc);
    if (st != QSD_OK) return st;
    const int si = (int)sched;
    if (!((si >= QSD_SCHED_AUTO && si <= QSD_SCHED_LSD) || (si > QSD_SCHED_TOPK && si < QSD_SCHED_TOPK + desc->order)))
        return QSD_ERR_UNSUPPORTED;
    auto* q = new qsd_plan_s();
    PlanData& p = q->p;
    p.r = desc->order;
    p.nnz = desc->nnz;
    p.crd_bytes = desc->crd_type == QSD_I64 ? 8 : 4;
    p.val_bytes = desc->val_type == QSD_F64 ? 8 : 4;
    p.flags = desc->flags;
    for (int m = 0; m < p.r; ++m) {
        p.ext[m] = desc->extents[m];
        p.bits[m] = bits_for_extent(desc->extents[m]);
        p.in_order[m] = desc->in_order[m];
        p.out_order[m] = desc->out_order[m];
    }
    if (!build_plan(p, (int)sched)) {
        delete q;
        return QSD_ERR_UNSUPPORTED;
    }
    int passes = 0;
    for (const auto& g : p.groups)
        for (const auto& s : g.subs) passes += (int)s.passes.size();
    // tile counters of every pass in the control block (its last 8 words serve the CSF expansion)
    if (passes * kPassCounters > kCtlWords - kCtlPassCnt - 8) {
        delete q;
        return QSD_ERR_UNSUPPORTED;
    }
    make_layout(q);
    *out = q;
    return QSD_OK;
}

void qsd_plan_destroy(qsd_plan_t plan) { delete plan; }

qsd_status qsd_plan_workspace(qsd_plan_t plan, size_t* bytes) {
    if (!plan || !bytes) return QSD_ERR_NULL;
    *bytes = plan->L.total;
    return QSD_OK;
}

qsd_status qsd_plan_describe(qsd_plan_t plan, char* buf, size_t len) {
    if (!plan || !buf) return QSD_ERR_NULL;
    std::string s = describe(plan->p);
    const Layout& L = plan->L;
    s += "layout tile=" + std::to_string(plan->tile) + " ctl=" + std::to_string(L.ctl) +
         " status0=" + std::to_string(L.status[0]) + " status1=" + std::to_string(L.status[1]) +
         " seg_start=" + std::to_string(L.seg_start) + " region_seg=" + std::to_string(L.region_seg) +
         " tile_map=" + std::to_string(L.tile_map) + " geo=" + std::to_string(L.geo) +
         " seg_hist=" + std::to_string(L.seg_hist) +
         " seg_bits=" + std::to_string(L.seg_bits) + " reuse=" + std::to_string(std::count(plan->reuse.begin(), plan->reuse.end(), 1)) +
         " total=" + std::to_string(L.total) + "\n";
    if (len == 0) return QSD_OK;
    const size_t n = std::min(len - 1, s.size());
    std::memcpy(buf, s.data(), n);
    buf[n] = 0;
    return QSD_OK;
}

qsd_status qsd_transpose(qsd_plan_t plan, int64_t nnz, const void* const* in_crd, const void* in_val,
                         void* const* out_crd, void* out_val, void* ws, size_t ws_bytes,
                         hipStream_t stream) {
    if (!plan || !in_crd || !out_crd) return QSD_ERR_NULL;
    const PlanData& p = plan->p;
    const Layout& L = plan->L;
    if (nnz < 0 || nnz > p.nnz) return QSD_ERR_TOO_LARGE;
    if (nnz == 0) return QSD_OK;
    if (!in_val || !out_val) return QSD_ERR_NULL;
    for (int m = 0; m < p.r; ++m)
        if (!in_crd[m] || !out_crd[m]) return QSD_ERR_NULL;
    if (!ws || ws_bytes < L.total) return QSD_ERR_WORKSPACE;

    const uint32_t n = (uint32_t)nnz;
    const uint32_t T = (uint32_t)plan->tile;
    char* W = (char*)ws;
    uint32_t* ctl = (uint32_t*)(W + L.ctl);
    uint32_t* S[2] = {(uint32_t*)(W + L.status[0]), (uint32_t*)(W + L.status[1])};
    hipError_t e;
#define QSD_CK(x)                              \
    do {                                       \
        if ((e = (x)) != hipSuccess) return QSD_ERR_HIP; \
    } while (0)

    {
        ZeroArgs z{};
        z.ctl = ctl;
        if (L.hist_words) {
            z.ptr[1] = (uint32_t*)(W + L.hist);
            z.words[1] = L.hist_words;
        }
        if (L.bstatus_words) {
            z.ptr[2] = (uint32_t*)(W + L.bstatus);
            z.words[2] = L.bstatus_words * plan->nseg_groups;
        }
        QSD_CK(timed(kZero, 0, stream, [&] { return launch_zero(z, stream); }));
    }
    if (p.flags & QSD_VALIDATE) {
        ValidateArgs va{};
        for (int m = 0; m < p.r; ++m) {
            va.crd[m] = in_crd[m];
            va.ext[m] = p.ext[m];
            va.in_order[m] = p.in_order[m];
        }
        va.r = p.r;
        va.n = n;
        va.flags = ctl + kCtlValid;
        QSD_CK(timed(kValidate, 0, stream, [&] { return launch_validate(va, p.crd_bytes, stream); }));
        uint32_t flags = 0;
        QSD_CK(hipMemcpyAsync(&flags, ctl + kCtlValid, 4, hipMemcpyDeviceToHost, stream));
        QSD_CK(hipStreamSynchronize(stream));
        if (flags & 1u) return QSD_ERR_COORD_RANGE;
        if (flags & 2u) return QSD_ERR_UNSORTED;
    }

    // buffer hops: every digit pass moves all records from one buffer to another; the last
    // lands in the output.  Hop h writes OUT when (H - 1 - h) is even, else the workspace.
    int H = 0;
    for (const auto& g : p.groups)
        for (const auto& s : g.subs) H += (int)s.passes.size();
    Bufs in{}, outb{}, wsb{};
    for (int m = 0; m < p.r; ++m) {
        in.crd[m] = in_crd[m];
        outb.crd[m] = out_crd[m];
        wsb.crd[m] = W + L.rec_crd[m];
    }
    in.val = in_val;
    outb.val = out_val;
    wsb.val = W + L.rec_val;
    if (H == 0) {
        for (int m = 0; m < p.r; ++m)
            QSD_CK(timed(kCopy, 2.0 * n * p.crd_bytes, stream,
                         [&] { return launch_copy(in_crd[m], out_crd[m], (uint64_t)n * p.crd_bytes, stream); }));
        QSD_CK(timed(kCopy, 2.0 * n * p.val_bytes, stream,
                     [&] { return launch_copy(in_val, out_val, (uint64_t)n * p.val_bytes, stream); }));
        return QSD_OK;
    }
    auto hop_dst = [&](int h) -> Bufs { return ((H - 1 - h) % 2 == 0) ? outb : wsb; };

    Bufs cur = in;
    int h = 0, q = 0, gsub = 0, gseg = 0, gi = -1;
    for (const auto& g : p.groups) {
        ++gi;
        if (!g.segmented) {
            for (const auto& sk : g.subs) {
                const int np = (int)sk.passes.size();
                DevKey key{};
                for (int m = 0; m < p.r; ++m) {
                    key.mask[m] = sk.key.width[m] ? ((sk.key.width[m] >= 64) ? ~0ull : ((1ull << sk.key.width[m]) - 1)) : 0;
                    key.src_lo[m] = sk.key.src_lo[m];
                    key.dst[m] = sk.key.dst[m];
                }
                uint32_t* hist = (uint32_t*)(W + L.hist) + plan->sub_hist_off[gsub++];
                const uint32_t ntiles = (n + T - 1) / T;
                HistArgs ha{};
                for (int m = 0; m < p.r; ++m) ha.crd[m] = cur.crd[m];
                ha.key = key;
                ha.npass = np;
                for (int i = 0; i < np; ++i) {
                    ha.lo[i] = sk.passes[i].lo;
                    ha.bits[i] = sk.passes[i].bits;
                }
                ha.n = n;
                ha.seg_mode = 0;
                ha.hist = hist;
                ha.status_zero = S[q % 2];
                ha.status_words = (uint64_t)ntiles * kBins;
                const int hgrid = (int)std::max<uint64_t>(
                    1, std::min<uint64_t>(cdiv(n, kBlock * 16), (uint64_t)device_cu_count() * hist_blocks_per_cu()));
                int kmodes = 0;
                for (int m = 0; m < p.r; ++m) kmodes += key.mask[m] ? 1 : 0;
                QSD_CK(timed(kHist, (double)n * p.crd_bytes * kmodes, stream,
                             [&] { return launch_hist(ha, p.r, p.crd_bytes, hgrid, stream); }));
                const bool pk = packable(plan, g);
                const double rec = p.r * p.crd_bytes + p.val_bytes, prec = 8.0 + p.val_bytes;
                void* P[2] = {W + L.pk[0], W + L.pk[1]};
                for (int i = 0; i < np; ++i) {
                    const Bufs dst = hop_dst(h);
                    DigitArgs da{};
                    int r_launch = p.r, cb_launch = p.crd_bytes;
                    double bytes = 2.0 * n * rec;
                    for (int m = 0; m < p.r; ++m) {
                        da.src_crd[m] = cur.crd[m];
                        da.dst_crd[m] = const_cast<void*>(dst.crd[m]);
                    }
                    da.key = key;
                    if (pk) {
                        pack_spec(p, sk.key, da);
                        if (i == 0) {  // coordinate arrays in, packed words out
                            da.pk = 1;
                            da.dst_crd[0] = P[0];
                            bytes = n * (rec + prec);
                        } else if (i + 1 < np) {  // packed words in and out: one 64-bit "mode"
                            da = DigitArgs{};
                            da.src_crd[0] = P[(i - 1) % 2];
                            da.dst_crd[0] = P[i % 2];
                            da.key.mask[0] = sk.key.bits >= 64 ? ~0ull : ((1ull << sk.key.bits) - 1);
                            r_launch = 1;
                            cb_launch = 8;
                            bytes = 2.0 * n * prec;
                        } else {  // packed words in, coordinate arrays out
                            da.pk = 2;
                            da.src_crd[0] = P[(i - 1) % 2];
                            bytes = n * (rec + prec);
                        }
                    }
                    da.src_val = cur.val;
                    da.dst_val = const_cast<void*>(dst.val);
                    da.lo = sk.passes[i].lo;
                    da.bits = sk.passes[i].bits;
                    da.n = n;
                    da.ntiles = ntiles;
                    da.seg_mode = 0;
                    da.hist = hist + (size_t)i * kBins;
                    da.status = S[q % 2];
                    da.status_next = (i + 1 < np) ? S[(q + 1) % 2] : nullptr;
                    da.tile_counter = ctl + kCtlPassCnt + kPassCounters * q;
                    da.err = ctl + kCtlErr;
                    QSD_CK(timed(kDigit, bytes, stream, [&] {
                        return launch_digit(da, r_launch, cb_launch, p.val_bytes, plan->items, stream);
                    }));
                    cur = dst;
                    ++h;
                    ++q;
                }
            }
            continue;
        }
        // ---- segmented group: buckets of equal prefix, sorted each on its own
        const int np = (int)g.subs[0].passes.size();
        const Bufs gsrc = cur;
        const Bufs gdst = hop_dst(h + np - 1);
        uint32_t* seg_start = (uint32_t*)(W + L.seg_start);
        uint32_t* region_seg = (uint32_t*)(W + L.region_seg);
        uint4* tile_geo = (uint4*)(W + L.tile_map);
        uint32_t* bstatus = (uint32_t*)(W + L.bstatus) + (size_t)gseg * L.bstatus_words;
        uint4* geo = (uint4*)(W + L.geo);
        uint32_t* seg_hist = (uint32_t*)(W + L.seg_hist);
        uint64_t* large_ctl = (uint64_t*)(ctl + kCtlLarge);
        if (gseg > 0) {  // counters of the previous segmented group
            ZeroArgs z{};
            z.ptr[0] = ctl + kCtlNb;
            z.words[0] = 6;  // nb, nmed, large (2 words), pad, pad
            z.ptr[1] = ctl + kCtlBoundCnt;
            z.words[1] = 1;
            QSD_CK(timed(kZero, 0, stream, [&] { return launch_zero(z, stream); }));
        }
        DevKey key{};
        {
            const KeySpec& ks = g.subs[0].key;
            for (int m = 0; m < p.r; ++m) {
                key.mask[m] = ks.width[m] ? ((1ull << ks.width[m]) - 1) : 0;
                key.src_lo[m] = ks.src_lo[m];
                key.dst[m] = ks.dst[m];
            }
        }
        BoundArgs ba{};
        for (int m = 0; m < p.r; ++m) ba.crd[m] = gsrc.crd[m];
        ba.nprefix = (int)g.prefix.size();
        for (int i = 0; i < ba.nprefix; ++i) ba.prefix[i] = g.prefix[i];
        uint64_t* seg_bits = (uint64_t*)(W + L.seg_bits);
        if (plan->reuse[gi]) {
            ba.prev_bits = seg_bits;
            ba.nskip = (int)p.groups[gi - 1].prefix.size();
        }
        if ((size_t)gi + 1 < p.groups.size() && plan->reuse[gi + 1]) ba.bits_out = seg_bits;
        ba.n = n;
        ba.seg_start = seg_start;
        ba.region_seg = region_seg;
        ba.status = bstatus;
        ba.tile_counter = ctl + kCtlBoundCnt;
        ba.nb_out = ctl + kCtlNb;
        ba.err = ctl + kCtlErr;
        QSD_CK(timed(kBoundary, 0, stream, [&] { return launch_boundary(ba, p.crd_bytes, stream); }));

        ClassArgs ca{};
        ca.seg_start = seg_start;
        ca.nb = ctl + kCtlNb;
        ca.tile = T;
        ca.nmed = ctl + kCtlNMed;
        ca.geo = geo;
        ca.region_seg = region_seg;
        ca.nregions = (n + kRegion - 1) / kRegion;
        ca.large_ctl = large_ctl;
        ca.tile_geo = tile_geo;
        ca.large = (uint4*)(W + L.large);
        ca.seg_hist = seg_hist;
        ca.hist_stride = (uint32_t)np * kBins;
        QSD_CK(timed(kClassify, 0, stream, [&] { return launch_classify(ca, n, stream); }));
        QSD_CK(timed(kClassify, 0, stream, [&] {
            return launch_tile_geo(ca, (uint32_t)std::min<uint64_t>(L.max_tiles_large, (uint64_t)(n + T - 1) / T + n / (kSmallCap + 1) + 1), stream);
        }));

        SmallArgs sa{};
        for (int m = 0; m < p.r; ++m) {
            sa.src_crd[m] = gsrc.crd[m];
            sa.dst_crd[m] = const_cast<void*>(gdst.crd[m]);
        }
        sa.src_val = gsrc.val;
        sa.dst_val = const_cast<void*>(gdst.val);
        sa.r = p.r;
        sa.key = key;
        sa.key_bits = g.key_bits;
        sa.n = n;
        sa.nregions = (n + kRegion - 1) / kRegion;
        sa.seg_start = seg_start;
        sa.nmed = ctl + kCtlNMed;
        sa.geo = geo;
        const uint32_t small_items = sa.nregions + (uint32_t)std::min<uint64_t>(L.max_med, n / (kTinyLen + 1) + 1);
        QSD_CK(timed(kSmall, 0, stream, [&] { return launch_small(sa, p.crd_bytes, p.val_bytes, small_items, stream); }));

        const SubKey& sk = g.subs[0];
        HistArgs ha{};
        for (int m = 0; m < p.r; ++m) ha.crd[m] = gsrc.crd[m];
        ha.key = key;
        ha.npass = np;
        for (int i = 0; i < np; ++i) {
            ha.lo[i] = sk.passes[i].lo;
            ha.bits[i] = sk.passes[i].bits;
        }
        ha.seg_mode = 1;
        ha.tile = T;
        ha.hist = seg_hist;
        ha.hist_stride = (uint32_t)np * kBins;
        ha.status_zero = S[q % 2];
        ha.large_ctl = large_ctl;
        ha.tile_geo = tile_geo;
        QSD_CK(timed(kHistSeg, 0, stream, [&] {
            return launch_hist(ha, p.r, p.crd_bytes, device_cu_count() * hist_blocks_per_cu(), stream);
        }));
        // every pass's digit offsets per large segment, read directly by the segment passes
        QSD_CK(timed(kHistSeg, 0, stream, [&] {
            return launch_hist_prefix_seg(seg_hist, large_ctl, (uint32_t)np, L.max_large * (uint32_t)np, stream);
        }));
        const uint32_t max_tiles = (uint32_t)std::min<uint64_t>(L.max_tiles_large, (uint64_t)(n + T - 1) / T + n / (kSmallCap + 1) + 1);
        const bool spk = packable_seg(plan, g);
        void* P[2] = {W + L.pk[0], W + L.pk[1]};
        for (int i = 0; i < np; ++i) {
            const Bufs dst = hop_dst(h);
            DigitArgs da{};
            int r_launch = p.r, cb_launch = p.crd_bytes;
            for (int m = 0; m < p.r; ++m) {
                da.src_crd[m] = cur.crd[m];
                da.dst_crd[m] = const_cast<void*>(dst.crd[m]);
            }
            da.key = key;
            if (spk) {  // as in a global group: the first pass packs, the last unpacks
                pack_spec(p, sk.key, da);
                if (i == 0) {
                    da.pk = 1;
                    da.dst_crd[0] = P[0];
                } else if (i + 1 < np) {  // packed words in and out: one 64-bit "mode"
                    da = DigitArgs{};
                    da.src_crd[0] = P[(i - 1) % 2];
                    da.dst_crd[0] = P[i % 2];
                    da.key.mask[0] = sk.key.bits >= 64 ? ~0ull : ((1ull << sk.key.bits) - 1);
                    r_launch = 1;
                    cb_launch = 8;
                } else {
                    da.pk = 2;
                    da.src_crd[0] = P[(i - 1) % 2];
                }
            }
            da.src_val = cur.val;
            da.dst_val = const_cast<void*>(dst.val);
            da.lo = sk.passes[i].lo;
            da.bits = sk.passes[i].bits;
            da.n = n;
            da.ntiles = max_tiles;
            da.seg_mode = 1;
            da.hist_stride = (uint32_t)np * kBins;
            da.hist = seg_hist + (size_t)i * kBins;
            da.status = S[q % 2];
            da.status_next = (i + 1 < np) ? S[(q + 1) % 2] : nullptr;
            da.tile_counter = ctl + kCtlPassCnt + kPassCounters * q;
            da.large_ctl = large_ctl;
            da.tile_map = reinterpret_cast<const uint32_t*>(tile_geo);
            da.err = ctl + kCtlErr;
            QSD_CK(timed(kDigitSeg, 0, stream, [&] { return launch_digit(da, r_launch, cb_launch, p.val_bytes, plan->items, stream); }));
            cur = dst;
            ++h;
            ++q;
        }
        cur = gdst;
        ++gseg;
    }
#undef QSD_CK
    return QSD_OK;
}

qsd_status qsd_profile_start(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& r : g_prof) {
        if (r.a) g_pool.push_back(r.a);
        if (r.b) g_pool.push_back(r.b);
    }
    g_prof.clear();
    g_prof_on = true;
    return QSD_OK;
}

qsd_status qsd_profile_stop(qsd_kernel_stat* out, int32_t max, int32_t* count) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = false;
    qsd_kernel_stat agg[kNumKinds];
    std::memset(agg, 0, sizeof(agg));
    qsd_status st = QSD_OK;
    for (auto& r : g_prof) {
        float ms = 0.f;
        if (!r.a || !r.b || hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
            st = QSD_ERR_HIP;
        agg[r.kind].launches += 1;
        agg[r.kind].total_ms += ms;
        agg[r.kind].bytes += r.bytes;
        if (r.a) g_pool.push_back(r.a);
        if (r.b) g_pool.push_back(r.b);
    }
    g_prof.clear();
    int n = 0;
    for (int k = 0; k < kNumKinds; ++k) {
        if (!agg[k].launches) continue;
        if (out && n < max) {
            out[n] = agg[k];
            std::strncpy(out[n].name, kKindName[k], sizeof(out[n].name) - 1);
        }
        ++n;
    }
    if (count) *count = out ? std::min(n, (int)max) : n;
    return st;
}

qsd_status qsd_device_status(void* ws, hipStream_t stream, uint32_t* code) {
    if (!ws || !code) return QSD_ERR_NULL;
    static const uint32_t zero = 0;
    uint32_t word = 0;
    if (hipMemcpyAsync(&word, (char*)ws + kCtlErr * 4, 4, hipMemcpyDeviceToHost, stream) != hipSuccess)
        return QSD_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return QSD_ERR_HIP;
    // read and clear: the bits accumulate until the host has seen them
    if (hipMemcpyAsync((char*)ws + kCtlErr * 4, &zero, 4, hipMemcpyHostToDevice, stream) != hipSuccess)
        return QSD_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return QSD_ERR_HIP;
    *code = word;
    return QSD_OK;
}

qsd_status qsd_csf_workspace(qsd_plan_t plan, size_t* bytes) {
    if (!plan || !bytes) return QSD_ERR_NULL;
    const uint64_t N = (uint64_t)std::max<int64_t>(plan->p.nnz, 1);
    *bytes = up(kCtlWords * 4) + up(cdiv(N, kCsfTile) * 8 * 4);
    return QSD_OK;
}

qsd_status qsd_pack_csf(qsd_plan_t plan, int64_t nnz, const void* const* sorted_crd, void* const* pos,
                        void* const* crd, int64_t* fiber_counts, void* ws, size_t ws_bytes,
                        hipStream_t stream) {
    if (!plan || !sorted_crd || !pos || !crd || !fiber_counts) return QSD_ERR_NULL;
    const PlanData& p = plan->p;
    if (nnz < 0 || nnz > p.nnz) return QSD_ERR_TOO_LARGE;
    size_t need = 0;
    qsd_csf_workspace(plan, &need);
    if (!ws || ws_bytes < need) return QSD_ERR_WORKSPACE;
    for (int m = 0; m < p.r; ++m)
        if (!sorted_crd[m] || !pos[m] || !crd[m]) return QSD_ERR_NULL;
    const uint32_t n = (uint32_t)nnz;
    char* W = (char*)ws;
    uint32_t* ctl = (uint32_t*)W;
    uint32_t* st = (uint32_t*)(W + up(kCtlWords * 4));
    const uint64_t tiles = cdiv(std::max<uint32_t>(n, 1), kCsfTile);
    ZeroArgs z{};
    z.ctl = ctl;
    z.ptr[1] = st;
    z.words[1] = tiles * 8;
    if (timed(kZero, 0, stream, [&] { return launch_zero(z, stream); }) != hipSuccess) return QSD_ERR_HIP;
    if (n == 0) {
        // one root with no children: F_0 = 1, pos_1 = [0, 0], F_d = 0 for d >= 1
        std::vector<int64_t> fc(p.r + 1, 0);
        fc[0] = 1;
        // small host->device copies of constants
        static thread_local std::vector<int64_t> keep;
        keep = fc;
        if (hipMemcpyAsync(fiber_counts, keep.data(), 8 * (p.r + 1), hipMemcpyHostToDevice, stream) != hipSuccess)
            return QSD_ERR_HIP;
        static const int64_t zeros[2] = {0, 0};
        if (hipMemcpyAsync(pos[0], zeros, p.crd_bytes == 8 ? 16 : 8, hipMemcpyHostToDevice, stream) != hipSuccess)
            return QSD_ERR_HIP;
        if (hipStreamSynchronize(stream) != hipSuccess) return QSD_ERR_HIP;
        return QSD_OK;
    }
    CsfArgs ca{};
    for (int d = 0; d < p.r; ++d) {
        ca.crd[d] = sorted_crd[p.out_order[d]];  // level d + 1 holds mode sigma_{d+1}
        ca.pos[d] = pos[d];
        ca.out_crd[d] = crd[d];
    }
    ca.r = p.r;
    ca.n = n;
    ca.fiber_counts = fiber_counts;
    ca.status = st;
    ca.tile_counter = ctl + kCtlBoundCnt;
    ca.err = ctl + kCtlErr;
    if (timed(kCsf, 0, stream, [&] { return launch_csf(ca, p.crd_bytes, stream); }) != hipSuccess) return QSD_ERR_HIP;
    return QSD_OK;
}

}  // extern "C"

// ---- CSF -> CSF: expansion to coordinates, the plan's transposition, the pack
namespace {
struct CsfTLayout {
    size_t plan_ws = 0, csf_ws = 0, status = 0, flags = 0, coo_in = 0, coo_out = 0, total = 0;
    uint64_t tiles = 0;
};
CsfTLayout csf_t_layout(qsd_plan_t plan) {
    const PlanData& p = plan->p;
    const uint64_t N = (uint64_t)std::max<int64_t>(p.nnz, 1);
    CsfTLayout L;
    size_t at = 0;
    L.plan_ws = at;  // first: its control block is the call's (status bits, counters)
    at = up(at + plan->L.total);
    size_t cw = 0;
    qsd_csf_workspace(plan, &cw);
    L.csf_ws = at;
    at = up(at + cw);
    L.tiles = cdiv(N, kBoundTile);
    L.status = at;
    at = up(at + (size_t)std::max(p.r - 1, 1) * L.tiles * 4);
    L.flags = at;
    at = up(at + (size_t)std::max(p.r - 1, 1) * up(N));
    L.coo_in = at;
    at = up(at + (size_t)p.r * up(N * p.crd_bytes));
    L.coo_out = at;
    at = up(at + (size_t)p.r * up(N * p.crd_bytes));
    L.total = at;
    return L;
}
}  // namespace

extern "C" {

qsd_status qsd_csf_transpose_workspace(qsd_plan_t plan, size_t* bytes) {
    if (!plan || !bytes) return QSD_ERR_NULL;
    *bytes = csf_t_layout(plan).total;
    return QSD_OK;
}

qsd_status qsd_csf_transpose(qsd_plan_t plan, int64_t nnz, const void* const* in_pos, const void* const* in_crd,
                             const void* in_val, void* const* out_pos, void* const* out_crd, void* out_val,
                             int64_t* fiber_counts, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!plan || !in_pos || !in_crd || !out_pos || !out_crd || !fiber_counts) return QSD_ERR_NULL;
    const PlanData& p = plan->p;
    if (nnz < 0 || nnz > p.nnz) return QSD_ERR_TOO_LARGE;
    const CsfTLayout L = csf_t_layout(plan);
    if (!ws || ws_bytes < L.total) return QSD_ERR_WORKSPACE;
    for (int m = 0; m < p.r; ++m)
        if (!in_pos[m] || !in_crd[m] || !out_pos[m] || !out_crd[m]) return QSD_ERR_NULL;
    if (nnz > 0 && (!in_val || !out_val)) return QSD_ERR_NULL;
    char* W = (char*)ws;
    const uint32_t n = (uint32_t)nnz;
    const uint64_t N = (uint64_t)std::max<int64_t>(p.nnz, 1);
    const void* coo_in[kMaxR];
    void* coo_out[kMaxR];
    for (int m = 0; m < p.r; ++m) coo_out[m] = W + L.coo_out + (size_t)m * up(N * p.crd_bytes);
    if (n > 0) {
        uint32_t* ctl = (uint32_t*)(W + L.plan_ws);
        ZeroArgs z{};
        z.ctl = ctl;
        z.ptr[0] = (uint32_t*)(W + L.status);
        z.words[0] = (uint64_t)std::max(p.r - 1, 1) * L.tiles;
        z.ptr[1] = (uint32_t*)(W + L.flags);
        z.words[1] = (uint64_t)std::max(p.r - 1, 1) * up(N) / 4;
        if (timed(kZero, 0, stream, [&] { return launch_zero(z, stream); }) != hipSuccess) return QSD_ERR_HIP;
        // levels 1 .. r-1 of the input tree (level d stores mode in_order[d-1]) expand into
        // coordinate arrays; the leaf level is the last mode's coordinate array already
        for (int d = 1; d < p.r; ++d) {
            CsfExpandArgs a{};
            for (int e = 0; e < p.r; ++e) {
                a.pos[e] = in_pos[e];
                a.crd[e] = in_crd[e];
            }
            a.r = p.r;
            a.level = d;
            a.n = n;
            a.flags = (uint8_t*)(W + L.flags) + (size_t)(d - 1) * up(N);
            a.status = (uint32_t*)(W + L.status) + (size_t)(d - 1) * L.tiles;
            a.tile_counter = ctl + kCtlWords - 1 - d;
            a.err = ctl + kCtlErr;
            void* out = W + L.coo_in + (size_t)p.in_order[d - 1] * up(N * p.crd_bytes);
            a.out = out;
            coo_in[p.in_order[d - 1]] = out;
            if (timed(kCsfExpand, (double)n * (1.0 + 2.0 * p.crd_bytes), stream,
                      [&] {
                          hipError_t e = launch_csf_mark(a, p.crd_bytes, stream);
                          return e == hipSuccess ? launch_csf_expand(a, p.crd_bytes, stream) : e;
                      }) != hipSuccess)
                return QSD_ERR_HIP;
        }
        coo_in[p.in_order[p.r - 1]] = in_crd[p.r - 1];
        const qsd_status st = qsd_transpose(plan, nnz, coo_in, in_val, coo_out, out_val, W + L.plan_ws,
                                            plan->L.total, stream);
        if (st != QSD_OK) return st;
    }
    size_t cw = 0;
    qsd_csf_workspace(plan, &cw);
    return qsd_pack_csf(plan, nnz, (const void* const*)coo_out, out_pos, out_crd, fiber_counts, W + L.csf_ws, cw,
                        stream);
}

}  // extern "C"

// =========================================================================================
// Batched transposition
// =========================================================================================
namespace {

DevKey dev_key(const KeySpec& ks, int r) {
    DevKey k{};
    for (int m = 0; m < r; ++m) {
        k.mask[m] = ks.width[m] ? ((ks.width[m] >= 64) ? ~0ull : ((1ull << ks.width[m]) - 1)) : 0;
        k.src_lo[m] = ks.src_lo[m];
        k.dst[m] = ks.dst[m];
    }
    return k;
}

struct BTensor {
    int r = 0;
    uint32_t n = 0;
    int bits[kMaxR] = {};
    int in_order[kMaxR] = {}, out_order[kMaxR] = {};
    std::vector<int> keys;       // flattened key, most significant first
    std::vector<SubKey> subs;    // least significant first
    int D = 0;                   // digit passes
    bool small = false;
    bool packed = false;         // first pass packs, middle passes move words, last unpacks
    uint32_t tile0 = 0, tiles = 0;
    size_t rec_off = 0;          // workspace record area (large tensors)
    size_t val_off = 0;          // workspace value array (large tensors)
    size_t pk_off[2] = {0, 0};   // packed-word ping-pong buffers (packed tensors)
    size_t hist_word = 0;        // first histogram word (large tensors)
};

// Record layouts of a batched pass; every tensor's pass p has one, and each layout present
// in pass p is one launch.
enum BatchKind { kKindSoA = 0, kKindPack = 1, kKindWords = 2, kKindUnpack = 3, kKinds = 4 };
int kind_of(const BTensor& x, int p) {
    if (!x.packed) return kKindSoA;
    return p == 0 ? kKindPack : (p == x.D - 1 ? kKindUnpack : kKindWords);
}

}  // namespace

struct qsd_batch_s {
    int crd_bytes = 4, val_bytes = 8, rmax = 1;
    qsd_tuning tun{0, 8, kSmallCap};
    std::vector<BTensor> t;
    // derived from the tuning
    int items = 16, tile = 4096, maxD = 0;
    bool pack = true;                              // packed records for tensors that fit
    uint32_t total_tiles = 0;
    std::vector<int> large, small;                 // tensor indices
    std::vector<std::vector<uint32_t>> launch_tiles;  // per (pass, layout): stable tile ids
    size_t hist_words = 0;
    // workspace layout
    size_t off_ctl = 0, off_rec = 0, off_hist = 0, off_status[2] = {0, 0}, off_tab = 0, total = 0;
    size_t tab_pass = 0, tab_map = 0, tab_job = 0, tab_hjob = 0, tab_sjob = 0, tab_bytes = 0;
    std::vector<size_t> map_off;                   // per (pass, layout): word offset in the map table
    // bound host tables
    std::vector<char> host_tab;
    bool bound = false;
    void* bound_ws = nullptr;
};

struct qsd_graph_s {
    hipGraphExec_t exec = nullptr;
};

namespace {

size_t rec_bytes(const qsd_batch_s* b, int r) { return (size_t)r * b->crd_bytes + b->val_bytes; }

qsd_status batch_derive(qsd_batch_s* b) {
    const qsd_tuning& tu = b->tun;
    b->items = digit_items(b->rmax, b->crd_bytes, b->val_bytes, tu.items);
    b->tile = kBlock * b->items;
    b->large.clear();
    b->small.clear();
    b->maxD = 0;
    b->total_tiles = 0;
    b->hist_words = 0;
    size_t rec = 0;
    for (size_t i = 0; i < b->t.size(); ++i) {
        BTensor& x = b->t[i];
        x.subs = make_subkeys(x.keys, x.bits, tu.radix_bits);
        x.D = 0;
        for (auto& sk : x.subs) x.D += (int)sk.passes.size();
        if (x.subs.size() > 2 || x.D > 16) return QSD_ERR_UNSUPPORTED;
        x.small = x.n <= (uint32_t)tu.small_cap;
        if (x.n == 0) continue;
        if (x.small) {
            b->small.push_back((int)i);
            continue;
        }
        if (x.D == 0) {  // identity: one zero-width pass copies the records stably
            SubKey sk{};
            std::memset(&sk.key, 0, sizeof(sk.key));
            sk.passes.push_back(PassSpec{0, 0});
            x.subs.assign(1, sk);
            x.D = 1;
        }
        b->large.push_back((int)i);
        x.tile0 = b->total_tiles;
        x.tiles = (x.n + b->tile - 1) / b->tile;
        b->total_tiles += x.tiles;
        x.hist_word = b->hist_words;
        b->hist_words += (size_t)x.D * kBins;
        int total_bits = 0;
        for (int m = 0; m < x.r; ++m) total_bits += x.bits[m];
        x.packed = b->pack && x.D >= 2 && x.subs.size() == 1 && total_bits <= 64;
        x.rec_off = rec;
        if (x.packed) {  // the coordinate arrays live only as words between the first and last pass
            for (int k = 0; k < 2; ++k) {
                x.pk_off[k] = rec;
                rec = up(rec + (size_t)x.n * 8);
            }
        } else {
            for (int m = 0; m < x.r; ++m) rec = up(rec + (size_t)x.n * b->crd_bytes);
        }
        x.val_off = rec;
        rec = up(rec + (size_t)x.n * b->val_bytes);
        b->maxD = std::max(b->maxD, x.D);
    }
    b->launch_tiles.assign((size_t)b->maxD * kKinds, {});
    for (int p = 0; p < b->maxD; ++p)
        for (int i : b->large)
            if (p < b->t[i].D) {
                auto& lt = b->launch_tiles[(size_t)p * kKinds + kind_of(b->t[i], p)];
                for (uint32_t k = 0; k < b->t[i].tiles; ++k) lt.push_back(b->t[i].tile0 + k);
            }
    // layout
    size_t at = 0;
    b->off_ctl = at;
    at = up(at + kCtlWords * 4);
    b->off_rec = at;
    at = up(at + rec);
    b->off_hist = at;
    at = up(at + b->hist_words * 4);
    for (int k = 0; k < 2; ++k) {
        b->off_status[k] = at;
        at = up(at + (size_t)b->total_tiles * kBins * 4);
    }
    const size_t nl = b->large.size();
    b->off_tab = at;
    size_t tb = 0;
    b->tab_pass = tb;
    tb = up(tb + (size_t)b->maxD * nl * sizeof(BatchPass));
    b->tab_map = tb;
    b->map_off.assign(b->launch_tiles.size(), 0);
    size_t words = 0;  // four words per launch tile
    for (size_t l = 0; l < b->launch_tiles.size(); ++l) {
        b->map_off[l] = words;
        words += 4 * b->launch_tiles[l].size();
    }
    tb = up(tb + words * 4);
    b->tab_job = tb;
    tb = up(tb + (size_t)b->total_tiles * 4);
    b->tab_hjob = tb;
    tb = up(tb + nl * sizeof(BatchHistJob));
    b->tab_sjob = tb;
    tb = up(tb + b->small.size() * sizeof(BatchSmallJob));
    b->tab_bytes = tb;
    at = up(at + tb);
    b->total = at;
    b->bound = false;
    return QSD_OK;
}

}  // namespace

extern "C" {

qsd_status qsd_batch_plan(const qsd_desc* descs, int32_t count, qsd_batch_t* out) {
    if (!out || (!descs && count > 0)) return QSD_ERR_NULL;
    *out = nullptr;
    if (count < 0) return QSD_ERR_TOO_LARGE;
    auto* b = new qsd_batch_s();
    for (int i = 0; i < count; ++i) {
        const qsd_status st = check_desc(&descs[i]);
        if (st != QSD_OK) {
            delete b;
            return st;
        }
        const int cb = descs[i].crd_type == QSD_I64 ? 8 : 4, vb = descs[i].val_type == QSD_F64 ? 8 : 4;
        if (i == 0) {
            b->crd_bytes = cb;
            b->val_bytes = vb;
        } else if (cb != b->crd_bytes || vb != b->val_bytes) {
            delete b;
            return QSD_ERR_UNSUPPORTED;
        }
        BTensor x;
        x.r = descs[i].order;
        x.n = (uint32_t)descs[i].nnz;
        for (int m = 0; m < x.r; ++m) {
            x.bits[m] = bits_for_extent(descs[i].extents[m]);
            x.in_order[m] = descs[i].in_order[m];
            x.out_order[m] = descs[i].out_order[m];
        }
        x.keys = flattened_key(x.r, x.in_order, x.out_order, x.bits);
        b->rmax = std::max(b->rmax, x.r);
        b->t.push_back(x);
    }
    const qsd_status st = batch_derive(b);
    if (st != QSD_OK) {
        delete b;
        return st;
    }
    *out = b;
    return QSD_OK;
}

void qsd_batch_destroy(qsd_batch_t b) { delete b; }

qsd_status qsd_batch_set_tuning(qsd_batch_t b, const qsd_tuning* tu) {
    if (!b || !tu) return QSD_ERR_NULL;
    if ((tu->items != 0 && tu->items != 8 && tu->items != 16) || tu->radix_bits < 4 || tu->radix_bits > 8 ||
        tu->small_cap < 0 || tu->small_cap > kSmallCap)
        return QSD_ERR_UNSUPPORTED;
    const qsd_tuning old = b->tun;
    b->tun = *tu;
    const qsd_status st = batch_derive(b);
    if (st != QSD_OK) {
        b->tun = old;
        batch_derive(b);
    }
    return st;
}

qsd_status qsd_batch_get_tuning(qsd_batch_t b, qsd_tuning* tu) {
    if (!b || !tu) return QSD_ERR_NULL;
    *tu = b->tun;
    tu->items = b->items;
    return QSD_OK;
}

qsd_status qsd_batch_workspace(qsd_batch_t b, size_t* bytes) {
    if (!b || !bytes) return QSD_ERR_NULL;
    *bytes = b->total;
    return QSD_OK;
}

qsd_status qsd_batch_workspace_max(qsd_batch_t b, size_t* bytes) {
    if (!b || !bytes) return QSD_ERR_NULL;
    // every tuning qsd_batch_set_tuning accepts; small_cap = 0 makes every tensor large, which
    // needs the most workspace for a given digit width and item count
    const qsd_tuning keep = b->tun;
    size_t mx = 0;
    for (int items : {8, 16})
        for (int rb = 4; rb <= 8; ++rb)
            for (int cap : {0, keep.small_cap}) {
                b->tun = qsd_tuning{items, rb, cap};
                if (batch_derive(b) == QSD_OK) mx = std::max(mx, b->total);
            }
    b->tun = keep;
    batch_derive(b);
    *bytes = mx;
    return QSD_OK;
}

qsd_status qsd_batch_bind(qsd_batch_t b, const qsd_batch_io* io, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!b || (!io && !b->t.empty())) return QSD_ERR_NULL;
    if (!ws || ws_bytes < b->total) return QSD_ERR_WORKSPACE;
    char* W = (char*)ws;
    b->host_tab.assign(b->tab_bytes, 0);
    char* H = b->host_tab.data();
    const size_t nl = b->large.size();
    // per-launch pass tables of the large tensors
    for (int p = 0; p < b->maxD; ++p) {
        for (size_t li = 0; li < nl; ++li) {
            const BTensor& x = b->t[b->large[li]];
            const qsd_batch_io& q = io[b->large[li]];
            BatchPass& e = ((BatchPass*)(H + b->tab_pass))[(size_t)p * nl + li];
            std::memset(&e, 0, sizeof(e));
            e.active = p < x.D;
            e.r = x.r;
            e.n = x.n;
            e.tile0 = x.tile0;
            if (!e.active) continue;
            // hop p writes OUT when (D-1-p) is even, else the tensor's workspace records
            auto buf = [&](int hop, int m) -> void* {
                const bool to_out = ((x.D - 1 - hop) % 2) == 0;
                if (to_out) return m < x.r ? q.out_crd[m] : q.out_val;
                if (m == x.r) return W + b->off_rec + x.val_off;
                size_t off = x.rec_off;
                for (int k = 0; k < m; ++k) off = up(off + (size_t)x.n * b->crd_bytes);
                return W + b->off_rec + off;
            };
            for (int m = 0; m <= x.r; ++m) {
                const void* src = p == 0 ? (m < x.r ? q.in_crd[m] : q.in_val) : buf(p - 1, m);
                void* dst = buf(p, m);
                if (m < x.r) {
                    e.src_crd[m] = src;
                    e.dst_crd[m] = dst;
                } else {
                    e.src_val = src;
                    e.dst_val = dst;
                }
            }
            int k = p, sub = 0;
            while (k >= (int)x.subs[sub].passes.size()) k -= (int)x.subs[sub++].passes.size();
            e.key = dev_key(x.subs[sub].key, x.r);
            e.lo = x.subs[sub].passes[k].lo;
            e.bits = x.subs[sub].passes[k].bits;
            e.hist = (const uint32_t*)(W + b->off_hist) + x.hist_word + (size_t)p * kBins;
            if (x.packed) {  // words in the tensor's two word buffers between the first and last pass
                pack_layout(x.r, x.bits, x.subs[0].key, e.pk_pos, e.pk_mask);
                void* P[2] = {W + b->off_rec + x.pk_off[0], W + b->off_rec + x.pk_off[1]};
                const int kind = kind_of(x, p);
                if (kind == kKindPack) {
                    e.dst_crd[0] = P[0];
                } else if (kind == kKindWords) {
                    std::memset(e.src_crd, 0, sizeof(e.src_crd));
                    std::memset(e.dst_crd, 0, sizeof(e.dst_crd));
                    e.src_crd[0] = P[(p - 1) % 2];
                    e.dst_crd[0] = P[p % 2];
                    std::memset(&e.key, 0, sizeof(e.key));
                    e.key.mask[0] = x.subs[0].key.bits >= 64 ? ~0ull : ((1ull << x.subs[0].key.bits) - 1);
                    e.r = 1;
                } else {  // unpacking: words in, coordinate arrays out
                    std::memset(e.src_crd, 0, sizeof(e.src_crd));
                    e.src_crd[0] = P[(p - 1) % 2];
                }
            }
        }
    }
    uint32_t* tj = (uint32_t*)(H + b->tab_job);
    for (size_t li = 0; li < nl; ++li) {
        const BTensor& x = b->t[b->large[li]];
        for (uint32_t k = 0; k < x.tiles; ++k) tj[x.tile0 + k] = (uint32_t)li;
    }
    // launch tiles: stable tile id, tensor, first record, records
    for (size_t l = 0; l < b->launch_tiles.size(); ++l) {
        uint32_t* map = (uint32_t*)(H + b->tab_map) + b->map_off[l];
        for (size_t j = 0; j < b->launch_tiles[l].size(); ++j) {
            const uint32_t t = b->launch_tiles[l][j];
            const uint32_t li = tj[t];
            const BTensor& x = b->t[b->large[li]];
            const uint32_t start = (t - x.tile0) * (uint32_t)b->tile;
            map[4 * j + 0] = t;
            map[4 * j + 1] = li;
            map[4 * j + 2] = start;
            map[4 * j + 3] = std::min<uint32_t>((uint32_t)b->tile, x.n - start);
        }
    }
    BatchHistJob* hj = (BatchHistJob*)(H + b->tab_hjob);
    for (size_t li = 0; li < nl; ++li) {
        const BTensor& x = b->t[b->large[li]];
        BatchHistJob& j = hj[li];
        std::memset(&j, 0, sizeof(j));
        for (int m = 0; m < x.r; ++m) j.crd[m] = io[b->large[li]].in_crd[m];
        j.r = x.r;
        j.nsub = (int)x.subs.size();
        int pidx = 0;
        for (int sidx = 0; sidx < j.nsub; ++sidx) {
            j.key[sidx] = dev_key(x.subs[sidx].key, x.r);
            for (const auto& ps : x.subs[sidx].passes) {
                j.lo[pidx] = ps.lo;
                j.bits[pidx] = ps.bits;
                j.sub[pidx] = sidx;
                ++pidx;
            }
        }
        j.npass = pidx;
        j.n = x.n;
        j.tile0 = x.tile0;
        j.hist = (uint32_t*)(W + b->off_hist) + x.hist_word;
    }
    BatchSmallJob* sj = (BatchSmallJob*)(H + b->tab_sjob);
    for (size_t si = 0; si < b->small.size(); ++si) {
        const BTensor& x = b->t[b->small[si]];
        const qsd_batch_io& q = io[b->small[si]];
        BatchSmallJob& j = sj[si];
        std::memset(&j, 0, sizeof(j));
        for (int m = 0; m < x.r; ++m) {
            j.src_crd[m] = q.in_crd[m];
            j.dst_crd[m] = q.out_crd[m];
        }
        j.src_val = q.in_val;
        j.dst_val = q.out_val;
        j.nsub = (int)x.subs.size();
        for (int sidx = 0; sidx < j.nsub; ++sidx) {
            j.key[sidx] = dev_key(x.subs[sidx].key, x.r);
            j.key_bits[sidx] = x.subs[sidx].key.bits;
        }
        j.r = x.r;
        j.n = x.n;
    }
    if (b->tab_bytes) {
        if (hipMemcpyAsync(W + b->off_tab, H, b->tab_bytes, hipMemcpyHostToDevice, stream) != hipSuccess)
            return QSD_ERR_HIP;
        if (hipStreamSynchronize(stream) != hipSuccess) return QSD_ERR_HIP;
    }
    b->bound = true;
    b->bound_ws = ws;
    return QSD_OK;
}

qsd_status qsd_batch_transpose(qsd_batch_t b, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!b) return QSD_ERR_NULL;
    if (!ws || ws_bytes < b->total || !b->bound || ws != b->bound_ws) return QSD_ERR_WORKSPACE;
    char* W = (char*)ws;
    uint32_t* ctl = (uint32_t*)(W + b->off_ctl);
    uint32_t* S[2] = {(uint32_t*)(W + b->off_status[0]), (uint32_t*)(W + b->off_status[1])};
    const char* T = W + b->off_tab;
    hipError_t e;
#define QSD_CK(x)                                        \
    do {                                                 \
        if ((e = (x)) != hipSuccess) return QSD_ERR_HIP; \
    } while (0)
    ZeroArgs z{};
    z.ctl = ctl;
    if (b->hist_words) {
        z.ptr[1] = (uint32_t*)(W + b->off_hist);
        z.words[1] = b->hist_words;
    }
    QSD_CK(timed(kZero, 0, stream, [&] { return launch_zero(z, stream); }));
    if (!b->large.empty()) {
        BatchHistArgs ha{};
        ha.jobs = (const BatchHistJob*)(T + b->tab_hjob);
        ha.tile_job = (const uint32_t*)(T + b->tab_job);
        ha.ntiles = b->total_tiles;
        ha.tile = (uint32_t)b->tile;
        ha.status_zero = S[0];
        const int grid = (int)std::max<uint32_t>(
            1, std::min<uint32_t>(b->total_tiles, (uint32_t)(device_cu_count() * hist_blocks_per_cu())));
        QSD_CK(timed(kHistBatch, 0, stream, [&] { return launch_hist_batch(ha, b->rmax, b->crd_bytes, grid, stream); }));
        QSD_CK(timed(kHistBatch, 0, stream, [&] {
            return launch_hist_prefix((uint32_t*)(W + b->off_hist), (uint32_t)(b->hist_words / kBins), stream);
        }));
    }
    if (!b->small.empty()) {
        const auto* jobs = (const BatchSmallJob*)(T + b->tab_sjob);
        const uint32_t nj = (uint32_t)b->small.size();
        QSD_CK(timed(kSmallBatch, 0, stream,
                     [&] { return launch_small_batch(jobs, nj, b->rmax, b->crd_bytes, b->val_bytes, stream); }));
    }
    const size_t nl = b->large.size();
    for (int p = 0; p < b->maxD; ++p) {
        for (int kind = 0; kind < kKinds; ++kind) {
            const size_t l = (size_t)p * kKinds + kind;
            if (b->launch_tiles[l].empty()) continue;
            DigitArgs da{};
            da.seg_mode = 2;
            da.pk = kind == kKindPack ? 1 : (kind == kKindUnpack ? 2 : 0);
            da.ntiles = (uint32_t)b->launch_tiles[l].size();
            da.tile_map = (const uint32_t*)(T + b->tab_map) + b->map_off[l];
            da.batch = (const BatchPass*)(T + b->tab_pass) + (size_t)p * nl;
            da.status = S[p % 2];
            da.status_next = (p + 1 < b->maxD) ? S[(p + 1) % 2] : nullptr;
            da.tile_counter = ctl + kCtlPassCnt + kPassCounters * l;
            da.err = ctl + kCtlErr;
            const int r_launch = kind == kKindWords ? 1 : b->rmax;
            const int cb_launch = kind == kKindWords ? 8 : b->crd_bytes;
            double bytes = 0;
            for (int i : b->large) {
                const BTensor& x = b->t[i];
                if (p >= x.D || kind_of(x, p) != kind) continue;
                const double soa = (double)rec_bytes(b, x.r), words = 8.0 + b->val_bytes;
                bytes += x.n * (kind == kKindSoA ? 2 * soa : kind == kKindWords ? 2 * words : soa + words);
            }
            QSD_CK(timed(kDigitBatch, bytes, stream, [&] {
                return launch_digit_batch(da, r_launch, cb_launch, b->val_bytes, b->items, stream);
            }));
        }
    }
#undef QSD_CK
    return QSD_OK;
}

qsd_status qsd_batch_tune(qsd_batch_t b, const qsd_batch_io* io, void* ws, size_t ws_bytes, hipStream_t stream,
                          int32_t reps, qsd_tuning* best, float* best_ms) {
    if (!b || !ws) return QSD_ERR_NULL;
    if (reps < 1) reps = 1;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return QSD_ERR_HIP;
    qsd_tuning bt = b->tun;
    float bms = -1.f;
    qsd_status st = QSD_OK;
    for (int items : {8, 16})
        for (int rb : {6, 7, 8})
            for (int cap : {0, 1024, kSmallCap}) {
                const qsd_tuning cand{items, rb, cap};
                if (qsd_batch_set_tuning(b, &cand) != QSD_OK || b->total > ws_bytes) continue;
                if ((st = qsd_batch_bind(b, io, ws, ws_bytes, stream)) != QSD_OK) goto done;
                if ((st = qsd_batch_transpose(b, ws, ws_bytes, stream)) != QSD_OK) goto done;  // warm-up
                float mn = 1e30f;
                for (int k = 0; k < reps; ++k) {
                    if (hipEventRecord(e0, stream) != hipSuccess) {
                        st = QSD_ERR_HIP;
                        goto done;
                    }
                    if ((st = qsd_batch_transpose(b, ws, ws_bytes, stream)) != QSD_OK) goto done;
                    float ms = 0.f;
                    if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                        st = QSD_ERR_HIP;
                        goto done;
                    }
                    mn = std::min(mn, ms);
                }
                if (bms < 0 || mn < bms) {
                    bms = mn;
                    bt = cand;
                }
            }
    if (qsd_batch_set_tuning(b, &bt) == QSD_OK) st = qsd_batch_bind(b, io, ws, ws_bytes, stream);
done:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best) *best = bt;
    if (best_ms) *best_ms = bms;
    return st;
}

qsd_status qsd_batch_tune_key(qsd_batch_t b, char* key, size_t key_bytes) {
    if (!b || !key) return QSD_ERR_NULL;
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return QSD_ERR_HIP;
    std::string arch(prop.gcnArchName);
    arch = arch.substr(0, arch.find(':'));  // without the feature suffixes
    uint64_t nnz = 0;
    for (const auto& x : b->t) nnz += x.n;
    auto lg = [](uint64_t v) { int k = 0; while (v > 1) { v >>= 1; ++k; } return k; };
    const std::string k = arch + "/c" + std::to_string(b->crd_bytes) + "/v" + std::to_string(b->val_bytes) + "/r" +
                          std::to_string(b->rmax) + "/n" + std::to_string(lg(nnz + 1)) + "/t" +
                          std::to_string(lg(std::max<uint64_t>(b->t.size(), 1)));
    if (k.size() + 1 > key_bytes) return QSD_ERR_TOO_LARGE;
    std::memcpy(key, k.c_str(), k.size() + 1);
    return QSD_OK;
}

qsd_status qsd_batch_tune_cached(qsd_batch_t b, const qsd_batch_io* io, void* ws, size_t ws_bytes,
                                 hipStream_t stream, int32_t reps, const char* cache_path, qsd_tuning* best,
                                 float* best_ms, int32_t* from_cache) {
    if (!b || !ws || !cache_path) return QSD_ERR_NULL;
    if (from_cache) *from_cache = 0;
    char key[128];
    qsd_status st = qsd_batch_tune_key(b, key, sizeof(key));
    if (st != QSD_OK) return st;
    if (FILE* f = std::fopen(cache_path, "r")) {
        char line[256], k[128];
        qsd_tuning t{};
        float ms = 0.f;
        bool hit = false;
        while (!hit && std::fgets(line, sizeof(line), f))  // the first matching line is used
            hit = std::sscanf(line, "%127s %d %d %d %f", k, &t.items, &t.radix_bits, &t.small_cap, &ms) == 5 &&
                  std::strcmp(k, key) == 0;
        std::fclose(f);
        if (hit) {
            const qsd_tuning old = b->tun;
            if (qsd_batch_set_tuning(b, &t) == QSD_OK && b->total <= ws_bytes) {
                st = qsd_batch_bind(b, io, ws, ws_bytes, stream);
                if (st == QSD_OK) {
                    if (best) *best = t;
                    if (best_ms) *best_ms = ms;
                    if (from_cache) *from_cache = 1;
                }
                return st;
            }
            qsd_batch_set_tuning(b, &old);  // unusable entry: tune afresh
        }
    }
    qsd_tuning t{};
    float ms = 0.f;
    st = qsd_batch_tune(b, io, ws, ws_bytes, stream, reps, &t, &ms);
    if (st != QSD_OK) return st;
    if (FILE* f = std::fopen(cache_path, "a")) {
        std::fprintf(f, "%s %d %d %d %.4f\n", key, t.items, t.radix_bits, t.small_cap, ms);
        std::fclose(f);
    }
    if (best) *best = t;
    if (best_ms) *best_ms = ms;
    return QSD_OK;
}

qsd_status qsd_batch_graph(qsd_batch_t b, void* ws, size_t ws_bytes, qsd_graph_t* out) {
    if (!b || !out) return QSD_ERR_NULL;
    *out = nullptr;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return QSD_ERR_HIP;
    hipGraph_t g = nullptr;
    qsd_status st = QSD_OK;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(s);
        return QSD_ERR_HIP;
    }
    st = qsd_batch_transpose(b, ws, ws_bytes, s);
    const hipError_t ec = hipStreamEndCapture(s, &g);
    (void)hipStreamDestroy(s);
    if (st != QSD_OK || ec != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return st != QSD_OK ? st : QSD_ERR_HIP;
    }
    auto* gr = new qsd_graph_s();
    const hipError_t ei = hipGraphInstantiate(&gr->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
        delete gr;
        return QSD_ERR_HIP;
    }
    *out = gr;
    return QSD_OK;
}

qsd_status qsd_graph_launch(qsd_graph_t g, hipStream_t stream) {
    if (!g || !g->exec) return QSD_ERR_NULL;
    return hipGraphLaunch(g->exec, stream) == hipSuccess ? QSD_OK : QSD_ERR_HIP;
}

void qsd_graph_destroy(qsd_graph_t g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    delete g;
}

}  // extern "C"
