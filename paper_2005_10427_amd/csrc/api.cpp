// C ABI of libqsd: argument checks, workspace layout, and the launch sequence of a plan.
#include "../../include/qsd.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

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
    size_t seg_start = 0, region_seg = 0, bstatus = 0, bstatus_words = 0, med = 0, large = 0, seg_hist = 0;
    size_t tile_map = 0;
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
    int tile = 0;
    int items = 16;
    std::vector<size_t> sub_hist_off;  // word offset of each global sub-key's histograms
    int nseg_groups = 0;
};

namespace {

void make_layout(qsd_plan_s* q) {
    const PlanData& p = q->p;
    Layout& L = q->L;
    const uint64_t N = (uint64_t)std::max<int64_t>(p.nnz, 1);
    int pref = 0;
    if (const char* e = std::getenv("QSD_DIGIT_ITEMS")) pref = std::atoi(e);  // tuning override
    q->items = digit_items(p.r, p.crd_bytes, p.val_bytes, pref);
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
        at = up(at + (size_t)L.max_tiles_large * 4);
        L.bstatus_words = cdiv(N, kBoundTile);
        L.bstatus = at;
        at = up(at + L.bstatus_words * 4 * q->nseg_groups);
        L.med = at;
        at = up(at + (size_t)L.max_med * 8);
        L.large = at;
        at = up(at + (size_t)L.max_large * sizeof(SegRec));
        L.seg_hist = at;
        at = up(at + (size_t)L.max_large * max_seg_passes * kBins * 4);
    }
    L.total = at;
}

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

struct Bufs {
    const void* crd[kMaxR];
    const void* val;
};

// ---- launch timing (qsd_profile_*)
enum Kind { kZero, kCopy, kValidate, kHist, kDigit, kBoundary, kClassify, kSmall, kHistSeg, kDigitSeg, kCsf, kNumKinds };
const char* kKindName[kNumKinds] = {"zero", "copy", "validate", "hist", "digit", "boundary",
                                    "classify", "small", "hist_seg", "digit_seg", "csf"};
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
    std::lock_guard<std::mutex> lk(g_prof_mu);
    ProfRec r{kind, pool_event(), pool_event(), bytes};
    if (r.a) hipEventRecord(r.a, s);
    const hipError_t e = fn();
    if (r.b) hipEventRecord(r.b, s);
    g_prof.push_back(r);
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
    if (sched < QSD_SCHED_AUTO || sched > QSD_SCHED_LSD) return QSD_ERR_UNSUPPORTED;
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
    if (passes > 200) {
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
         " tile_map=" + std::to_string(L.tile_map) + " med=" + std::to_string(L.med) +
         " large=" + std::to_string(L.large) + " seg_hist=" + std::to_string(L.seg_hist) +
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
        z.ptr[0] = ctl;
        z.words[0] = kCtlWords;
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
    int h = 0, q = 0, gsub = 0, gseg = 0;
    for (const auto& g : p.groups) {
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
                const int hgrid = (int)std::max<uint64_t>(1, std::min<uint64_t>(cdiv(n, kBlock * 16), (uint64_t)device_cu_count() * 4));
                int kmodes = 0;
                for (int m = 0; m < p.r; ++m) kmodes += key.mask[m] ? 1 : 0;
                QSD_CK(timed(kHist, (double)n * p.crd_bytes * kmodes, stream,
                             [&] { return launch_hist(ha, p.r, p.crd_bytes, hgrid, stream); }));
                for (int i = 0; i < np; ++i) {
                    const Bufs dst = hop_dst(h);
                    DigitArgs da{};
                    for (int m = 0; m < p.r; ++m) {
                        da.src_crd[m] = cur.crd[m];
                        da.dst_crd[m] = const_cast<void*>(dst.crd[m]);
                    }
                    da.src_val = cur.val;
                    da.dst_val = const_cast<void*>(dst.val);
                    da.key = key;
                    da.lo = sk.passes[i].lo;
                    da.bits = sk.passes[i].bits;
                    da.n = n;
                    da.ntiles = ntiles;
                    da.seg_mode = 0;
                    da.hist = hist + (size_t)i * kBins;
                    da.status = S[q % 2];
                    da.status_next = (i + 1 < np) ? S[(q + 1) % 2] : nullptr;
                    da.tile_counter = ctl + kCtlPassCnt + q;
                    da.err = ctl + kCtlErr;
                    QSD_CK(timed(kDigit, 2.0 * n * (p.r * p.crd_bytes + p.val_bytes), stream,
                                 [&] { return launch_digit(da, p.r, p.crd_bytes, p.val_bytes, plan->items, stream); }));
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
        uint32_t* tile_map = (uint32_t*)(W + L.tile_map);
        uint32_t* bstatus = (uint32_t*)(W + L.bstatus) + (size_t)gseg * L.bstatus_words;
        uint2* med = (uint2*)(W + L.med);
        SegRec* large = (SegRec*)(W + L.large);
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
        ca.med = med;
        ca.large_ctl = large_ctl;
        ca.large = large;
        ca.tile_map = tile_map;
        ca.seg_hist = seg_hist;
        ca.hist_stride = (uint32_t)np * kBins;
        QSD_CK(timed(kClassify, 0, stream, [&] { return launch_classify(ca, n, stream); }));

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
        sa.region_seg = region_seg;
        sa.nmed = ctl + kCtlNMed;
        sa.med = med;
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
        ha.large = large;
        ha.tile_map = tile_map;
        QSD_CK(timed(kHistSeg, 0, stream, [&] { return launch_hist(ha, p.r, p.crd_bytes, device_cu_count() * 4, stream); }));
        const uint32_t max_tiles = (uint32_t)std::min<uint64_t>(L.max_tiles_large, (uint64_t)(n + T - 1) / T + n / (kSmallCap + 1) + 1);
        for (int i = 0; i < np; ++i) {
            const Bufs dst = hop_dst(h);
            DigitArgs da{};
            for (int m = 0; m < p.r; ++m) {
                da.src_crd[m] = cur.crd[m];
                da.dst_crd[m] = const_cast<void*>(dst.crd[m]);
            }
            da.src_val = cur.val;
            da.dst_val = const_cast<void*>(dst.val);
            da.key = key;
            da.lo = sk.passes[i].lo;
            da.bits = sk.passes[i].bits;
            da.n = n;
            da.ntiles = max_tiles;
            da.seg_mode = 1;
            da.hist_stride = (uint32_t)np * kBins;
            da.hist = seg_hist + (size_t)i * kBins;
            da.status = S[q % 2];
            da.status_next = (i + 1 < np) ? S[(q + 1) % 2] : nullptr;
            da.tile_counter = ctl + kCtlPassCnt + q;
            da.large_ctl = large_ctl;
            da.large = large;
            da.tile_map = tile_map;
            da.err = ctl + kCtlErr;
            QSD_CK(timed(kDigitSeg, 0, stream, [&] { return launch_digit(da, p.r, p.crd_bytes, p.val_bytes, plan->items, stream); }));
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
    if (hipMemcpyAsync(code, (char*)ws + kCtlErr * 4, 4, hipMemcpyDeviceToHost, stream) != hipSuccess)
        return QSD_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return QSD_ERR_HIP;
    return QSD_OK;
}

qsd_status qsd_csf_workspace(qsd_plan_t plan, size_t* bytes) {
    if (!plan || !bytes) return QSD_ERR_NULL;
    const uint64_t N = (uint64_t)std::max<int64_t>(plan->p.nnz, 1);
    *bytes = up(kCtlWords * 4) + up(cdiv(N, kBlock * 8) * 8 * 4);
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
    const uint64_t tiles = cdiv(std::max<uint32_t>(n, 1), kBlock * 8);
    ZeroArgs z{};
    z.ptr[0] = ctl;
    z.words[0] = kCtlWords;
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
    for (int m = 0; m < p.r; ++m) {
        ca.crd[m] = sorted_crd[m];
        ca.sigma[m] = p.out_order[m];
        ca.pos[m] = pos[m];
        ca.out_crd[m] = crd[m];
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
