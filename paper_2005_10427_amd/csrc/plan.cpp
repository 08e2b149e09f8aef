// Host planner: QuesadillaSort (Alg. 3), Top-K-sadilla (Sec. 3.6), full LSD radix (Sec. 3),
// grouping of calls that keep the same prefix, and digit splitting.
#include "plan.h"

#include <algorithm>
#include <cstdio>
#include <cstring>

namespace qsd {

int bits_for_extent(int64_t n) {
    int b = 0;
    uint64_t v = (n > 1) ? (uint64_t)(n - 1) : 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

namespace {

struct RawGroup {
    std::vector<int> prefix;
    std::vector<int> keys;
};

// Alg. 3 on `target` for an input sorted under `in_order`.  The paper states it for the
// simple input order; relabelling every mode by its position in the input order reduces the
// general case to that one (Sec. 2.2).  The scan loop's test -- f(sigma, sigma_{k+1}) not a
// subset of the input's f(., sigma_{k+1}) -- holds exactly when some later mode of the target
// precedes sigma_{k+1} in the input.
void alg3(int r, const int* in_order, const int* target, std::vector<Call>* calls,
          std::vector<RawGroup>* groups) {
    int pos[kMaxR], lab[kMaxR];
    for (int i = 0; i < r; ++i) pos[in_order[i]] = i;
    for (int i = 0; i < r; ++i) lab[i] = pos[target[i]];
    auto must_move = [&](int i) {
        for (int j = i + 1; j < r; ++j)
            if (lab[j] < lab[i]) return true;
        return false;
    };
    int l = 0;
    while (l < r) {
        int k = l;
        while (k + 1 < r && must_move(k)) ++k;  // target[k] is sigma_{k+1}
        const int l_next = k + 1;
        if (k > l) {
            RawGroup g;
            g.prefix.assign(target, target + l);
            g.keys.assign(target + l, target + k);  // sigma_{l+1} .. sigma_k
            if (groups) groups->push_back(g);
        }
        for (int kk = k; kk > l; --kk) {  // PartialSort(A, (sigma_1..sigma_l), sigma_kk)
            Call c;
            c.prefix.assign(target, target + l);
            c.mode = target[kk - 1];
            if (calls) calls->push_back(c);
        }
        l = l_next;
    }
}

int split_keys(const std::vector<int>& keys, const int* bits, int radix_bits, std::vector<SubKey>* subs) {
    // composite layout: the least significant key mode sits at bit 0
    int lo[kMaxR] = {}, w[kMaxR] = {};
    int shift = 0;
    for (int i = (int)keys.size() - 1; i >= 0; --i) {
        const int m = keys[i];
        lo[m] = shift;
        w[m] = bits[m];
        shift += bits[m];
    }
    subs->clear();
    for (int c0 = 0; c0 < shift; c0 += 64) {
        const int c1 = std::min(shift, c0 + 64);
        SubKey sk{};
        std::memset(&sk.key, 0, sizeof(sk.key));
        for (int m : keys) {
            const int a = lo[m], b = lo[m] + w[m];
            const int s = std::max(a, c0), e = std::min(b, c1);
            if (e > s) {
                sk.key.src_lo[m] = s - a;
                sk.key.width[m] = e - s;
                sk.key.dst[m] = s - c0;
            }
        }
        sk.key.bits = c1 - c0;
        const int B = c1 - c0;
        const int D = (B + radix_bits - 1) / radix_bits;
        const int base = B / D, extra = B % D;
        int at = 0;
        for (int d = 0; d < D; ++d) {
            const int wd = base + (d < extra ? 1 : 0);
            sk.passes.push_back(PassSpec{at, wd});
            at += wd;
        }
        subs->push_back(sk);
    }
    return shift;
}

void split_digits(Group& g, const PlanData& p) {
    g.key_bits = split_keys(g.keys, p.bits, p.radix_bits, &g.subs);
    if (!g.subs.empty()) g.local_key = g.subs[0].key;
}

bool make_group(PlanData& p, RawGroup raw, std::vector<Group>* out) {
    Group g;
    g.prefix = raw.prefix;
    for (int m : raw.keys)
        if (p.bits[m] > 0) g.keys.push_back(m);  // a mode of extent 1 never reorders anything
    if (g.keys.empty()) return true;
    g.segmented = !g.prefix.empty();
    split_digits(g, p);
    // In-LDS segment sorts put a 12-bit segment number above the key in one 64-bit word.
    // Wider keys are sorted globally with the prefix as the most significant part instead:
    // the input is sorted on the prefix, so a stable sort on (prefix, keys) keeps buckets.
    bool flatten = g.segmented && g.key_bits > 52;
    if (g.segmented && !flatten && !(p.flags & kKeepBuckets)) {
        // Bucket discovery plus segment sorts against one global sort on (prefix, keys) with
        // packed records: prefer the latter when every nonzero packs into 64 bits and the
        // prefix adds at most one digit pass (a cost rule in the spirit of Sec. 5).  Two extra
        // passes cost more than the segment sorts: (0,2,1) of the 1e8-nonzero 3-mode tensor
        // ran in 4.34 ms flattened (5 passes) and 3.01 ms bucketed, (0,2,1,3) of the
        // 2e8-nonzero 4-mode tensor in 6.24 and 3.97 ms.
        int total = 0, prefix_bits = 0;
        for (int m = 0; m < p.r; ++m) total += p.bits[m];
        for (int m : g.prefix) prefix_bits += p.bits[m];
        const int flat_bits = prefix_bits + g.key_bits;
        const int d_key = (g.key_bits + p.radix_bits - 1) / p.radix_bits;
        const int d_flat = (flat_bits + p.radix_bits - 1) / p.radix_bits;
        flatten = total <= 64 && flat_bits <= 64 && d_flat <= d_key + 1;
    }
    if (flatten) {
        std::vector<int> flat;
        for (int m : g.prefix)
            if (p.bits[m] > 0) flat.push_back(m);
        flat.insert(flat.end(), g.keys.begin(), g.keys.end());
        g.prefix.clear();
        g.keys = flat;
        g.segmented = false;
        split_digits(g, p);
    }
    for (auto& s : g.subs)
        if ((int)s.passes.size() > kMaxPassesPerSub) return false;
    out->push_back(g);
    return true;
}

}  // namespace

std::vector<SubKey> make_subkeys(const std::vector<int>& keys, const int* bits, int radix_bits) {
    std::vector<SubKey> subs;
    split_keys(keys, bits, radix_bits, &subs);
    return subs;
}

std::vector<int> flattened_key(int r, const int* in_order, const int* out_order, const int* bits) {
    int pos[kMaxR];
    for (int i = 0; i < r; ++i) pos[in_order[i]] = i;
    int q = r - 1;  // first mode of the in-order tail; a single last mode always is
    while (q - 1 >= 0 && pos[out_order[q - 1]] < pos[out_order[q]]) --q;
    if (r == 0) q = 0;
    std::vector<int> keys;
    for (int i = 0; i < q; ++i)
        if (bits[out_order[i]] > 0) keys.push_back(out_order[i]);
    return keys;
}

std::vector<Call> quesadilla_calls(int r, const int* in_order, const int* out_order) {
    std::vector<Call> calls;
    alg3(r, in_order, out_order, &calls, nullptr);
    return calls;
}

// Top-K-sadilla (Sec. 3.6): QuesadillaSort towards sigma^K = (sigma_1..sigma_K, the other modes
// in input order), then every bucket of equal (sigma_1..sigma_K) sorted completely.
void topk(PlanData& p, int K, std::vector<RawGroup>* raw) {
    const int r = p.r;
    p.K = K;
    int target[kMaxR];
    int n = 0;
    for (int i = 0; i < K; ++i) target[n++] = p.out_order[i];
    for (int i = 0; i < r; ++i) {
        const int m = p.in_order[i];
        bool head = false;
        for (int j = 0; j < K; ++j) head |= (p.out_order[j] == m);
        if (!head) target[n++] = m;
    }
    alg3(r, p.in_order, target, &p.calls, raw);
    // Inside a bucket of equal (sigma_1..sigma_K) the other modes are in input order, so a
    // stable sort on sigma_{K+1}..sigma_q finishes the bucket, where sigma_{q+1}..sigma_r is the
    // longest tail that is already in input order.
    int pos[kMaxR];
    for (int i = 0; i < r; ++i) pos[p.in_order[i]] = i;
    int q = r - 1;  // first mode of the in-order tail; a single last mode always is
    while (q - 1 >= K && pos[p.out_order[q - 1]] < pos[p.out_order[q]]) --q;
    RawGroup tail;
    tail.prefix.assign(p.out_order, p.out_order + K);
    tail.keys.assign(p.out_order + K, p.out_order + q);
    if (!tail.keys.empty()) raw->push_back(tail);
}

bool build_plan(PlanData& p, int sched) {
    if (sched == kSchedAuto) sched = kSchedMinimal;
    p.sched = sched;
    p.calls.clear();
    p.groups.clear();
    std::vector<RawGroup> raw;
    const int r = p.r;
    if (sched == kSchedMinimal) {
        p.K = 0;
        alg3(r, p.in_order, p.out_order, &p.calls, &raw);
    } else if (sched == kSchedTop2) {
        topk(p, std::max(0, std::min(2, r - 2)), &raw);
    } else if (sched > kSchedTopK && sched < kSchedTopK + r) {
        topk(p, sched - kSchedTopK, &raw);
    } else if (sched == kSchedLsd) {
        p.K = 0;
        RawGroup g;
        g.keys.assign(p.out_order, p.out_order + r);
        for (int i = r - 1; i >= 0; --i) p.calls.push_back(Call{{}, p.out_order[i]});
        raw.push_back(g);
    } else {
        return false;
    }
    for (auto& g : raw)
        if (!make_group(p, g, &p.groups)) return false;
    return true;
}

static std::string join(const std::vector<int>& v) {
    std::string s;
    for (size_t i = 0; i < v.size(); ++i) {
        if (i) s += ",";
        s += std::to_string(v[i]);
    }
    return s;
}

std::string describe(const PlanData& p) {
    static const char* names[] = {"AUTO", "MINIMAL", "TOP2", "LSD"};
    const std::string name = p.sched >= kSchedTopK ? "TOPK" : names[p.sched];
    std::string s = "sched=" + name + " K=" + std::to_string(p.K) + "\n";
    for (const auto& c : p.calls)
        s += "call prefix=" + join(c.prefix) + " mode=" + std::to_string(c.mode) + "\n";
    for (const auto& g : p.groups) {
        int passes = 0;
        for (const auto& sk : g.subs) passes += (int)sk.passes.size();
        s += "group prefix=" + join(g.prefix) + " keys=" + join(g.keys) +
             " bits=" + std::to_string(g.key_bits) + " passes=" + std::to_string(passes) +
             (g.segmented ? " segmented=1" : " segmented=0") + "\n";
    }
    return s;
}

}  // namespace qsd
