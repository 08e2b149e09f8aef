// Host-only exercise of the planner for sanitizer builds (AddressSanitizer and
// UndefinedBehaviorSanitizer): every pair of input and output orders for r = 1..5 and a sample
// for r = 6..8, random extents (some of extent 1, some beyond 2^32), every schedule, with and
// without kept buckets.  Checks structural invariants of each plan; prints "ok" when all hold.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <random>
#include <vector>

#include "plan.h"

using namespace qsd;

static int failures = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            if (++failures < 20) std::printf("check failed: %s (line %d)\n", #c, __LINE__); \
        }                                                                         \
    } while (0)

static void check_plan(const PlanData& p) {
    std::vector<int> seen_keys;
    for (const Group& g : p.groups) {
        CHECK(!g.keys.empty());
        for (int m : g.prefix) CHECK(m >= 0 && m < p.r);
        for (int m : g.keys) CHECK(m >= 0 && m < p.r);
        // a group never sorts a mode it keeps
        for (int m : g.keys) CHECK(std::find(g.prefix.begin(), g.prefix.end(), m) == g.prefix.end());
        CHECK(!g.segmented || !g.prefix.empty());
        int bits = 0;
        for (int m : g.keys) bits += p.bits[m];
        CHECK(g.key_bits == bits);
        // the sub-keys' digits cover the key exactly once
        int covered = 0;
        for (const SubKey& s : g.subs) {
            int sb = 0, lo = 0;
            for (const PassSpec& ps : s.passes) {
                CHECK(ps.lo == lo);
                CHECK(ps.bits >= 1 && ps.bits <= 8);
                lo += ps.bits;
                sb += ps.bits;
            }
            CHECK(sb == s.key.bits);
            CHECK(s.key.bits <= 64);
            covered += sb;
        }
        CHECK(covered == bits);
    }
    const std::string d = describe(p);
    CHECK(!d.empty());
}

int main() {
    std::mt19937_64 rng(20050427);
    long plans = 0;
    for (int r = 1; r <= 8; ++r) {
        std::vector<int> tau(r), sigma(r);
        std::iota(tau.begin(), tau.end(), 0);
        std::vector<std::pair<std::vector<int>, std::vector<int>>> pairs;
        if (r <= 5) {
            std::vector<int> a = tau;
            do {
                std::vector<int> b = tau;
                do pairs.push_back({a, b});
                while (std::next_permutation(b.begin(), b.end()));
            } while (std::next_permutation(a.begin(), a.end()));
        } else {
            for (int k = 0; k < 200; ++k) {
                std::vector<int> a = tau, b = tau;
                std::shuffle(a.begin(), a.end(), rng);
                std::shuffle(b.begin(), b.end(), rng);
                pairs.push_back({a, b});
            }
        }
        for (const auto& pr : pairs) {
            for (int trial = 0; trial < 2; ++trial) {
                PlanData base;
                base.r = r;
                base.nnz = 1 + (int64_t)(rng() % 100000);
                for (int m = 0; m < r; ++m) {
                    const int kind = (int)(rng() % 8);
                    base.ext[m] = kind == 0 ? 1 : kind == 1 ? ((int64_t)1 << 33) + (int64_t)(rng() % 1000)
                                                            : 1 + (int64_t)(rng() % 3000000);
                    base.bits[m] = bits_for_extent(base.ext[m]);
                    base.in_order[m] = pr.first[m];
                    base.out_order[m] = pr.second[m];
                }
                std::vector<int> scheds = {kSchedMinimal, kSchedTop2, kSchedLsd};
                for (int K = 1; K < r; ++K) scheds.push_back(kSchedTopK + K);
                for (int sched : scheds)
                    for (uint32_t flags : {0u, kKeepBuckets}) {
                        PlanData p = base;
                        p.flags = flags;
                        if (!build_plan(p, sched)) continue;
                        check_plan(p);
                        ++plans;
                    }
                const std::vector<int> fk = flattened_key(r, base.in_order, base.out_order, base.bits);
                for (int m : fk) CHECK(m >= 0 && m < r && base.bits[m] > 0);
                const std::vector<Call> calls = quesadilla_calls(r, base.in_order, base.out_order);
                CHECK((int)calls.size() <= r);
            }
        }
    }
    std::printf("%ld plans, %d failures\n", plans, failures);
    if (failures == 0) std::printf("ok\n");
    return failures == 0 ? 0 : 1;
}
