// Host-side plan: which stable partial sorts run, and how each is split into radix digits.
//
// A transposition is executed as a list of GROUPS.  A group is a run of consecutive
// PartialSort calls of QuesadillaSort (Alg. 3) that keep the same prefix (sigma_1..sigma_l):
// the calls sort sigma_k, sigma_{k-1}, ..., sigma_{l+1} one after the other, which is one
// stable sort, inside every bucket of equal prefix, by the composite key
// (sigma_{l+1}, ..., sigma_k) -- most significant first.  Doing the bucket discovery once
// per group is the paper's "discover the buckets once" improvement (Sec. 5).
//
// A group with l = 0 is a global sort.  A group with l > 0 is segmented: its buckets are
// contiguous runs of the current order (Alg. 2 needs the input sorted on the prefix).
//
// The composite key of a group is cut into radix digits (Sec. 5, "a radix smaller than the
// dimension") that are sorted least significant first.  Keys wider than 64 bits are cut
// into 64-bit sub-keys processed least significant first.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace qsd {

constexpr int kMaxR = 8;
constexpr uint32_t kKeepBuckets = 2;  // plan flag: bucketed groups stay segment sorts
constexpr int kMaxPassesPerSub = 16;

// key64 = OR over modes m of ((crd[m] >> src_lo[m]) & ((1 << width[m]) - 1)) << dst[m]
struct KeySpec {
    int32_t src_lo[kMaxR];
    int32_t width[kMaxR];
    int32_t dst[kMaxR];
    int32_t bits;
};

// digit = (key64 >> lo) & ((1 << bits) - 1)
struct PassSpec {
    int32_t lo;
    int32_t bits;
};

struct SubKey {
    KeySpec key;
    std::vector<PassSpec> passes;  // least significant first
};

struct Call {  // one PartialSort(A, prefix, mode) of Alg. 3
    std::vector<int> prefix;
    int mode;
};

struct Group {
    std::vector<int> prefix;   // kept prefix (original mode labels)
    std::vector<int> keys;     // sorted modes, most significant first
    int key_bits = 0;
    bool segmented = false;    // prefix non-empty and sorted segment by segment
    std::vector<SubKey> subs;  // least significant sub-key first
    KeySpec local_key{};       // whole key in one word, for in-LDS segment sorts
};

enum Sched { kSchedAuto = 0, kSchedMinimal = 1, kSchedTop2 = 2, kSchedLsd = 3, kSchedTopK = 16 };

struct PlanData {
    int r = 0;
    int64_t nnz = 0;
    int64_t ext[kMaxR] = {};
    int bits[kMaxR] = {};
    int crd_bytes = 4, val_bytes = 8;
    int in_order[kMaxR] = {};
    int out_order[kMaxR] = {};
    uint32_t flags = 0;
    int sched = kSchedMinimal;
    int K = 0;                 // Top-K depth (TOP2 and TOPK + K)
    int radix_bits = 8;        // digit width of global passes
    std::vector<Call> calls;   // QuesadillaSort calls (towards the Top-K target for TOP2)
    std::vector<Group> groups; // execution order
};

// Bits needed for coordinates in [0, n): 0 when n == 1.
int bits_for_extent(int64_t n);

// QuesadillaSort (Alg. 3) for an input sorted under in_order; modes are original labels.
std::vector<Call> quesadilla_calls(int r, const int* in_order, const int* out_order);

// Build the groups of a schedule.  Returns false on an unsupported combination.
bool build_plan(PlanData& p, int sched);

std::string describe(const PlanData& p);

// Digit passes of one composite key: `keys` most significant first, `bits` indexed by mode.
// Sub-keys of at most 64 bits, least significant first; digits of at most radix_bits.
std::vector<SubKey> make_subkeys(const std::vector<int>& keys, const int* bits, int radix_bits);

// The flattened key of a transposition: sigma_1..sigma_q where sigma_{q+1}..sigma_r is the
// longest tail of sigma already in input order; modes of extent 1 are dropped.
std::vector<int> flattened_key(int r, const int* in_order, const int* out_order, const int* bits);

}  // namespace qsd
