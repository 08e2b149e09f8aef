// Device kernels of the schedule selector: sampled feature counts, the features and the choice
// of one request, and the 40-64-64-6 perceptron's forward pass, backward pass and Adam update.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace qsd {

constexpr int kNFeat = 40, kH1 = 64, kH2 = 64, kNOut = 6;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kH1 * kNFeat;  // 2560
constexpr int kOffW2 = kOffB1 + kH1;           // 2624
constexpr int kOffB2 = kOffW2 + kH2 * kH1;     // 6720
constexpr int kOffW3 = kOffB2 + kH2;           // 6784
constexpr int kOffB3 = kOffW3 + kNOut * kH2;   // 7168
constexpr int kNParam = kOffB3 + kNOut;        // 7174
constexpr int kNSets = 4;                      // mode sets Q0..Q3 of the joint-change counts

constexpr uint32_t kFeatSample = 16384;
constexpr uint32_t kFeatMapBits = 1u << 16;
constexpr uint32_t kFeatBuckets = 1024;

struct FeatArgs {
    const void* crd[8];
    int32_t r;
    uint32_t S;        // sampled positions
    uint64_t n;        // nonzeros
    uint32_t mask[kNSets];  // mode sets whose joint changes are counted
    uint32_t* out;          // 3 words per mode, then 3 per mask
};

// Everything about one request that the features need besides the sampled counts.
struct SelectArgs {
    const uint32_t* counts;    // k_feat's output
    int32_t r;
    double n;                  // nonzeros
    uint32_t S, pairs;
    int32_t slot_mode[5];      // mode sigma_{s+1} of slot s
    int32_t bits[8];           // per mode
    int32_t crd_bytes, val_bytes;
    int32_t valid[kNOut];
    int32_t gp[kNOut], sb[kNOut];
    int32_t set_nonempty[kNSets];
    const float* params;       // null: features only
    float margin;
    float* out;                // [0] candidate (as int32 bits), [1..6] predictions, [8..47] features
};
constexpr int kSelectOutFloats = 8 + kNFeat;

hipError_t launch_feat(const FeatArgs& a, int crd_bytes, hipStream_t s);
hipError_t launch_select(const SelectArgs& a, hipStream_t s);
hipError_t launch_mlp_fwd(const float* P, const float* X, int n, float* H1, float* H2, float* Y, hipStream_t s);
// per-row deltas of the three layers and the row's squared error (targets that are not a
// number contribute nothing)
hipError_t launch_mlp_delta(const float* P, const float* H1, const float* H2, const float* Y, const float* T,
                            int n, float* D1, float* D2, float* D3, float* rowloss, hipStream_t s);
// parameter gradients: sums over the rows, in row order
hipError_t launch_mlp_grad(const float* X, const float* H1, const float* H2, const float* D1, const float* D2,
                           const float* D3, int n, float* G, hipStream_t s);
// loss = sum(rowloss) * scale, summed by one workgroup in a fixed order
hipError_t launch_sum(const float* v, int n, float scale, float* out, hipStream_t s);
hipError_t launch_adam(float* P, const float* G, float* M, float* V, float lr, float b1, float b2, float eps,
                       float c1, float c2, hipStream_t s);
hipError_t launch_gather_rows(const float* X, const float* T, const uint32_t* idx, int n, float* Xb, float* Tb,
                              hipStream_t s);

}  // namespace qsd
