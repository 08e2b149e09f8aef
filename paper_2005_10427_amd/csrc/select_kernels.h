// Device kernels of the schedule selector: sampled feature counts and the 32-64-64-3
// perceptron's forward pass, backward pass and Adam update.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace qsd {

constexpr int kNFeat = 32, kH1 = 64, kH2 = 64, kNOut = 3;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kH1 * kNFeat;  // 2048
constexpr int kOffW2 = kOffB1 + kH1;           // 2112
constexpr int kOffB2 = kOffW2 + kH2 * kH1;     // 6208
constexpr int kOffW3 = kOffB2 + kH2;           // 6272
constexpr int kOffB3 = kOffW3 + kNOut * kH2;   // 6464
constexpr int kNParam = kOffB3 + kNOut;        // 6467

constexpr uint32_t kFeatSample = 16384;
constexpr uint32_t kFeatMapBits = 1u << 16;
constexpr uint32_t kFeatBuckets = 1024;

struct FeatArgs {
    const void* crd[8];
    int32_t r;
    uint32_t S;        // sampled positions
    uint64_t n;        // nonzeros
    uint32_t mask[2];  // mode sets whose joint changes are counted
    uint32_t* out;     // 3 words per mode, then 3 per mask
};

hipError_t launch_feat(const FeatArgs& a, int crd_bytes, hipStream_t s);
hipError_t launch_mlp_fwd(const float* P, const float* X, int n, float* H1, float* H2, float* Y, hipStream_t s);
// per-row deltas of the three layers and the row's squared error
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
