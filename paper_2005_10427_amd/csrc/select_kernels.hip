// Schedule-selector kernels.  The network is tiny (7174 parameters), so every kernel keeps
// the weights it needs in LDS and gives one thread a whole row (forward, deltas) or a whole
// parameter (gradient sums over the rows, in row order, so results are reproducible).
#include "select_kernels.h"

namespace qsd {
namespace {

constexpr int kThreads = 256;

// SplitMix64's output function (Steele, Lea and Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// A workgroup barrier that also waits for this wave's LDS atomics without return value
// (the barrier alone does not wait for them on this target).
__device__ __forceinline__ void barrier_after_lds_atomics() {
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ T block_reduce(T v, T* s_tmp, bool take_max) {
    for (int o = 32; o > 0; o >>= 1) {
        const T w = __shfl_xor(v, o, 64);
        v = take_max ? (w > v ? w : v) : v + w;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) s_tmp[wave] = v;
    __syncthreads();
    T r = s_tmp[0];
    for (int w = 1; w < kThreads / 64; ++w) r = take_max ? (s_tmp[w] > r ? s_tmp[w] : r) : r + s_tmp[w];
    return r;
}

// Block b < r: the counts of mode b.  Block r + q: joint changes of mode set q.
template <typename CT>
__global__ void __launch_bounds__(kThreads) k_feat(FeatArgs a) {
    __shared__ uint32_t s_map[kFeatMapBits / 32];
    __shared__ uint32_t s_bkt[kFeatBuckets];
    __shared__ uint32_t s_tmp[kThreads / 64];
    const int tid = threadIdx.x, b = blockIdx.x;
    uint32_t change = 0;
    if (b < a.r) {
        for (int i = tid; i < (int)(kFeatMapBits / 32); i += kThreads) s_map[i] = 0;
        for (int i = tid; i < (int)kFeatBuckets; i += kThreads) s_bkt[i] = 0;
        __syncthreads();
        const CT* c = (const CT*)a.crd[b];
        // U samples per thread per round, all loads issued before any is used
        constexpr int U = 16;
        for (uint32_t k0 = tid; k0 < a.S; k0 += kThreads * U) {
            CT x[U], y[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t k = k0 + u * kThreads;
                const uint64_t j = (uint64_t)k * a.n / a.S;
                x[u] = k < a.S ? c[j] : CT(0);
                y[u] = (k < a.S && j + 1 < a.n) ? c[j + 1] : x[u];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (k0 + u * kThreads >= a.S) continue;
                const uint64_t h = mix64((uint64_t)(int64_t)x[u]);
                atomicOr(&s_map[(uint32_t)(h & 0xFFFF) >> 5], 1u << (uint32_t)(h & 31));
                atomicAdd(&s_bkt[(uint32_t)(h >> 16) & (kFeatBuckets - 1)], 1u);
                if (y[u] != x[u]) ++change;
            }
        }
        barrier_after_lds_atomics();
        uint32_t zero = 0, top = 0;
        for (int i = tid; i < (int)(kFeatMapBits / 32); i += kThreads) zero += (uint32_t)__popc(~s_map[i]);
        for (int i = tid; i < (int)kFeatBuckets; i += kThreads) top = s_bkt[i] > top ? s_bkt[i] : top;
        zero = block_reduce<uint32_t>(zero, s_tmp, false);
        top = block_reduce<uint32_t>(top, s_tmp, true);
        change = block_reduce<uint32_t>(change, s_tmp, false);
        if (tid == 0) {
            a.out[3 * b + 0] = zero;
            a.out[3 * b + 1] = top;
            a.out[3 * b + 2] = change;
        }
    } else {
        const uint32_t mask = a.mask[b - a.r];
        constexpr int U = 8;
        for (uint32_t k0 = tid; mask && k0 < a.S; k0 += kThreads * U) {
            bool d[U];
#pragma unroll
            for (int u = 0; u < U; ++u) d[u] = false;
            for (int m = 0; m < a.r; ++m) {
                if (!((mask >> m) & 1u)) continue;
                const CT* c = (const CT*)a.crd[m];
                CT x[U], y[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t k = k0 + u * kThreads;
                    const uint64_t j = (uint64_t)k * a.n / a.S;
                    const bool ok = k < a.S && j + 1 < a.n;
                    x[u] = ok ? c[j] : CT(0);
                    y[u] = ok ? c[j + 1] : CT(0);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) d[u] |= x[u] != y[u];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) change += d[u] ? 1u : 0u;
        }
        change = block_reduce<uint32_t>(change, s_tmp, false);
        if (tid == 0) {
            a.out[3 * b + 0] = change;
            a.out[3 * b + 1] = 0;
            a.out[3 * b + 2] = 0;
        }
    }
}

__global__ void __launch_bounds__(kThreads) k_mlp_fwd(const float* __restrict__ P, const float* __restrict__ X,
                                                      int n, float* H1, float* H2, float* Y) {
    __shared__ float w[kNParam];
    for (int i = threadIdx.x; i < kNParam; i += kThreads) w[i] = P[i];
    __syncthreads();
    const int row = blockIdx.x * kThreads + threadIdx.x;
    if (row >= n) return;
    float x[kNFeat], h1[kH1], h2[kH2];
#pragma unroll
    for (int i = 0; i < kNFeat; ++i) x[i] = X[(size_t)row * kNFeat + i];
#pragma unroll 4
    for (int o = 0; o < kH1; ++o) {
        float s = w[kOffB1 + o];
#pragma unroll
        for (int i = 0; i < kNFeat; ++i) s += w[kOffW1 + o * kNFeat + i] * x[i];
        h1[o] = s > 0.f ? s : 0.f;
    }
#pragma unroll 4
    for (int o = 0; o < kH2; ++o) {
        float s = w[kOffB2 + o];
#pragma unroll
        for (int i = 0; i < kH1; ++i) s += w[kOffW2 + o * kH1 + i] * h1[i];
        h2[o] = s > 0.f ? s : 0.f;
    }
#pragma unroll
    for (int o = 0; o < kNOut; ++o) {
        float s = w[kOffB3 + o];
#pragma unroll
        for (int i = 0; i < kH2; ++i) s += w[kOffW3 + o * kH2 + i] * h2[i];
        Y[(size_t)row * kNOut + o] = s;
    }
    if (H1)
#pragma unroll
        for (int i = 0; i < kH1; ++i) H1[(size_t)row * kH1 + i] = h1[i];
    if (H2)
#pragma unroll
        for (int i = 0; i < kH2; ++i) H2[(size_t)row * kH2 + i] = h2[i];
}

// The features of one request from its sampled counts (in double precision, as defined in the
// selector's header), then the forward pass (the same sums, in the same order, as k_mlp_fwd)
// and the choice: candidate 0 unless a valid candidate is predicted faster by more than the
// margin.  One wave.
__global__ void __launch_bounds__(64) k_select(SelectArgs a) {
    __shared__ float x[kNFeat];
    __shared__ float h1[kH1];
    __shared__ float h2[kH2];
    __shared__ float y[kNOut];
    const int tid = threadIdx.x;
    if (tid == 0) {
        double f[kNFeat];
        for (int i = 0; i < kNFeat; ++i) f[i] = 0.0;
        const double M = (double)kFeatMapBits;
        f[0] = a.n > 0 ? log2(a.n) / 32.0 : 0.0;
        f[1] = a.r / 8.0;
        for (int s = 0; s < 5 && s < a.r; ++s) {
            const int m = a.slot_mode[s];
            const uint32_t zero = a.counts[3 * m], top = a.counts[3 * m + 1], change = a.counts[3 * m + 2];
            const double D = zero == 0 ? M * log(M) : -M * log((double)zero / M);
            f[2 + 4 * s] = a.bits[m] / 32.0;
            f[3 + 4 * s] = a.S ? log2(1.0 + D) / 24.0 : 0.0;
            f[4 + 4 * s] = a.pairs ? (double)change / a.pairs : 0.0;
            f[5 + 4 * s] = a.S ? (double)top / a.S : 0.0;
        }
        f[22] = a.crd_bytes / 8.0;
        f[23] = a.val_bytes / 8.0;
        for (int c = 0; c < kNOut; ++c) {
            if (!a.valid[c]) continue;
            f[24 + 2 * c] = a.gp[c] / 16.0;
            f[25 + 2 * c] = a.sb[c] / 64.0;
        }
        for (int q = 0; q < kNSets; ++q)
            if (a.pairs && a.set_nonempty[q]) f[36 + q] = (double)a.counts[3 * (a.r + q)] / a.pairs;
        for (int i = 0; i < kNFeat; ++i) {
            x[i] = (float)f[i];
            a.out[8 + i] = x[i];
        }
    }
    __syncthreads();
    if (!a.params) return;
    const float* w = a.params;
    {
        float s = w[kOffB1 + tid];
        for (int i = 0; i < kNFeat; ++i) s += w[kOffW1 + tid * kNFeat + i] * x[i];
        h1[tid] = s > 0.f ? s : 0.f;
    }
    __syncthreads();
    {
        float s = w[kOffB2 + tid];
        for (int i = 0; i < kH1; ++i) s += w[kOffW2 + tid * kH1 + i] * h1[i];
        h2[tid] = s > 0.f ? s : 0.f;
    }
    __syncthreads();
    if (tid < kNOut) {
        float s = w[kOffB3 + tid];
        for (int i = 0; i < kH2; ++i) s += w[kOffW3 + tid * kH2 + i] * h2[i];
        y[tid] = s;
        a.out[1 + tid] = s;
    }
    __syncthreads();
    if (tid == 0) {
        bool in_range = true;
        for (int i = 0; i < kNFeat; ++i) in_range &= (x[i] == x[i]) && x[i] >= 0.f && x[i] <= 4.f;
        int best = 0;
        if (in_range)
            for (int c = 1; c < kNOut; ++c)
                if (a.valid[c] && y[c] < y[0] - a.margin && y[c] < y[best]) best = c;
        a.out[0] = __int_as_float(best);
    }
}

__global__ void __launch_bounds__(kThreads) k_mlp_delta(const float* __restrict__ P, const float* __restrict__ H1,
                                                        const float* __restrict__ H2, const float* __restrict__ Y,
                                                        const float* __restrict__ T, int n, float* D1, float* D2,
                                                        float* D3, float* rowloss) {
    __shared__ float w2[kH2 * kH1];
    __shared__ float w3[kNOut * kH2];
    for (int i = threadIdx.x; i < kH2 * kH1; i += kThreads) w2[i] = P[kOffW2 + i];
    for (int i = threadIdx.x; i < kNOut * kH2; i += kThreads) w3[i] = P[kOffW3 + i];
    __syncthreads();
    const int row = blockIdx.x * kThreads + threadIdx.x;
    if (row >= n) return;
    const float scale = 2.0f / ((float)n * (float)kNOut);
    float d3[kNOut], err = 0.f;
#pragma unroll
    for (int k = 0; k < kNOut; ++k) {
        const float t = T[(size_t)row * kNOut + k];
        const float e = t == t ? Y[(size_t)row * kNOut + k] - t : 0.f;  // a NaN target: no error
        err += e * e;
        d3[k] = e * scale;
        D3[(size_t)row * kNOut + k] = d3[k];
    }
    rowloss[row] = err;
    float d2[kH2];
#pragma unroll 4
    for (int o = 0; o < kH2; ++o) {
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < kNOut; ++k) s += w3[k * kH2 + o] * d3[k];
        d2[o] = H2[(size_t)row * kH2 + o] > 0.f ? s : 0.f;
        D2[(size_t)row * kH2 + o] = d2[o];
    }
#pragma unroll 4
    for (int i = 0; i < kH1; ++i) {
        float s = 0.f;
#pragma unroll
        for (int o = 0; o < kH2; ++o) s += w2[o * kH1 + i] * d2[o];
        D1[(size_t)row * kH1 + i] = H1[(size_t)row * kH1 + i] > 0.f ? s : 0.f;
    }
}

__global__ void __launch_bounds__(kThreads) k_mlp_grad(const float* __restrict__ X, const float* __restrict__ H1,
                                                       const float* __restrict__ H2, const float* __restrict__ D1,
                                                       const float* __restrict__ D2, const float* __restrict__ D3,
                                                       int n, float* G) {
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= kNParam) return;
    const float* d;
    const float* a = nullptr;
    int dw, aw, o, i = 0;
    if (p < kOffB1) {
        o = p / kNFeat, i = p % kNFeat, d = D1, dw = kH1, a = X, aw = kNFeat;
    } else if (p < kOffW2) {
        o = p - kOffB1, d = D1, dw = kH1, aw = 0;
    } else if (p < kOffB2) {
        const int q = p - kOffW2;
        o = q / kH1, i = q % kH1, d = D2, dw = kH2, a = H1, aw = kH1;
    } else if (p < kOffW3) {
        o = p - kOffB2, d = D2, dw = kH2, aw = 0;
    } else if (p < kOffB3) {
        const int q = p - kOffW3;
        o = q / kH2, i = q % kH2, d = D3, dw = kNOut, a = H2, aw = kH2;
    } else {
        o = p - kOffB3, d = D3, dw = kNOut, aw = 0;
    }
    float s = 0.f;
    if (a) {
        for (int b = 0; b < n; ++b) s += d[(size_t)b * dw + o] * a[(size_t)b * aw + i];
    } else {
        for (int b = 0; b < n; ++b) s += d[(size_t)b * dw + o];
    }
    G[p] = s;
}

__global__ void __launch_bounds__(kThreads) k_sum(const float* __restrict__ v, int n, float scale, float* out) {
    __shared__ float s_tmp[kThreads / 64];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += kThreads) s += v[i];
    s = block_reduce<float>(s, s_tmp, false);
    if (threadIdx.x == 0) *out = s * scale;
}

__global__ void __launch_bounds__(kThreads) k_adam(float* P, const float* __restrict__ G, float* M, float* V,
                                                   float lr, float b1, float b2, float eps, float c1, float c2) {
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= kNParam) return;
    const float g = G[p];
    const float m = b1 * M[p] + (1.f - b1) * g;
    const float v = b2 * V[p] + (1.f - b2) * g * g;
    M[p] = m;
    V[p] = v;
    P[p] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

__global__ void __launch_bounds__(kThreads) k_gather_rows(const float* __restrict__ X, const float* __restrict__ T,
                                                          const uint32_t* __restrict__ idx, int n, float* Xb,
                                                          float* Tb) {
    const int e = blockIdx.x * kThreads + threadIdx.x;
    constexpr int W = kNFeat + kNOut;
    if (e >= n * W) return;
    const int b = e / W, c = e % W;
    const size_t src = idx[b];
    if (c < kNFeat)
        Xb[(size_t)b * kNFeat + c] = X[src * kNFeat + c];
    else
        Tb[(size_t)b * kNOut + (c - kNFeat)] = T[src * kNOut + (c - kNFeat)];
}

unsigned blocks(long long work) { return (unsigned)((work + kThreads - 1) / kThreads); }

}  // namespace

hipError_t launch_select(const SelectArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_select, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_feat(const FeatArgs& a, int crd_bytes, hipStream_t s) {
    const dim3 grid(a.r + kNSets);
    if (crd_bytes == 8)
        hipLaunchKernelGGL(k_feat<int64_t>, grid, dim3(kThreads), 0, s, a);
    else
        hipLaunchKernelGGL(k_feat<int32_t>, grid, dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mlp_fwd(const float* P, const float* X, int n, float* H1, float* H2, float* Y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_fwd, dim3(blocks(n)), dim3(kThreads), 0, s, P, X, n, H1, H2, Y);
    return hipGetLastError();
}

hipError_t launch_mlp_delta(const float* P, const float* H1, const float* H2, const float* Y, const float* T,
                            int n, float* D1, float* D2, float* D3, float* rowloss, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_delta, dim3(blocks(n)), dim3(kThreads), 0, s, P, H1, H2, Y, T, n, D1, D2, D3, rowloss);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* X, const float* H1, const float* H2, const float* D1, const float* D2,
                           const float* D3, int n, float* G, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_grad, dim3(blocks(kNParam)), dim3(kThreads), 0, s, X, H1, H2, D1, D2, D3, n, G);
    return hipGetLastError();
}

hipError_t launch_sum(const float* v, int n, float scale, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, s, v, n, scale, out);
    return hipGetLastError();
}

hipError_t launch_adam(float* P, const float* G, float* M, float* V, float lr, float b1, float b2, float eps,
                       float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3(blocks(kNParam)), dim3(kThreads), 0, s, P, G, M, V, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const float* X, const float* T, const uint32_t* idx, int n, float* Xb, float* Tb,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_rows, dim3(blocks((long long)n * (kNFeat + kNOut))), dim3(kThreads), 0, s, X, T,
                       idx, n, Xb, Tb);
    return hipGetLastError();
}

}  // namespace qsd
