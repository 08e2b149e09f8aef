// CSF kernels for gfx950: the pack of a sorted coordinate list into CSF (one pass, fibers of
// every level numbered with a decoupled look-back per level) and the per-level expansion of a
// CSF tensor back into coordinates.
#include "csf_kernels.h"
#include "kernels_impl.h"

namespace qsd {
namespace {

// ------------------------------------------------------------------------------ CSF pack

// CSF of n records sorted under sigma, given in level order.  Record j starts a level-d fiber
// (1-based d < R) when its prefix sigma_1..sigma_d differs from record j-1's, i.e. when the
// first level lev(j) at which its coordinates differ is below d (record 0 starts every level);
// every record is a leaf (level R).  The fiber number of a start is the number of starts of
// that level before it, so one pass over the records writes everything: crd_d at the fiber
// number, pos_{d+1} at the parent's fiber number (the first child of a new fiber is the fiber
// or leaf that starts at the same record), the leaves in place.
//
// Persistent workgroups take tiles of csf_tile<R, CT>() records in increasing order from one
// counter; all R coordinate arrays of a tile are loaded at once, the previous record of each
// lane comes from the lane below (DPP) or, for lane 0, from lane 63 of the previous item (the
// record before a wave's first item is one uniform load).  Per level the tile's starts are counted
// with ballots and numbered by a decoupled look-back over the tiles, one wave per level.
// Records per tile: as many as the registers allow, since larger tiles mean fewer look-backs
// and longer runs of contiguous stores: 8192 for r c <= 12 bytes, 4096 for r c <= 16, else
// kCsfTile (the 1e8-nonzero 3-mode int32 pack: 731, 576 and 498 us with 2048-, 4096- and
// 8192-record tiles).
template <int R, typename CT>
constexpr int csf_tile() {
    return R * (int)sizeof(CT) <= 12 ? 4 * kCsfTile : R * (int)sizeof(CT) <= 16 ? 2 * kCsfTile : kCsfTile;
}

template <int R, typename CT, typename PT>
__global__ void __launch_bounds__(256) k_csf(CsfArgs a) {
    constexpr int TILE = csf_tile<R, CT>(), ITEMS = TILE / kBlock;
    constexpr int L = R - 1;           // counted levels (0-based d = 0..L-1 is level d + 1)
    constexpr int LS = L > 0 ? L : 1;
    __shared__ uint32_t s_wsum[LS][kWaves];
    __shared__ uint32_t s_excl[LS];
    __shared__ uint32_t s_t;
    const int tid = threadIdx.x, lane = tid & 63;
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane(tid >> 6);
    for (;;) {
        if (tid == 0) s_t = atomicAdd(a.tile_counter, 1u);
        __syncthreads();
        const uint32_t t = __builtin_amdgcn_readfirstlane(s_t);
        const uint32_t start = t * TILE;
        if (start >= a.n) break;
        const uint32_t len = min((uint32_t)TILE, a.n - start);
        const uint32_t w0 = wave * 64u * ITEMS;  // this wave's first record in the tile
        const uint32_t wb = w0 + lane;
        CT x[R][ITEMS];
#pragma unroll
        for (int d = 0; d < R; ++d) load_items<CT, ITEMS>((const CT*)a.crd[d], start, len, wb, x[d]);

        // lev: first level (0-based) whose coordinate differs from the previous record's;
        // L when none of the counted levels differs
        uint32_t lev[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) lev[i] = L;
        const bool has_prev = w0 < len && start + w0 > 0;
#pragma unroll
        for (int d = L - 1; d >= 0; --d) {  // deepest first, so that the shallowest level wins
            CT carry = has_prev ? ((const CT*)a.crd[d])[start + w0 - 1] : CT(0);
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const CT below = lane_below(x[d][i]);
                const CT prv = lane == 0 ? carry : below;
                carry = lane63(x[d][i]);
                if (x[d][i] != prv) lev[i] = (uint32_t)d;
            }
        }
        if (start + wb == 0) lev[0] = 0;  // record 0 starts every level

        // starts per level in this wave
        uint32_t wcnt[LS];
#pragma unroll
        for (int d = 0; d < LS; ++d) wcnt[d] = 0;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const bool ok = wb + i * 64 < len;
#pragma unroll
            for (int d = 0; d < L; ++d) wcnt[d] += (uint32_t)__popcll(ballot(ok && lev[i] <= (uint32_t)d));
        }
        if (lane == 0) {
#pragma unroll
            for (int d = 0; d < L; ++d) s_wsum[d][wave] = wcnt[d];
        }
        __syncthreads();
        // starts before this tile: one wave per level, 64 predecessors per round trip
        for (uint32_t d = wave; d < (uint32_t)L; d += kWaves) {
            uint32_t tot = 0;
            for (int w = 0; w < kWaves; ++w) tot += s_wsum[d][w];
            uint32_t* st = a.status + (size_t)t * 8 + d;
            uint32_t excl = 0;
            if (t == 0) {
                if (lane == 0) st_status(st, kFlagP | tot);
            } else {
                if (lane == 0) st_status(st, kFlagA | tot);
                excl = wave_look_back(a.status, t, 8, d, 0, a.err);
                if (lane == 0) st_status(st, kFlagP | (excl + tot));
            }
            if (lane == 0) s_excl[d] = excl;
        }
        __syncthreads();
        uint32_t base[LS];  // fiber number of this wave's next start, per level
#pragma unroll
        for (int d = 0; d < L; ++d) {
            uint32_t b = s_excl[d];
            for (uint32_t w = 0; w < wave; ++w) b += s_wsum[d][w];
            base[d] = b;
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t off = wb + i * 64;
            const bool ok = off < len;
            const uint32_t e = start + off;
            const uint32_t lv = lev[i];
            uint32_t fid[LS];
#pragma unroll
            for (int d = 0; d < L; ++d) {
                const uint64_t m = ballot(ok && lv <= (uint32_t)d);
                fid[d] = base[d] + lanes_below(m);
                base[d] += (uint32_t)__popcll(m);
            }
            if (ok) {
                ((CT*)a.out_crd[R - 1])[e] = x[R - 1][i];
#pragma unroll
                for (int d = 0; d < L; ++d)
                    if (lv <= (uint32_t)d) ((CT*)a.out_crd[d])[fid[d]] = x[d][i];
                if (e == 0) ((PT*)a.pos[0])[0] = 0;
                // a new fiber at (0-based) level d - 1 records its first child at level d
#pragma unroll
                for (int d = 1; d < R; ++d)
                    if (lv <= (uint32_t)(d - 1)) ((PT*)a.pos[d])[fid[d - 1]] = (PT)(d == R - 1 ? e : fid[d < L ? d : 0]);
            }
        }
        if (tid == 0 && start + len == a.n) {
            // F_d of every level, and the closing entries pos_d[F_{d-1}] = F_d
            uint64_t F[R + 1];
            F[0] = 1;
#pragma unroll
            for (int d = 0; d < L; ++d) F[d + 1] = s_excl[d] + s_wsum[d][0] + s_wsum[d][1] + s_wsum[d][2] + s_wsum[d][3];
            F[R] = a.n;
#pragma unroll
            for (int d = 0; d <= R; ++d) a.fiber_counts[d] = (int64_t)F[d];
#pragma unroll
            for (int d = 1; d <= R; ++d) ((PT*)a.pos[d - 1])[F[d - 1]] = (PT)F[d];
        }
        __syncthreads();  // s_wsum / s_excl / s_t are rewritten by the next tile
    }
}

// ------------------------------------------------------------------------------ CSF expansion

// F_d of a CSF tensor: F_0 = 1 and F_e = pos[e-1][F_{e-1}].
template <typename PT>
__device__ __forceinline__ uint64_t csf_fibers(const CsfExpandArgs& a, int d) {
    uint64_t f = 1;
    for (int e = 1; e <= d; ++e) f = (uint64_t)((const PT*)a.pos[e - 1])[f];
    return f;
}

// Every level-d fiber marks its first leaf: following the first child down from level d to the
// leaves, x <- pos[e][x] for e = d .. r-1.  Leaf indices are clamped into [0, n) so that a
// malformed tensor cannot write outside the flags.
template <typename PT>
__global__ void __launch_bounds__(256) k_csf_mark(CsfExpandArgs a) {
    uint64_t Fe[9];  // fiber counts of every level, each index below clamped to its array
    Fe[0] = 1;
    for (int e = 1; e <= a.r; ++e) Fe[e] = (uint64_t)((const PT*)a.pos[e - 1])[Fe[e - 1]];
    const uint64_t F = Fe[a.level];
    for (uint64_t f = blockIdx.x * (uint64_t)kBlock + threadIdx.x; f < F; f += gridDim.x * (uint64_t)kBlock) {
        uint64_t x = f;
        for (int e = a.level; e < a.r; ++e) x = (uint64_t)((const PT*)a.pos[e])[min(x, Fe[e])];
        if (x < a.n) a.flags[x] = 1;
    }
}

// The level-d coordinate of every leaf: its level-d ancestor is the number of fibers whose first
// leaf is at or before it, minus one (an inclusive count of the flags, tiles chained by a
// one-word decoupled look-back), and the coordinate is that fiber's entry of crd[d-1].
template <typename CT>
__global__ void __launch_bounds__(256) k_csf_expand(CsfExpandArgs a) {
    constexpr int ITEMS = kBoundTile / kBlock;
    __shared__ uint32_t s_wsum[kWaves];
    __shared__ uint32_t s_geo[2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_geo[0] = atomicAdd(a.tile_counter, 1u);
    __syncthreads();
    const uint32_t t = s_geo[0];
    const uint32_t start = t * kBoundTile;
    if (start >= a.n) return;
    const uint32_t len = min((uint32_t)kBoundTile, a.n - start);
    const uint32_t wb = (uint32_t)wave * 64u * ITEMS + lane;
    uint64_t flags[ITEMS];
    uint32_t wcount = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t off = wb + i * 64;
        flags[i] = ballot(off < len && a.flags[start + off] != 0);
        wcount += (uint32_t)__popcll(flags[i]);
    }
    if (lane == 0) s_wsum[wave] = wcount;
    __syncthreads();
    if (wave == 0) {
        uint32_t tot = 0;
        for (int w = 0; w < kWaves; ++w) tot += s_wsum[w];
        uint32_t* st = a.status + t;
        if (lane == 0) st_status(st, (t == 0 ? kFlagP : kFlagA) | tot);
        const uint32_t excl = t == 0 ? 0u : wave_look_back(a.status, t, 1, 0, 0, a.err);
        if (lane == 0) {
            if (t != 0) st_status(st, kFlagP | (excl + tot));
            s_geo[1] = excl;
        }
    }
    __syncthreads();
    uint32_t pos = s_geo[1];
    for (int w = 0; w < wave; ++w) pos += s_wsum[w];
    const CT* crd = (const CT*)a.crd[a.level - 1];
    const uint64_t F = csf_fibers<CT>(a, a.level);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint64_t f = flags[i];
        const uint32_t off = wb + i * 64;
        const uint32_t incl = pos + lanes_below(f) + (uint32_t)((f >> lane) & 1ull);  // flags at or before
        if (off < len) {
            const uint64_t anc = incl ? min((uint64_t)incl - 1, F ? F - 1 : 0) : 0;
            ((CT*)a.out)[start + off] = crd[anc];
        }
        pos += (uint32_t)__popcll(f);
    }
}

template <typename CT, typename PT, int R>
hipError_t csf_r(const CsfArgs& a, hipStream_t s) {
    static int resident = 0;  // persistent grid: the workgroups that fit at once
    if (!resident) resident = resident_blocks(k_csf<R, CT, PT>);
    const uint32_t tiles = (a.n + csf_tile<R, CT>() - 1) / csf_tile<R, CT>();
    hipLaunchKernelGGL((k_csf<R, CT, PT>), dim3(std::min<uint32_t>(tiles, (uint32_t)resident)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <typename CT, typename PT>
hipError_t csf_c(const CsfArgs& a, hipStream_t s) {
    switch (a.r) {
        case 1: return csf_r<CT, PT, 1>(a, s);
        case 2: return csf_r<CT, PT, 2>(a, s);
        case 3: return csf_r<CT, PT, 3>(a, s);
        case 4: return csf_r<CT, PT, 4>(a, s);
        case 5: return csf_r<CT, PT, 5>(a, s);
        case 6: return csf_r<CT, PT, 6>(a, s);
        case 7: return csf_r<CT, PT, 7>(a, s);
        case 8: return csf_r<CT, PT, 8>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_csf_mark(const CsfExpandArgs& a, int crd_bytes, hipStream_t s) {
    const uint32_t grid = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>((a.n + kBlock - 1) / kBlock, (uint64_t)device_cu_count() * 8));
    if (crd_bytes == 8)
        hipLaunchKernelGGL(k_csf_mark<uint64_t>, dim3(grid), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_csf_mark<uint32_t>, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_csf_expand(const CsfExpandArgs& a, int crd_bytes, hipStream_t s) {
    const uint32_t grid = (a.n + kBoundTile - 1) / kBoundTile;
    if (!grid) return hipSuccess;
    if (crd_bytes == 8)
        hipLaunchKernelGGL(k_csf_expand<uint64_t>, dim3(grid), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_csf_expand<uint32_t>, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_csf(const CsfArgs& a, int crd_bytes, hipStream_t s) {
    if (!a.n) return hipSuccess;
    return crd_bytes == 8 ? csf_c<uint64_t, int64_t>(a, s) : csf_c<uint32_t, int32_t>(a, s);
}

}  // namespace qsd
