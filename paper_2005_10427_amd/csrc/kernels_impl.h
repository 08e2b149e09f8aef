// HIP kernels for gfx950 (CDNA4, wave64).
//
// The digit pass is a stable counting-sort pass (Alg. 1: count, prefix sum, move in input
// order) made single-pass on the GPU:
//   * the global count of every digit comes from an upfront histogram kernel (the count
//     loop, done once for all digit passes of a key since counts do not depend on order);
//   * each workgroup ranks a tile of records by digit with wave64 ballots (stable within the
//     tile), publishes its per-digit counts and reads its predecessors' counts with a
//     decoupled look-back (Merrill & Garland, 2016) -- the "private count arrays merged in
//     order" of Sec. 3.1, merged in (digit-major, tile-minor) order;
//   * the tile is reordered through LDS so that every digit's run is written contiguously,
//     and whole records (all coordinates and the value bits) move, so no final gather runs.
// Bucketed groups (Alg. 2) are sorted segment by segment (the paper's decomposition along
// bucket boundaries, Sec. 3.2): short segments entirely in LDS, long ones by the same digit
// pass restricted to each segment.
#pragma once
#include "kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

namespace qsd {
namespace {

constexpr uint32_t kFlagA = 1u << 30;  // aggregate of this tile only
constexpr uint32_t kFlagP = 2u << 30;  // inclusive prefix up to this tile
constexpr uint32_t kCntMask = (1u << 30) - 1;
constexpr uint32_t kSpinLimit = 1u << 20;
// Word 3 of a raw (unformatted, unswizzled) buffer resource on gfx9-family targets.
constexpr int kBufferWord3 = 0x00020000;
constexpr int kHistU = 8;   // records per thread per round of a histogram (loads in flight)
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ uint32_t ld_status(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
// Wait until this wave's LDS operations have completed (lgkmcnt(0); vmcnt and expcnt left at
// their maximum).  The barrier of __syncthreads() does not wait for LDS atomics that return
// nothing on this target, so a flush of LDS-atomic counters must wait explicitly first.
__device__ __forceinline__ void lds_wait() { __builtin_amdgcn_s_waitcnt(0xC07F); }
__device__ __forceinline__ void sync_after_lds_atomics() {
    lds_wait();
    __syncthreads();
}
// The value of the lane below (lane 0 gets ~0): a whole-wave DPP shift, no LDS round trip.
__device__ __forceinline__ uint32_t from_lane_below(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)x, 0x138 /* wave_shr:1 */, 0xF, 0xF, false);
}
// The value of the lane below, for 32- or 64-bit values (lane 0 receives ~0).
template <typename CT>
__device__ __forceinline__ CT lane_below(CT x) {
    if constexpr (sizeof(CT) == 8) {
        const uint64_t lo = from_lane_below((uint32_t)x), hi = from_lane_below((uint32_t)((uint64_t)x >> 32));
        return (CT)((hi << 32) | lo);
    } else {
        return (CT)from_lane_below((uint32_t)x);
    }
}
// The value held by lane 63 (uniform).
template <typename CT>
__device__ __forceinline__ CT lane63(CT x) {
    if constexpr (sizeof(CT) == 8) {
        const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, 63);
        const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)x >> 32), 63);
        return (CT)((hi << 32) | lo);
    } else {
        return (CT)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, 63);
    }
}

// Values that are the same in every lane, moved into scalar registers.
__device__ __forceinline__ uint32_t uni32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    return ((uint64_t)uni32((uint32_t)(v >> 32)) << 32) | uni32((uint32_t)v);
}
template <typename P>
__device__ __forceinline__ P* uni_ptr(P* p) {
    return reinterpret_cast<P*>(uni64(reinterpret_cast<uint64_t>(p)));
}
// One count per lane into s_h[slot].  A wave whose lanes all hold one slot (sorted digits)
// adds 64 once.  Otherwise consecutive lanes holding the same slot (long runs in sorted
// inputs) are added once, from the run's first lane, by the run's length, instead of one
// conflicting atomic per lane; when at least half of the lanes start a run (the usual case for
// unsorted digits, where the few repeated slots cost the LDS little) each lane adds 1
// directly, skipping the run lengths.  Every lane is counted once.
__device__ __forceinline__ void count_slot(uint32_t* s_h, uint32_t slot, int lane) {
    const uint32_t s0 = uni32(slot);
    if (ballot(slot != s0) == 0) {  // one slot in the whole wave (sorted digits): one add of 64
        if (lane == 0) atomicAdd(&s_h[s0], 64u);
        return;
    }
    // lane 0 always starts a run: the value "below" it is ~0, which no slot equals
    const uint64_t heads = ballot(from_lane_below(slot) != slot);
    if (__popcll(heads) >= 32) {
        atomicAdd(&s_h[slot], 1u);
    } else if ((heads >> lane) & 1ull) {
        const uint64_t after = (heads >> 1) >> lane;  // heads above this lane
        const uint32_t run = after ? (uint32_t)__builtin_ctzll(after) + 1u : 64u - lane;
        atomicAdd(&s_h[slot], run);
    }
}
// number of set bits of m in lanes below this one
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread over the block; s_tmp holds kWaves words.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* s_tmp, uint32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(v, lane);
    if (lane == 63) s_tmp[wave] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t s = s_tmp[w];
        before += (w < wave) ? s : 0;
        tot += s;
    }
    __syncthreads();
    if (total) *total = tot;
    return before + inc - v;
}

template <typename CT>
__device__ __forceinline__ uint64_t compose_key(const CT (&c)[8], const DevKey& k, int r) {
    uint64_t key = 0;
    for (int m = 0; m < r; ++m)
        if (k.mask[m]) key |= (((uint64_t)c[m] >> k.src_lo[m]) & k.mask[m]) << k.dst[m];
    return key;
}

// ------------------------------------------------------------------------------ utility

__global__ void __launch_bounds__(256) k_zero(ZeroArgs a) {
    if (a.ctl) {
        for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < (uint32_t)kCtlWords; i += gridDim.x * 256u)
            if (i != kCtlErr && i != kCtlMagic) a.ctl[i] = 0;
        if (blockIdx.x == 0 && threadIdx.x == 0 && a.ctl[kCtlMagic] != kCtlStickyMagic) {
            a.ctl[kCtlErr] = 0;
            a.ctl[kCtlMagic] = kCtlStickyMagic;
        }
    }
    for (int r = 0; r < 4; ++r) {
        uint32_t* p = a.ptr[r];
        if (!p) continue;
        for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < a.words[r]; i += gridDim.x * 256ull)
            p[i] = 0;
    }
}

// Streaming copy: four independent 16-byte loads per thread in flight, then four stores, with
// the non-temporal cache policy (the data is touched once); the bytes past the last whole
// 16-byte word one at a time.  16 workgroups per CU: 5.8 TB/s (read + write) on 1.6 GB.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                              uint64_t n16, const uint8_t* __restrict__ sb,
                                              uint8_t* __restrict__ db, uint64_t bytes) {
    constexpr int U = 4;
    const uint64_t stride = (uint64_t)gridDim.x * 256 * U;
    for (uint64_t base = blockIdx.x * 256ull * U + threadIdx.x; base < n16; base += stride) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = base + u * 256ull;
            if (i < n16) v[u] = __builtin_nontemporal_load(&src[i]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = base + u * 256ull;
            if (i < n16) __builtin_nontemporal_store(v[u], &dst[i]);
        }
    }
    for (uint64_t i = n16 * 16 + blockIdx.x * 256ull + threadIdx.x; i < bytes; i += gridDim.x * 256ull)
        db[i] = sb[i];
}

// ------------------------------------------------------------------------------ histograms

// Counts of every digit of every pass of one key, over all records (global) or per large
// segment.  Also clears the look-back words of the key's first digit pass.
// At most 64 registers (eight waves per SIMD): the kernel waits on its loads, and more waves in
// flight hide them better (plain workload: 227 -> 219 us per launch).
template <int R, typename CT>
__global__ void __launch_bounds__(256, 8) k_hist(HistArgs a) {
    constexpr int U = kHistU;
    constexpr int MAXP = 16;
    __shared__ uint32_t s_h[MAXP * kBins + kBins];  // + one spare block for out-of-range items
    const int tid = threadIdx.x, lane = tid & 63;
    const int npass = a.npass;
    const int words = npass * kBins;
    for (int i = tid; i < words; i += kBlock) s_h[i] = 0;
    const uint32_t spare = MAXP * kBins;  // items past the end count into the spare block
    uint32_t kw[R];  // width of each key field
#pragma unroll
    for (int m = 0; m < R; ++m) kw[m] = a.key.mask[m] ? 64u - (uint32_t)__builtin_clzll(a.key.mask[m]) : 0u;

    // count the digits of records [lo, hi) with U loads per key mode in flight.  The key is
    // built in two 32-bit halves; a pass's digit is one funnel shift (or one shift above bit
    // 31) and one and-or that also adds the pass's block offset.  Whether a pass's digits come
    // in runs is decided once per round from its first record (a wave where at least half of
    // the lanes start a run counts every lane directly); both ways count every lane once.
    // One round: U records per thread.  FULL rounds (every record below hi, all but the last)
    // need no range checks.
    auto round = [&](uint32_t base, uint32_t hi, auto full) __attribute__((always_inline)) {
        constexpr bool FULL = decltype(full)::value;
        uint32_t klo[U], khi[U];
#pragma unroll
        for (int u = 0; u < U; ++u) klo[u] = khi[u] = 0;
#pragma unroll
        for (int m = 0; m < R; ++m) {
            if (!a.key.mask[m]) continue;
            const CT* src = (const CT*)a.crd[m];
            CT c[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t e = base + u * kBlock + tid;
                c[u] = (FULL || e < hi) ? src[e] : CT(0);
            }
            const uint32_t sl = a.key.src_lo[m], ds = a.key.dst[m];
            if (sizeof(CT) == 4 && ds >= 32) {
                // 32-bit coordinates: the field lands in one half unless it straddles bit 32
#pragma unroll
                for (int u = 0; u < U; ++u) khi[u] |= (((uint32_t)c[u] >> sl) & (uint32_t)a.key.mask[m]) << (ds - 32);
            } else if (sizeof(CT) == 4 && ds + kw[m] <= 32) {
#pragma unroll
                for (int u = 0; u < U; ++u) klo[u] |= (((uint32_t)c[u] >> sl) & (uint32_t)a.key.mask[m]) << ds;
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint64_t f = (((uint64_t)c[u] >> sl) & a.key.mask[m]) << ds;
                    klo[u] |= (uint32_t)f;
                    khi[u] |= (uint32_t)(f >> 32);
                }
            }
        }
        bool ok[U];  // records past the end count into the spare block
#pragma unroll
        for (int u = 0; u < U; ++u) ok[u] = FULL || base + u * kBlock + tid < hi;
        // one copy of the pass loop (its shift and mask are scalar loads of the arguments)
#pragma unroll 1
        for (int p = 0; p < npass; ++p) {
            const uint32_t plo = (uint32_t)a.lo[p], pmask = (1u << a.bits[p]) - 1u;
            uint32_t slot[U];
            if (plo >= 32) {
#pragma unroll
                for (int u = 0; u < U; ++u) slot[u] = khi[u] >> (plo - 32);
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) slot[u] = __builtin_amdgcn_alignbit(khi[u], klo[u], plo);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t v = (slot[u] & pmask) | (uint32_t)(p * kBins);
                slot[u] = (FULL || ok[u]) ? v : spare;
            }
            // lane 0 always starts a run: the value "below" it is ~0, which no slot equals
            if (__popcll(ballot(from_lane_below(slot[0]) != slot[0])) >= 32) {
#pragma unroll
                for (int u = 0; u < U; ++u) atomicAdd(&s_h[slot[u]], 1u);
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) count_slot(s_h, slot[u], lane);
            }
        }
    };
    // count the digits of records [lo, hi) with U loads per key mode in flight.  The key is
    // built in two 32-bit halves; a pass's digit is one funnel shift (or one shift above bit
    // 31) and one and-or that also adds the pass's block offset.  Whether a pass's digits come
    // in runs is decided once per round from its first record (a wave where at least half of
    // the lanes start a run counts every lane directly); both ways count every lane once.
    auto count_range = [&](uint32_t lo, uint32_t hi) __attribute__((always_inline)) {
        uint32_t base = lo;
        for (; base + kBlock * U <= hi; base += kBlock * U) round(base, hi, std::true_type{});
        if (base < hi) round(base, hi, std::false_type{});
    };
    __syncthreads();
    if (!a.seg_mode) {
        const uint32_t chunk = kBlock * U;
        const uint32_t nchunks = (a.n + chunk - 1) / chunk;
        const uint32_t per = (nchunks + gridDim.x - 1) / gridDim.x;
        const uint32_t c0 = blockIdx.x * per, c1 = min(nchunks, c0 + per);
        if (c0 < c1) count_range(c0 * chunk, min(a.n, c1 * chunk));
        sync_after_lds_atomics();
        for (int i = tid; i < words; i += kBlock) {
            const uint32_t c = s_h[i];
            if (c) atomicAdd(&a.hist[i], c);
        }
        for (uint64_t i = blockIdx.x * (uint64_t)kBlock + tid; i < a.status_words; i += gridDim.x * (uint64_t)kBlock)
            a.status_zero[i] = 0;
        return;
    }
    // segment mode: a static range of large-segment tiles per workgroup; histograms are
    // flushed to the segment's block whenever the segment changes
    const uint32_t nT = (uint32_t)*a.large_ctl;
    const uint32_t per = (nT + gridDim.x - 1) / gridDim.x;
    const uint32_t t0 = blockIdx.x * per, t1 = min(nT, t0 + per);
    uint32_t cur = 0xFFFFFFFFu;
    for (uint32_t t = t0; t < t1; ++t) {
        const uint4 g = a.tile_geo[t];  // first record, records, segment's first tile, segment
        const uint32_t k = g.w;
        if (k != cur) {
            sync_after_lds_atomics();
            if (cur != 0xFFFFFFFFu) {
                for (int i = tid; i < words; i += kBlock) {
                    const uint32_t c = s_h[i];
                    if (c) atomicAdd(&a.hist[(size_t)cur * a.hist_stride + i], c);
                    s_h[i] = 0;
                }
            }
            cur = k;
            __syncthreads();
        }
        count_range(g.x, g.x + g.y);
        a.status_zero[(size_t)t * kBins + tid] = 0;
    }
    sync_after_lds_atomics();
    if (cur != 0xFFFFFFFFu) {
        for (int i = tid; i < words; i += kBlock) {
            const uint32_t c = s_h[i];
            if (c) atomicAdd(&a.hist[(size_t)cur * a.hist_stride + i], c);
        }
    }
}

// ------------------------------------------------------------------------------ digit pass

constexpr int kLookWin = 8;  // status words read per look-back round trip
// Global passes hand tiles out from 8 queues (one per XCD when workgroups are dispatched to the
// 8 XCDs round-robin), each in chunks of kTileChunk consecutive tiles, so that the partial
// cache lines where neighbouring tiles' digit runs meet are mostly written through one L2
// (plain workload: 891 -> 810 us per pass; chunks of 4, 16 and 32 tiles: 833, 812, 834 us).
// Below kQueueMinTiles tiles a launch uses one queue: with few tiles, chunks of 8 leave most
// queues (and their workgroups) without work.
constexpr uint32_t kTileQueues = 8;
constexpr uint32_t kTileChunk = 8;
constexpr uint32_t kQueueMinTiles = 2048;

// Decoupled look-back done by one whole wave for one counter: lane l reads the status of
// tile j - l, so 64 predecessors are inspected per round trip.  Statuses are at
// status[tile * stride + slot]; `lowest` is the first tile (it always publishes a prefix).
// Every lane returns the same exclusive prefix.
__device__ __forceinline__ uint32_t wave_look_back(const uint32_t* status, uint32_t t, uint32_t stride,
                                                   uint32_t slot, uint32_t lowest, uint32_t* err) {
    const int lane = threadIdx.x & 63;
    uint32_t excl = 0, spins = 0;
    uint32_t j = t - 1;  // most recent predecessor not yet accounted for
    for (;;) {
        const uint32_t avail = j - lowest + 1;
        const uint32_t w = (uint32_t)lane < avail ? ld_status(&status[(size_t)(j - lane) * stride + slot]) : 0u;
        const uint32_t f = w & ~kCntMask;
        const uint64_t notready = ballot((uint32_t)lane < avail && f == 0);
        const uint64_t prefix = ballot(f == kFlagP);
        const uint32_t stop_nr = notready ? (uint32_t)__builtin_ctzll(notready) : 64u;
        const uint32_t stop_p = prefix ? (uint32_t)__builtin_ctzll(prefix) : 64u;
        // lanes before the first not-ready one are usable; include the first prefix if it
        // comes before that
        const uint32_t use = stop_p < stop_nr ? stop_p + 1 : min(stop_nr, min(avail, 64u));
        uint32_t part = (uint32_t)lane < use ? (w & kCntMask) : 0u;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
        excl += part;
        if (stop_p < stop_nr) return excl;
        j -= use;
        if (stop_nr < 64 && stop_nr < avail) {
            if (++spins > kSpinLimit) {
                if (lane == 0) atomicOr(err, 1u);
                return excl;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
}

// Decoupled look-back for one digit: sum the counts of the predecessors of tile t back to
// the nearest one that has published an inclusive prefix.  kLookWin status words are read
// per round trip; `lowest` (the first tile of the segment) always publishes a prefix.
__device__ __forceinline__ uint32_t look_back(const uint32_t* status, uint32_t t, uint32_t lowest,
                                              uint32_t b, uint32_t* err) {
    uint32_t excl = 0, spins = 0;
    uint32_t j = t - 1;  // next predecessor to read
    {
        // usually the immediate predecessor has already published its prefix
        const uint32_t w = ld_status(&status[(size_t)j * kBins + b]);
        const uint32_t f = w & ~kCntMask;
        if (f == kFlagP) return w & kCntMask;
        if (f == kFlagA) {
            excl = w & kCntMask;
            --j;
        }
    }
    for (;;) {
        const uint32_t avail = j - lowest + 1;
        uint32_t w[kLookWin];
#pragma unroll
        for (int i = 0; i < kLookWin; ++i)
            w[i] = ((uint32_t)i < avail) ? ld_status(&status[(size_t)(j - i) * kBins + b]) : 0u;
        uint32_t used = 0;
        bool done = false, stalled = false;
#pragma unroll
        for (int i = 0; i < kLookWin; ++i) {
            if (done || stalled || (uint32_t)i >= avail) continue;
            const uint32_t f = w[i] & ~kCntMask;
            if (f == 0) {
                stalled = true;
                continue;
            }
            excl += w[i] & kCntMask;
            ++used;
            if (f == kFlagP) done = true;
        }
        if (done) return excl;
        j -= used;
        if (stalled) {
            if (++spins > kSpinLimit) {
                atomicOr(err, 1u);
                return excl;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
}

// Move one array of the tile: registers -> LDS (local slot lp) -> global (slot gp), with
// the next array's loads issued before the barrier.
template <typename T, int ITEMS>
__device__ __forceinline__ void load_items(const T* __restrict__ src, uint32_t start, uint32_t len,
                                           uint32_t wb, T (&x)[ITEMS]) {
    // A buffer resource over exactly this tile's records (len * sizeof(T) bytes from record
    // `start`).  The whole byte offset of every item, (wb + 64 i) * sizeof(T), goes into the
    // range-checked operands (the vector offset, with the compiler free to move a constant of up
    // to 4095 bytes into the instruction offset); the scalar offset, which the hardware range
    // check does not cover on gfx9-family targets, is always 0.  A load at or past `len` returns 0
    // without touching memory, so no access leaves records [start, start + len).
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)(src + start), 0, (int)(len * sizeof(T)), kBufferWord3);
    int voff = (int)(wb * sizeof(T));
    // kept opaque per call so that the per-item constants stay beside their loads, where they
    // fold into the instruction offset, instead of being hoisted into one register per item
    asm volatile("" : "+v"(voff));
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int off = voff + i * 64 * (int)sizeof(T);
        if constexpr (sizeof(T) == 8) {
            const auto w = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
            x[i] = (T)(((uint64_t)w[1] << 32) | w[0]);
        } else {
            x[i] = (T)__builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
        }
    }
}

template <typename T, int ITEMS>
__device__ __forceinline__ void stage_items(T* sx, uint32_t len, uint32_t wb, const T (&x)[ITEMS],
                                            const uint32_t (&lp)[ITEMS]) {
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
        if (wb + i * 64 < len) sx[lp[i]] = x[i];
}

// Local slot j goes to global position s_base[digit of slot j] + j.
__device__ __forceinline__ uint32_t slot_dest(const uint8_t* s_dig, const uint32_t* s_base, uint32_t j) {
    return s_base[s_dig[j]] + j;
}

template <typename T, int ITEMS>
__device__ __forceinline__ void drain_items(const T* sx, T* __restrict__ dst, uint32_t len, const uint8_t* s_dig,
                                            const uint32_t* s_base) {
#pragma unroll 4
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = i * kBlock + threadIdx.x;
        if (j < len) dst[slot_dest(s_dig, s_base, j)] = sx[j];
    }
}

// MODE 0: one segment [0, n).  MODE 1: the large segments of a bucketed group.  MODE 2: a
// batch of tensors (each tensor is one segment; its parameters come from a device table).
// PK: 0 records as given; 1 pack the R coordinate arrays into one array of 64-bit words on the
// way out; 2 unpack such words into R coordinate arrays.
template <int R, typename CT, typename VT, int ITEMS, int MODE, int PK>
__device__ __forceinline__ void digit_body(const DigitArgs& a) {
    constexpr bool PACK = PK == 1, UNPACK = PK == 2;
    constexpr int TILE = kBlock * ITEMS;
    __shared__ uint64_t s_x[TILE];               // record exchange (4- or 8-byte words)
    __shared__ uint32_t s_cnt[kWaves * kBins];   // per-wave digit counters, then wave prefixes
    __shared__ uint32_t s_cnt2[kWaves * kBins];  // second half of each wave's items
    __shared__ uint32_t s_tstart[kBins];         // first local slot of each digit
    __shared__ uint32_t s_base[kBins];           // global slot of local slot 0 of each digit
    __shared__ uint8_t s_dig[TILE];
    __shared__ uint32_t s_tmp[2 * kWaves];
    __shared__ uint32_t s_geo[6];                // tile, start, len, segment base, k, first tile
    __shared__ uint32_t s_hpre[kBins];           // one segment: exclusive prefix of the digit counts
    // batch mode: the table entry of the tile's tensor, copied once per tile
    __shared__ uint32_t s_bp[MODE == 2 ? sizeof(BatchPass) / 4 : 1];
    static_assert(sizeof(BatchPass) % 4 == 0, "the table entry is copied in 32-bit words");

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (MODE == 0) s_hpre[tid] = block_excl_scan(a.hist[tid], s_tmp, nullptr);  // same for every tile
    // segment mode: tiles of the large segments, written by the previous kernel
    const uint32_t seg_tiles = MODE == 1 ? (uint32_t)*a.large_ctl : 0u;

    for (;;) {
        if (tid < 64) {
            // queue q (of G) hands out chunks q, q + G, q + 2G, ... of kTileChunk consecutive
            // (launch) tiles.  Every queue has a workgroup (G <= grid),
            // each queue's tiles go out in increasing order, and a tile waits only for lower
            // tiles, so the lowest unfinished tile always has a running workgroup or a free one
            // that will take it.  Wave 0 computes the geometry (lane 0 takes the tile).
            const uint32_t G = (MODE == 1 ? seg_tiles : a.ntiles) >= kQueueMinTiles ? min(kTileQueues, gridDim.x) : 1u;
            const uint32_t qi = blockIdx.x % G;
            uint32_t taken = 0;
            if (tid == 0) taken = atomicAdd(a.tile_counter + qi, 1u);
            const uint32_t lt = uni32(taken);
            uint32_t t = lt, ntiles = a.ntiles, start = 0, len = 0, base = 0, k = 0, lowest = 0;
            bool live = false;
            if (MODE == 1) {
                ntiles = seg_tiles;
                t = ((lt / kTileChunk) * G + qi) * kTileChunk + lt % kTileChunk;
                if (t < ntiles) {
                    // one load: first record, records, the segment's first tile, segment
                    const uint4 g = reinterpret_cast<const uint4*>(a.tile_map)[t];
                    start = g.x;
                    len = g.y;
                    lowest = g.z;
                    k = g.w;
                    base = start - (t - lowest) * TILE;
                    live = true;
                }
            } else if (MODE == 2) {
                const uint32_t lq = ((lt / kTileChunk) * G + qi) * kTileChunk + lt % kTileChunk;
                if (lq < ntiles) {
                    // one load: stable tile id (the look-back words are indexed by it), tensor,
                    // first record and record count of the launch tile
                    const uint4 g = reinterpret_cast<const uint4*>(a.tile_map)[lq];
                    t = g.x;
                    k = g.y;
                    start = g.z;
                    len = g.w;
                    lowest = t - start / TILE;  // the tensor's first tile
                    live = true;
                    // the tensor's table entry, read by the whole wave at once
                    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.batch + k);
                    for (int i = tid; i < (int)(sizeof(BatchPass) / 4); i += 64) s_bp[i] = src[i];
                }
            } else {
                t = ((lt / kTileChunk) * G + qi) * kTileChunk + lt % kTileChunk;
                if (t < ntiles) {
                    start = t * TILE;
                    len = min((uint32_t)TILE, a.n - start);
                    live = true;
                }
            }
            if (tid == 0) {
                s_geo[0] = live ? t : 0xFFFFFFFFu;
                s_geo[1] = start;
                s_geo[2] = len;
                s_geo[3] = base;
                s_geo[4] = k;
                s_geo[5] = lowest;
            }
        }
        __syncthreads();
        // tile geometry is uniform: keep it in scalar registers
        const uint32_t t = __builtin_amdgcn_readfirstlane(s_geo[0]);
        if (t == 0xFFFFFFFFu) break;
        const uint32_t start = __builtin_amdgcn_readfirstlane(s_geo[1]);
        const uint32_t len = __builtin_amdgcn_readfirstlane(s_geo[2]);
        const uint32_t seg_base = __builtin_amdgcn_readfirstlane(s_geo[3]);
        const uint32_t k = __builtin_amdgcn_readfirstlane(s_geo[4]);
        const uint32_t lowest = __builtin_amdgcn_readfirstlane(s_geo[5]);
        const bool first = (t == lowest);
        // the pass's parameters.  Batch mode reads the tensor's table entry from its LDS copy
        // into scalar registers once per tile: read from global memory, each use would be
        // reloaded after every store, since the compiler cannot tell that the stores leave the
        // table alone.
        const BatchPass& J = *reinterpret_cast<const BatchPass*>(s_bp);
        DevKey key;
        const void* src_crd[R];
        void* dst_crd[R];
        int32_t pk_pos[R];
        uint64_t pk_mask[R];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            key.mask[m] = MODE == 2 ? uni64(J.key.mask[m]) : a.key.mask[m];
            key.src_lo[m] = MODE == 2 ? (int32_t)uni32((uint32_t)J.key.src_lo[m]) : a.key.src_lo[m];
            key.dst[m] = MODE == 2 ? (int32_t)uni32((uint32_t)J.key.dst[m]) : a.key.dst[m];
            src_crd[m] = MODE == 2 ? uni_ptr(J.src_crd[m]) : a.src_crd[m];
            dst_crd[m] = MODE == 2 ? uni_ptr(J.dst_crd[m]) : a.dst_crd[m];
            pk_pos[m] = MODE == 2 ? (int32_t)uni32((uint32_t)J.pk_pos[m]) : a.pk_pos[m];
            pk_mask[m] = MODE == 2 ? uni64(J.pk_mask[m]) : a.pk_mask[m];
        }
        const int lo_bit = MODE == 2 ? (int)uni32((uint32_t)J.lo) : a.lo;
        const int nbits = MODE == 2 ? (int)uni32((uint32_t)J.bits) : a.bits;
        const int r = MODE == 2 ? (int)uni32((uint32_t)J.r) : R;
        const void* src_val = MODE == 2 ? uni_ptr(J.src_val) : a.src_val;
        void* dst_val = MODE == 2 ? uni_ptr(J.dst_val) : a.dst_val;
        const uint32_t* hist = MODE == 2 ? uni_ptr(J.hist) : a.hist + (size_t)k * a.hist_stride;
        const uint32_t dmask = (1u << nbits) - 1u;
        const uint32_t wb = (uint32_t)wave * 64u * ITEMS + lane;  // wave w owns a contiguous slice

        // ---- key modes first: the tile's digit counts are published as early as possible;
        // the other arrays are loaded while the look-back waits on the predecessors
        CT c[UNPACK ? 1 : R][ITEMS];
        uint64_t pw[UNPACK ? ITEMS : 1];  // packed words (unpacking pass)
        VT v[ITEMS];
        uint32_t dg[ITEMS], lp[ITEMS];
        if constexpr (UNPACK) {
            // the group's composite key sits in the low bits of every word
            load_items<uint64_t, ITEMS>((const uint64_t*)src_crd[0], start, len, wb, pw);
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) dg[i] = (uint32_t)(pw[i] >> lo_bit) & dmask;
        } else {
#pragma unroll
            for (int m = 0; m < R; ++m)
                if (m < r && key.mask[m]) load_items<CT, ITEMS>((const CT*)src_crd[m], start, len, wb, c[m]);
            if constexpr (sizeof(CT) == 4) {
                // 32-bit coordinates: the digit is assembled from each key mode's slice of the
                // digit window (one bit-field extract and one shift-or per mode) instead of
                // building the 64-bit key
                DigitSlice sl[R];
#pragma unroll
                for (int m = 0; m < R; ++m)
                    sl[m] = (m < r && key.mask[m])
                                ? digit_slice(key.dst[m], key.src_lo[m], 64 - __builtin_clzll(key.mask[m]), lo_bit, nbits)
                                : DigitSlice{0u, 0u, 0u};
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    uint32_t dv = 0;
#pragma unroll
                    for (int m = 0; m < R; ++m)
                        if (m < r && key.mask[m])
                            dv |= __builtin_amdgcn_ubfe((uint32_t)c[m][i], sl[m].rs, sl[m].ln) << sl[m].ls;
                    dg[i] = dv;
                }
            } else {
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    uint64_t kv = 0;
#pragma unroll
                    for (int m = 0; m < R; ++m)
                        if (m < r && key.mask[m])
                            kv |= (((uint64_t)c[m][i] >> key.src_lo[m]) & key.mask[m]) << key.dst[m];
                    dg[i] = (uint32_t)(kv >> lo_bit) & dmask;
                }
            }
        }

        // ---- stable rank inside each wave: ballot-match the digit, count lanes below.  Two
        // counter sets: the first and second halves of a wave's items form two independent
        // read-modify-write chains on LDS; the second half then adds the first half's totals.
        for (int b = lane; b < kBins; b += 64) {
            s_cnt[wave * kBins + b] = 0;
            s_cnt2[wave * kBins + b] = 0;
        }
        constexpr int kHalf = ITEMS / 2;
#pragma unroll
        for (int h = 0; h < kHalf; ++h) {
#pragma unroll
            for (int part = 0; part < 2; ++part) {
                const int i = part * kHalf + h;
                uint32_t* cnt = part ? s_cnt2 : s_cnt;
                const bool ok = (wb + i * 64) < len;
                const uint32_t d = dg[i];
                // peers: the lanes whose digit equals this lane's, bit by bit.  sm is this lane's
                // bit b smeared over the word (0 or ~0); a lane j agrees with it on bit b iff
                // bit j of ~(ballot ^ sm) is set.  Kept as two 32-bit halves.  All 8 bits are
                // visited: above the pass's width every digit has 0, which leaves the mask as is.
                const uint64_t pk0 = ballot(ok);
                uint32_t plo = (uint32_t)pk0, phi = (uint32_t)(pk0 >> 32);
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    uint32_t sm = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);
                    asm("" : "+v"(sm));  // opaque: the ballot then compares sm itself
                    const uint64_t bb = ballot(sm != 0u);
                    // acc & ~(ballot ^ sm) in one three-input operation per half (truth table
                    // 0x90: set where acc is set and the other two agree)
                    plo = __builtin_amdgcn_bitop3_b32(plo, (uint32_t)bb, sm, 0x90);
                    phi = __builtin_amdgcn_bitop3_b32(phi, (uint32_t)(bb >> 32), sm, 0x90);
                }
                const uint64_t peers = ((uint64_t)phi << 32) | plo;
                const uint32_t below = lanes_below(peers);
                uint32_t old = 0;
                if (ok) old = cnt[wave * kBins + d];
                lp[i] = old + below;
                if (ok && below == 0) cnt[wave * kBins + d] = old + (uint32_t)__popcll(peers);
            }
        }
#pragma unroll
        for (int i = kHalf; i < ITEMS; ++i)
            if ((wb + i * 64) < len) lp[i] += s_cnt[wave * kBins + dg[i]];
        for (int b = lane; b < kBins; b += 64) s_cnt[wave * kBins + b] += s_cnt2[wave * kBins + b];
        __syncthreads();

        // ---- per digit: wave prefixes, tile count and the tile-local digit starts; the tile's
        // counts are published at once
        uint32_t tcnt, tstart, hstart;  // of digit b = tid
        {
            const uint32_t b = tid;
            uint32_t run = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t x = s_cnt[w * kBins + b];
                s_cnt[w * kBins + b] = run;
                run += x;
            }
            tcnt = run;
            st_status(&a.status[(size_t)t * kBins + b], (first ? kFlagP : kFlagA) | tcnt);
            // the rest of the records, in flight during the scans and the look-back
            if constexpr (!UNPACK) {
#pragma unroll
                for (int m = 0; m < R; ++m)
                    if (m < r && !key.mask[m]) load_items<CT, ITEMS>((const CT*)src_crd[m], start, len, wb, c[m]);
            }
            load_items<VT, ITEMS>((const VT*)src_val, start, len, wb, v);
            tstart = block_excl_scan(tcnt, s_tmp, nullptr);
            // one sort: computed once per workgroup; segments and batches: offsets stored by
            // k_hist_prefix_seg / k_hist_prefix
            hstart = MODE == 0 ? s_hpre[b] : hist[b];
            s_tstart[b] = tstart;
        }
        // ---- the global offset of every digit: decoupled look-back over the predecessors
        {
            const uint32_t b = tid;
            uint32_t excl = 0;
            if (!first) {
                excl = look_back(a.status, t, lowest, b, a.err);
                st_status(&a.status[(size_t)t * kBins + b], kFlagP | (excl + tcnt));
            }
            s_base[b] = seg_base + hstart + excl - tstart;
            if (a.status_next) a.status_next[(size_t)t * kBins + b] = 0;
        }
        __syncthreads();

        // ---- local slot of every record and the digit of every local slot; the first array is
        // staged in LDS by local slot in the same sweep (it is already in registers)
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if ((wb + i * 64) < len) {
                const uint32_t d = dg[i];
                lp[i] += s_tstart[d] + s_cnt[wave * kBins + d];
                s_dig[lp[i]] = (uint8_t)d;
                if constexpr (UNPACK) {
                    s_x[lp[i]] = pw[i];
                } else if constexpr (PACK) {
                    uint64_t w = 0;
#pragma unroll
                    for (int m = 0; m < R; ++m)
                        if (m < r) w |= ((uint64_t)c[m][i] & pk_mask[m]) << pk_pos[m];
                    s_x[lp[i]] = w;
                } else {
                    ((CT*)s_x)[lp[i]] = c[0][i];
                }
            }
        }
        __syncthreads();

        // ---- move every array through LDS: contiguous runs per digit on the way out
        if constexpr (UNPACK) {
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t j = i * kBlock + tid;
                if (j < len) {
                    const uint64_t w = s_x[j];
                    const uint32_t g = slot_dest(s_dig, s_base, j);
#pragma unroll
                    for (int m = 0; m < R; ++m)
                        if (m < r) ((CT*)dst_crd[m])[g] = (CT)((w >> pk_pos[m]) & pk_mask[m]);
                }
            }
            __syncthreads();
        } else if constexpr (PACK) {
            drain_items<uint64_t, ITEMS>(s_x, (uint64_t*)dst_crd[0], len, s_dig, s_base);
            __syncthreads();
        } else {
#pragma unroll
            for (int m = 0; m < R; ++m) {
                if (m >= r) break;
                if (m > 0) {
                    stage_items<CT, ITEMS>((CT*)s_x, len, wb, c[m], lp);
                    __syncthreads();
                }
                drain_items<CT, ITEMS>((const CT*)s_x, (CT*)dst_crd[m], len, s_dig, s_base);
                __syncthreads();
            }
        }
        stage_items<VT, ITEMS>((VT*)s_x, len, wb, v, lp);
        __syncthreads();
        drain_items<VT, ITEMS>((const VT*)s_x, (VT*)dst_val, len, s_dig, s_base);
        __syncthreads();
    }
}

template <int R, typename CT, typename VT, int ITEMS, int MODE, int PK>
__global__ void __launch_bounds__(256) k_digit(DigitArgs a) {
    digit_body<R, CT, VT, ITEMS, MODE, PK>(a);
}

// The same pass compiled for three resident workgroups per CU: for the record layouts whose
// registers fit (packed words in, i.e. the middle and the unpacking passes), the extra
// workgroup hides the look-back and barrier latencies of the other two.
template <int R, typename CT, typename VT, int ITEMS, int MODE, int PK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) k_digit3(DigitArgs a) {
    digit_body<R, CT, VT, ITEMS, MODE, PK>(a);
}

// ------------------------------------------------------------------------------ buckets

// Segment starts: positions where the prefix (sigma_1..sigma_l) differs from the previous
// record (Alg. 2's bucket discovery), compacted in order with a single-word look-back.  The work
// per record is tiny, so tiles are large (kDiscTile records, eight sub-chunks per wave whose
// 64-record flag masks wait in LDS): with 4096-record tiles, thousands of tiles were in flight
// at once and each look-back found the nearest published prefix far behind it, 64 tiles per
// memory round trip, which bounded the whole kernel.
template <typename CT>
__global__ void __launch_bounds__(256) k_boundary(BoundArgs a) {
    constexpr int SUB = 16;                               // 64-record items per wave and sub-chunk
    constexpr int WSPAN = kDiscTile / kWaves;             // records of one wave
    constexpr int NSUB = WSPAN / (SUB * 64);
    constexpr int NP = sizeof(BoundArgs::prefix) / sizeof(int32_t);  // prefix modes at most
    static_assert(NSUB * SUB * 64 * kWaves == kDiscTile, "tile shape");
    __shared__ uint64_t s_mask[kDiscTile / 64];           // flags, one word per 64 records
    __shared__ uint32_t s_wsum[kWaves];
    __shared__ uint32_t s_geo[2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) {
        const uint32_t t = atomicAdd(a.tile_counter, 1u);
        s_geo[0] = t;
    }
    __syncthreads();
    const uint32_t t = s_geo[0];
    const uint32_t start = t * kDiscTile;
    if (start >= a.n) return;
    const uint32_t len = min((uint32_t)kDiscTile, a.n - start);
    const uint32_t w0 = (uint32_t)wave * WSPAN;           // the wave's first record in the tile
    const int j0 = a.prev_bits ? a.nskip : 0;
    // the previous record of each prefix mode: for the wave's first record one scalar load,
    // then lane 63 of the item before
    CT carry[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        carry[j] = CT(0);
        if (j >= j0 && j < a.nprefix && w0 < len && start + w0 > 0) carry[j] = ((const CT*)a.crd[a.prefix[j]])[start + w0 - 1];
    }
    uint32_t wcount = 0;
    for (int k = 0; k < NSUB; ++k) {
        const uint32_t o0 = w0 + (uint32_t)k * SUB * 64;  // sub-chunk's first record in the tile
        bool f[SUB];
#pragma unroll
        for (int i = 0; i < SUB; ++i) f[i] = (start + o0 + i * 64 + lane == 0);
        if (a.prev_bits) {  // the previous group's segment starts: one word per 64 records
#pragma unroll
            for (int i = 0; i < SUB; ++i) {
                const uint64_t w = o0 + i * 64 < len ? a.prev_bits[(start + o0) / 64u + i] : 0ull;
                f[i] |= ((w >> lane) & 1ull) != 0;
            }
        }
        // one prefix mode at a time, all of its loads in flight together (range-checked: 0
        // past the tile); each record's predecessor comes from the lane below or the carry
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            if (j >= j0 && j < a.nprefix) {
                CT cur[SUB];
                load_items<CT, SUB>((const CT*)a.crd[a.prefix[j]], start, len, o0 + lane, cur);
#pragma unroll
                for (int i = 0; i < SUB; ++i) {
                    const CT below = lane_below(cur[i]);
                    const CT prv = lane == 0 ? carry[j] : below;
                    carry[j] = lane63(cur[i]);
                    f[i] |= cur[i] != prv;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < SUB; ++i) {
            const bool valid = o0 + i * 64 < len;
            const uint64_t m = ballot(f[i] && o0 + i * 64 + lane < len);
            wcount += (uint32_t)__popcll(m);
            if (lane == 0) {
                s_mask[o0 / 64 + i] = m;
                if (a.bits_out && valid) a.bits_out[(start + o0) / 64u + i] = m;
            }
        }
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
            if (start + len == a.n) {
                *a.nb_out = excl + tot;
                a.seg_start[excl + tot] = a.n;
                a.region_seg[(a.n + kRegion - 1) / kRegion] = excl + tot;
            }
        }
    }
    __syncthreads();
    uint32_t pos = s_geo[1];
    for (int w = 0; w < wave; ++w) pos += s_wsum[w];
    for (int q = 0; q < NSUB * SUB; ++q) {
        const uint32_t o = w0 + (uint32_t)q * 64;
        const uint64_t f = s_mask[o / 64];
        const uint32_t e = start + o + lane;
        const uint32_t before = pos + lanes_below(f);  // segments starting before e
        if ((f >> lane) & 1ull) a.seg_start[before] = e;
        if (o + lane < len && e % (uint32_t)kRegion == 0) a.region_seg[e / kRegion] = before;
        pos += (uint32_t)__popcll(f);
    }
}

// Sort segments into three classes: tiny (sorted together with the other tiny segments that
// start in the same region), medium (one workgroup each) and large (digit passes over tiles of
// the segment).  Writes the LDS sort's work items: one per region, then one per medium segment.
__global__ void __launch_bounds__(256) k_classify(ClassArgs a) {
    const uint32_t nb = *a.nb;
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t r = blockIdx.x * kBlock + threadIdx.x; r < a.nregions; r += stride) {
        // segments starting in [r*kRegion, (r+1)*kRegion): sa .. se-1; only the last of them
        // can be longer than the region (kTinyLen == kRegion), and it is left out if it is
        const uint32_t sa = a.region_seg[r];
        uint32_t se = a.region_seg[r + 1];
        if (se > sa && a.seg_start[se] - a.seg_start[se - 1] > (uint32_t)kTinyLen) --se;
        const uint32_t rs = a.seg_start[sa];
        a.geo[r] = make_uint4(rs, a.seg_start[se] - rs, sa, se);
    }
    for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < nb; k += stride) {
        const uint32_t s = a.seg_start[k];
        const uint32_t len = a.seg_start[k + 1] - s;
        if (len <= (uint32_t)kTinyLen) continue;
        if (len <= (uint32_t)kSmallCap) {
            const uint32_t i = atomicAdd(a.nmed, 1u);
            a.geo[a.nregions + i] = make_uint4(s, len, 0, 0);
        } else {
            const uint32_t tiles = (len + a.tile - 1) / a.tile;
            const unsigned long long old =
                atomicAdd((unsigned long long*)a.large_ctl, (1ull << 32) | (unsigned long long)tiles);
            // segments and their tiles are numbered in the same order: first tiles increase
            // with the segment number (k_tile_geo searches them)
            const uint32_t idx = (uint32_t)(old >> 32);
            a.large[idx] = make_uint4(s, len, (uint32_t)old, 0);
            uint32_t* h = a.seg_hist + (size_t)idx * a.hist_stride;
            for (uint32_t i = 0; i < a.hist_stride; ++i) h[i] = 0;
        }
    }
}

// One geometry entry per large-segment tile (first record, records, the segment's first tile,
// segment), one thread per tile: the tile's segment is the last one whose first tile is at or
// before it.  Spread over the grid, so that a segment of thousands of tiles costs no single
// thread thousands of stores.
__global__ void __launch_bounds__(256) k_tile_geo(ClassArgs a) {
    const uint64_t ctl = *a.large_ctl;
    const uint32_t nl = (uint32_t)(ctl >> 32), nt = (uint32_t)ctl;
    for (uint32_t t = blockIdx.x * kBlock + threadIdx.x; t < nt; t += gridDim.x * kBlock) {
        uint32_t lo = 0, hi = nl - 1;  // nl >= 1 whenever nt >= 1
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) / 2;
            if (a.large[mid].z <= t) lo = mid; else hi = mid - 1;
        }
        const uint4 g = a.large[lo];
        const uint32_t i = t - g.z;
        a.tile_geo[t] = make_uint4(g.x + i * a.tile, min(a.tile, g.y - i * a.tile), g.z, lo);
    }
}

// Range-checked access to the n elements of type T from base through a buffer resource: a
// load outside returns 0 and a store outside is dropped, neither touching memory, and neither
// needs a branch (a branch per element would wait for each load before the next).  The scalar
// offset, which the hardware range check does not cover on gfx9-family targets, is always 0.
using u32x2 = uint32_t __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t elem_rsrc(const void* base, uint32_t n) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)(n * sizeof(T)), kBufferWord3);
}
template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, int off) {
    if constexpr (sizeof(T) == 8) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        return (T)(((uint64_t)w[1] << 32) | w[0]);
    } else {
        return (T)__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
    }
}
template <typename T>
__device__ __forceinline__ void buf_st(T v, __amdgpu_buffer_rsrc_t r, int off) {
    if constexpr (sizeof(T) == 8) {
        u32x2 w;
        w[0] = (uint32_t)(uint64_t)v;
        w[1] = (uint32_t)((uint64_t)v >> 32);
        __builtin_amdgcn_raw_buffer_store_b64(w, r, off, 0, 0);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32((uint32_t)v, r, off, 0, 0);
    }
}

// Stable sort of short runs of records in LDS, by (segment number, group key).  Work items
// (k_classify): the tiny segments starting in each region of kRegion records (their union is
// one run of fewer than kSmallCap records), then every medium segment.  Only the key modes are
// loaded up front; each thread keeps the 64-bit keys of its slots in registers, and every LSD
// pass over the key bits that vary inside the run publishes one digit byte per slot and moves
// 16-bit slot numbers through LDS.  The records are then gathered in sorted order straight from
// global memory (the key modes were just read: mostly cache hits) and written back at the same
// positions of the destination, which may be the source itself.  With no records held in
// registers and 26 KB of LDS, several runs share a CU; the next item's geometry is loaded one
// item ahead.
template <int R, typename CT, typename VT, int W>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W, 8))) k_small(SmallArgs a) {
    constexpr int CAP = kSmallCap, ITEMS = CAP / kBlock;
    static_assert(kTinyLen == kRegion && kRegion + kTinyLen <= kSmallCap, "a region run must fit");
    __shared__ uint16_t s_ia[CAP], s_ib[CAP];  // slot permutations; s_ib first holds segment numbers
    __shared__ uint8_t s_dig[CAP];             // this pass's digit of every slot
    __shared__ uint32_t s_cnt[kWaves * kBins];
    __shared__ uint32_t s_bstart[kBins];
    __shared__ uint32_t s_tmp[2 * kWaves];
    __shared__ uint64_t s_red[2 * kWaves];
    __shared__ uint32_t s_run[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // written by the previous kernel: fixed for the whole launch
    const uint32_t nitems = a.nregions + *a.nmed;
    uint4 gnext = make_uint4(0, 0, 0, 0);  // thread 0: geometry of the workgroup's next item
    if (tid == 0 && blockIdx.x < nitems) gnext = a.geo[blockIdx.x];
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        if (tid == 0) {
            s_run[0] = gnext.x;
            s_run[1] = gnext.y;
            s_run[2] = gnext.z;
            s_run[3] = gnext.w;
            if (item + gridDim.x < nitems) gnext = a.geo[item + gridDim.x];
        }
        __syncthreads();
        // the thread's index, opaque per item: slot indices derived from it are recomputed
        // where they are used instead of being hoisted out of the loop and spilled
        int ot = tid;
        asm volatile("" : "+v"(ot));
        const uint32_t rs = __builtin_amdgcn_readfirstlane(s_run[0]);
        const uint32_t L = __builtin_amdgcn_readfirstlane(s_run[1]);
        const uint32_t sa = __builtin_amdgcn_readfirstlane(s_run[2]);
        const uint32_t se = __builtin_amdgcn_readfirstlane(s_run[3]);
        if (L == 0) {
            __syncthreads();
            continue;
        }

        // ---- group key of every slot j = i*kBlock + tid (the key modes of a group of modes are
        // loaded together), and the starts of the run's segments after its first (regions only:
        // a medium item has sa == se == 0)
        uint64_t key[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) key[i] = 0;
        constexpr int KG = sizeof(CT) == 4 ? 4 : 2;  // modes loaded at once
        uint32_t st[ITEMS / 2];  // at most kRegion segments start in a region
#pragma unroll
        for (int m0 = 0; m0 < R; m0 += KG) {
            CT x[KG][ITEMS];
#pragma unroll
            for (int g = 0; g < KG; ++g) {
                if (m0 + g < R) {
                    // a mode outside the key gets an empty range: its loads touch no memory
                    const __amdgpu_buffer_rsrc_t rc =
                        elem_rsrc<CT>((const CT*)a.src_crd[m0 + g] + rs, a.key.mask[m0 + g] ? L : 0u);
#pragma unroll
                    for (int i = 0; i < ITEMS; ++i) x[g][i] = buf_ld<CT>(rc, (int)((i * kBlock + ot) * sizeof(CT)));
                }
            }
            if (m0 == 0) {
                // seg_start[sa+1 .. se-1]; 0 past the end (never above rs)
                const __amdgpu_buffer_rsrc_t rc = elem_rsrc<uint32_t>(a.seg_start + sa + 1, se > sa ? se - sa - 1 : 0u);
#pragma unroll
                for (int i = 0; i < ITEMS / 2; ++i) st[i] = buf_ld<uint32_t>(rc, (int)((i * kBlock + ot) * 4));
            }
#pragma unroll
            for (int g = 0; g < KG; ++g) {
                if (m0 + g < R) {
                    const uint64_t mk = a.key.mask[m0 + g];
                    const int lo = a.key.src_lo[m0 + g], dst = a.key.dst[m0 + g];
#pragma unroll
                    for (int i = 0; i < ITEMS; ++i) key[i] |= (((uint64_t)x[g][i] >> lo) & mk) << dst;
                }
            }
        }

        // ---- segment number of every slot (in s_ib)
        uint16_t* s_seg = s_ib;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) s_seg[i * kBlock + ot] = 0;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS / 2; ++i)
            if (st[i] > rs) s_seg[st[i] - rs] = 1;
        __syncthreads();
        {
            // blocked inclusive scan: thread tid owns slots [tid*ITEMS, tid*ITEMS+ITEMS)
            uint32_t loc[ITEMS], sum = 0;
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t j = ot * ITEMS + i;
                sum += (j < L) ? s_seg[j] : 0;
                loc[i] = sum;
            }
            const uint32_t before = block_excl_scan(sum, s_tmp, nullptr);
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t j = ot * ITEMS + i;
                if (j < L) s_seg[j] = (uint16_t)(before + loc[i]);
            }
        }
        __syncthreads();
        // ---- composite keys: (segment number << key bits) | group key
        uint64_t kor = 0, kand = ~0ull;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t j = i * kBlock + ot;
            if (j < L) {
                key[i] |= (uint64_t)s_seg[j] << a.key_bits;
                kor |= key[i];
                kand &= key[i];
            }
            s_ia[j] = (uint16_t)j;
        }
        for (int o = 32; o > 0; o >>= 1) {
            kor |= __shfl_xor(kor, o, 64);
            kand &= __shfl_xor(kand, o, 64);
        }
        if (lane == 0) {
            s_red[wave] = kor;
            s_red[kWaves + wave] = kand;
        }
        __syncthreads();  // also: every read of s_seg is done before s_ib serves as a permutation
        kor = 0;
        kand = ~0ull;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            kor |= s_red[w];
            kand &= s_red[kWaves + w];
        }
        const uint64_t vary = kor ^ kand;
        // ---- LSD passes over the bits that vary inside this run.  Each wave ranks one
        // contiguous quarter of the run (C positions, a multiple of 64), so a short run costs
        // every wave the same few steps.
        uint16_t* cur = s_ia;
        uint16_t* nxt = s_ib;
        const uint32_t C = (L + kBlock - 1) / kBlock * 64u;
        const uint32_t wb = (uint32_t)wave * C + lane;
        if (vary) {
            const int lo = __builtin_ctzll(vary), hi = 63 - __builtin_clzll(vary);
            for (int sh = lo; sh <= hi; sh += 8) {
                const int nbits = min(8, hi - sh + 1);
                const uint32_t dmask = (1u << nbits) - 1u;
                if (((vary >> sh) & dmask) == 0) continue;  // digit constant over the run
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    const uint32_t j = i * kBlock + ot;
                    if (j < L) s_dig[j] = (uint8_t)((key[i] >> sh) & dmask);
                }
                for (int b = lane; b < kBins; b += 64) s_cnt[wave * kBins + b] = 0;
                __syncthreads();
                uint32_t dg[ITEMS], lp[ITEMS];
                uint16_t sv[ITEMS];
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    const uint32_t j = wb + i * 64;
                    const bool ok = i * 64u < C && j < L;
                    sv[i] = ok ? cur[j] : 0;
                    dg[i] = ok ? s_dig[sv[i]] : 0;
                    lp[i] = 0;
                }
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    if (i * 64u < C) {
                        const bool ok = (wb + i * 64) < L;
                        const uint32_t d = dg[i];
                        // peers: the lanes whose digit equals this lane's.  sm is this lane's bit b
                        // smeared over the word; lane j agrees with it on bit b iff bit j of
                        // ~(ballot ^ sm) is set (bitop3 truth table 0x90: acc & ~(x ^ y)).
                        const uint64_t pk0 = ballot(ok);
                        uint32_t plo = (uint32_t)pk0, phi = (uint32_t)(pk0 >> 32);
#pragma unroll
                        for (int b = 0; b < 8; ++b) {
                            if (b < nbits) {
                                uint32_t sm = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);
                                asm("" : "+v"(sm));  // opaque: the ballot then compares sm itself
                                const uint64_t bb = ballot(sm != 0u);
                                plo = __builtin_amdgcn_bitop3_b32(plo, (uint32_t)bb, sm, 0x90);
                                phi = __builtin_amdgcn_bitop3_b32(phi, (uint32_t)(bb >> 32), sm, 0x90);
                            }
                        }
                        const uint64_t peers = ((uint64_t)phi << 32) | plo;
                        const uint32_t below = lanes_below(peers);
                        uint32_t old = 0;
                        if (ok) old = s_cnt[wave * kBins + d];
                        lp[i] = old + below;
                        if (ok && below == 0) s_cnt[wave * kBins + d] = old + (uint32_t)__popcll(peers);
                    }
                }
                __syncthreads();
                {
                    const uint32_t b = ot;
                    uint32_t run = 0;
#pragma unroll
                    for (int w = 0; w < kWaves; ++w) {
                        const uint32_t x = s_cnt[w * kBins + b];
                        s_cnt[w * kBins + b] = run;
                        run += x;
                    }
                    s_bstart[b] = block_excl_scan(run, s_tmp, nullptr);
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    if (i * 64u < C && (wb + i * 64) < L) {
                        const uint32_t d = dg[i];
                        nxt[lp[i] + s_bstart[d] + s_cnt[wave * kBins + d]] = sv[i];
                    }
                }
                __syncthreads();
                uint16_t* t = cur;
                cur = nxt;
                nxt = t;
            }
        }
        // ---- gather every array in sorted order and write it back at the run's positions.
        // The destination may be the source: each round's loads have all returned, in every
        // wave, before any of its stores.
        uint32_t pm[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) pm[i] = cur[i * kBlock + ot];
        auto gather_rounds = [&](auto tag, const void* const* srcs, void* const* dsts, int nar) __attribute__((always_inline)) {
            using T = decltype(tag);
            constexpr int G = sizeof(T) == 4 ? 5 : 2;  // arrays per round: at most 80 data VGPRs
#pragma unroll
            for (int m0 = 0; m0 < nar; m0 += G) {
                T x[G][ITEMS];
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    if (m0 + g < nar) {
                        const __amdgpu_buffer_rsrc_t rc = elem_rsrc<T>((const T*)srcs[m0 + g] + rs, L);
#pragma unroll
                        for (int i = 0; i < ITEMS; ++i) x[g][i] = buf_ld<T>(rc, (int)(pm[i] * sizeof(T)));
                    }
                }
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                __syncthreads();
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    if (m0 + g < nar) {
                        // slots at or past L fall outside the range and are not written
                        const __amdgpu_buffer_rsrc_t rc = elem_rsrc<T>((T*)dsts[m0 + g] + rs, L);
#pragma unroll
                        for (int i = 0; i < ITEMS; ++i) buf_st<T>(x[g][i], rc, (int)((i * kBlock + ot) * sizeof(T)));
                    }
                }
            }
        };
        if constexpr (sizeof(CT) == sizeof(VT)) {
            const void* srcs[R + 1];
            void* dsts[R + 1];
#pragma unroll
            for (int m = 0; m < R; ++m) {
                srcs[m] = a.src_crd[m];
                dsts[m] = a.dst_crd[m];
            }
            srcs[R] = a.src_val;
            dsts[R] = a.dst_val;
            gather_rounds(CT(0), srcs, dsts, R + 1);
        } else {
            gather_rounds(CT(0), a.src_crd, a.dst_crd, R);
            const void* vs[1] = {a.src_val};
            void* vd[1] = {a.dst_val};
            gather_rounds(VT(0), vs, vd, 1);
        }
        __syncthreads();
    }
}

// W resident waves per SIMD (workgroups per CU): 3 allow 168 VGPRs, 4 allow 128.  Four spill
// nothing up to two modes and 20 bytes for three int32 modes with fp64 values (that layout's
// sort: 984 -> 853 us on the 1e8-nonzero (0,2,1)), but 60-270 bytes elsewhere (four int32
// modes with fp32 values: 33% slower).
template <int R, typename CT, typename VT>
constexpr int small_waves() { return R <= 2 || (R == 3 && sizeof(CT) == 4 && sizeof(VT) == 8) ? 4 : 3; }

// ------------------------------------------------------------------------------ batches

// Upfront digit histograms of every pass of every tensor of a batch.  Each workgroup takes a
// static range of stable tiles; the tensor's key spec and pass list are held in registers
// and reloaded only when the tensor changes, when the counts are flushed.  Also clears the
// look-back words of the first batched launch.
template <int R, typename CT>
__global__ void __launch_bounds__(256) k_hist_batch(BatchHistArgs a) {
    constexpr int U = kHistU, MAXP = 16;
    __shared__ uint32_t s_h[MAXP * kBins + kBins];  // + a spare block for items past the end
    __shared__ uint32_t s_pass[3][MAXP];            // per pass of the current tensor: lo, mask, sub-key
    const int tid = threadIdx.x, lane = tid & 63;
    const uint32_t spare = MAXP * kBins;
    for (int i = tid; i < MAXP * kBins; i += kBlock) s_h[i] = 0;
    const uint32_t per = (a.ntiles + gridDim.x - 1) / gridDim.x;
    const uint32_t t0 = blockIdx.x * per, t1 = min(a.ntiles, t0 + per);
    uint32_t cur = 0xFFFFFFFFu, n = 0, tile0 = 0;
    int npass = 0, nsub = 1, words = 0;
    uint32_t* hist = nullptr;
    uint64_t km[2][R];
    uint32_t ks[2][R], kd[2][R];
    const CT* src[R];
    auto flush = [&]() {
        sync_after_lds_atomics();
        for (int i = tid; i < words; i += kBlock) {
            const uint32_t c = s_h[i];
            if (c) atomicAdd(&hist[i], c);
            s_h[i] = 0;
        }
    };
    // One round of U records per thread: the key (one or two 64-bit sub-keys) as 32-bit halves,
    // then each pass's digit by one funnel shift; the run aggregation of consecutive lanes is
    // skipped for a pass whose first record of the round starts a run in at least half of the
    // lanes (unsorted digits), and either way every lane is counted once.
    auto round = [&](uint32_t base, uint32_t end) __attribute__((always_inline)) {
        uint32_t k[2][2][U];  // [sub-key][half][u]
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) k[q][0][u] = k[q][1][u] = 0;
#pragma unroll
        for (int m = 0; m < R; ++m) {
            if (!(km[0][m] | km[1][m])) continue;
            // the index is clamped to the tensor's last record instead of branching, so the U
            // loads are issued back to back; records past the end are counted into the spare
            // block below whatever their value
            CT c[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t e = base + u * kBlock + tid;
                c[u] = src[m][min(e, end - 1u)];
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                if (q >= nsub) break;  // keys wider than 64 bits only
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint64_t f = (((uint64_t)c[u] >> ks[q][m]) & km[q][m]) << kd[q][m];
                    k[q][0][u] |= (uint32_t)f;
                    k[q][1][u] |= (uint32_t)(f >> 32);
                }
            }
        }
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) ok[u] = base + u * kBlock + tid < end;
#pragma unroll 1
        for (int p = 0; p < npass; ++p) {
            const uint32_t plo = uni32(s_pass[0][p]), pmask = uni32(s_pass[1][p]);
            const bool hi_sub = uni32(s_pass[2][p]) != 0;
            uint32_t slot[U];
            if (hi_sub) {
                if (plo >= 32) {
#pragma unroll
                    for (int u = 0; u < U; ++u) slot[u] = k[1][1][u] >> (plo - 32);
                } else {
#pragma unroll
                    for (int u = 0; u < U; ++u) slot[u] = __builtin_amdgcn_alignbit(k[1][1][u], k[1][0][u], plo);
                }
            } else {
                if (plo >= 32) {
#pragma unroll
                    for (int u = 0; u < U; ++u) slot[u] = k[0][1][u] >> (plo - 32);
                } else {
#pragma unroll
                    for (int u = 0; u < U; ++u) slot[u] = __builtin_amdgcn_alignbit(k[0][1][u], k[0][0][u], plo);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) slot[u] = ok[u] ? ((slot[u] & pmask) | (uint32_t)(p * kBins)) : spare;
            // lane 0 always starts a run: the value "below" it is ~0, which no slot equals
            if (__popcll(ballot(from_lane_below(slot[0]) != slot[0])) >= 32) {
#pragma unroll
                for (int u = 0; u < U; ++u) atomicAdd(&s_h[slot[u]], 1u);
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) count_slot(s_h, slot[u], lane);
            }
        }
    };
    __syncthreads();
    for (uint32_t t = t0; t < t1; ++t) {
        const uint32_t j = a.tile_job[t];
        if (j != cur) {
            if (cur != 0xFFFFFFFFu) flush();
            cur = j;
            const BatchHistJob& J = a.jobs[j];
            npass = J.npass;
            nsub = J.nsub;
            n = J.n;
            tile0 = J.tile0;
            hist = J.hist;
            words = npass * kBins;
            const int r = J.r;
            if (tid < MAXP) {
                const bool on = tid < npass;
                s_pass[0][tid] = on ? (uint32_t)J.lo[tid] : 0u;
                s_pass[1][tid] = on ? (1u << J.bits[tid]) - 1u : 0u;
                s_pass[2][tid] = on ? (uint32_t)J.sub[tid] : 0u;
            }
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int m = 0; m < R; ++m) {
                    // the same for every lane: held in scalar registers
                    const bool on = q < nsub && m < r;
                    km[q][m] = on ? uni64(J.key[q].mask[m]) : 0ull;
                    ks[q][m] = on ? uni32((uint32_t)J.key[q].src_lo[m]) : 0u;
                    kd[q][m] = on ? uni32((uint32_t)J.key[q].dst[m]) : 0u;
                }
#pragma unroll
            for (int m = 0; m < R; ++m) src[m] = uni_ptr((const CT*)J.crd[m]);
            __syncthreads();
        }
        const uint32_t start = (t - tile0) * a.tile;
        const uint32_t end = min(n, start + a.tile);
        for (uint32_t base = start; base < end; base += kBlock * U) round(base, end);
        a.status_zero[(size_t)t * kBins + tid] = 0;
    }
    if (cur != 0xFFFFFFFFu) flush();
}

// Exclusive prefix of every 256-word block of digit counts, in place (one block per
// workgroup): the digit passes of a batch then read their digit offsets directly.
__global__ void __launch_bounds__(256) k_hist_prefix(uint32_t* hist) {
    __shared__ uint32_t s_tmp[kWaves];
    uint32_t* h = hist + (size_t)blockIdx.x * kBins;
    const uint32_t c = h[threadIdx.x];
    h[threadIdx.x] = block_excl_scan(c, s_tmp, nullptr);
}

// The same for the per-segment blocks of a segmented group: rows_per_seg blocks (one per pass)
// for every large segment that k_classify found.
__global__ void __launch_bounds__(256) k_hist_prefix_seg(uint32_t* hist, const uint64_t* large_ctl, uint32_t rows_per_seg) {
    __shared__ uint32_t s_tmp[kWaves];
    const uint32_t rows = (uint32_t)(*large_ctl >> 32) * rows_per_seg;
    for (uint32_t row = blockIdx.x; row < rows; row += gridDim.x) {
        uint32_t* h = hist + (size_t)row * kBins;
        const uint32_t c = h[threadIdx.x];
        h[threadIdx.x] = block_excl_scan(c, s_tmp, nullptr);
        __syncthreads();  // s_tmp is reused by the next row
    }
}

// One small tensor per workgroup, sorted entirely in LDS by its flattened key: LSD passes
// over the varying bits of every sub-key (least significant sub-key first), then every
// array written out in sorted order.
template <int R, typename CT, typename VT>
__global__ void __launch_bounds__(256) k_small_batch(const BatchSmallJob* __restrict__ jobs, uint32_t njobs) {
    constexpr int CAP = kSmallCap, ITEMS = CAP / kBlock;
    __shared__ uint64_t s_key[CAP];
    __shared__ uint16_t s_ia[CAP], s_ib[CAP];
    __shared__ uint32_t s_cnt[kWaves * kBins];
    __shared__ uint32_t s_bstart[kBins];
    __shared__ uint32_t s_tmp[2 * kWaves];
    __shared__ uint64_t s_red[2 * kWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (uint32_t jb = blockIdx.x; jb < njobs; jb += gridDim.x) {
        const BatchSmallJob& J = jobs[jb];
        const int r = J.r;
        const uint32_t L = J.n;
        CT c[R][ITEMS];
        VT v[ITEMS];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            if (m >= r) break;
            const CT* src = (const CT*)J.src_crd[m];
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t j = i * kBlock + tid;
                c[m][i] = j < L ? src[j] : CT(0);
            }
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t j = i * kBlock + tid;
            v[i] = j < L ? ((const VT*)J.src_val)[j] : VT(0);
            s_ia[j] = (uint16_t)j;
        }
        uint16_t* cur = s_ia;
        uint16_t* nxt = s_ib;
        for (int q = 0; q < J.nsub; ++q) {
            __syncthreads();
            uint64_t kor = 0, kand = ~0ull;
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t j = i * kBlock + tid;
                uint64_t kv = 0;
#pragma unroll
                for (int m = 0; m < R; ++m)
                    if (m < r && J.key[q].mask[m])
                        kv |= (((uint64_t)c[m][i] >> J.key[q].src_lo[m]) & J.key[q].mask[m]) << J.key[q].dst[m];
                s_key[j] = kv;
                if (j < L) {
                    kor |= kv;
                    kand &= kv;
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                kor |= __shfl_xor(kor, o, 64);
                kand &= __shfl_xor(kand, o, 64);
            }
            if (lane == 0) {
                s_red[wave] = kor;
                s_red[kWaves + wave] = kand;
            }
            __syncthreads();
            kor = 0;
            kand = ~0ull;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                kor |= s_red[w];
                kand &= s_red[kWaves + w];
            }
            const uint64_t vary = kor ^ kand;
            if (!vary) continue;
            const int lo = __builtin_ctzll(vary), hi = 63 - __builtin_clzll(vary);
            for (int sh = lo; sh <= hi; sh += 8) {
                const int nb = min(8, hi - sh + 1);
                const uint32_t dmask = (1u << nb) - 1u;
                if (((vary >> sh) & dmask) == 0) continue;
                for (int b = lane; b < kBins; b += 64) s_cnt[wave * kBins + b] = 0;
                uint32_t dg[ITEMS], lp[ITEMS];
                uint16_t sv[ITEMS];
                const uint32_t wb = (uint32_t)wave * 64u * ITEMS + lane;
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    const uint32_t j = wb + i * 64;
                    const bool ok = j < L;
                    sv[i] = ok ? cur[j] : 0;
                    dg[i] = ok ? (uint32_t)(s_key[sv[i]] >> sh) & dmask : 0;
                }
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    const bool ok = (wb + i * 64) < L;
                    const uint32_t d = dg[i];
                    uint64_t peers = ballot(ok);
                    for (int b = 0; b < nb; ++b) {
                        const bool bit = (d >> b) & 1u;
                        const uint64_t bb = ballot(bit);
                        peers &= bit ? bb : ~bb;
                    }
                    const uint32_t below = lanes_below(peers);
                    uint32_t old = 0;
                    if (ok) old = s_cnt[wave * kBins + d];
                    lp[i] = old + below;
                    if (ok && below == 0) s_cnt[wave * kBins + d] = old + (uint32_t)__popcll(peers);
                }
                __syncthreads();
                {
                    const uint32_t b = tid;
                    uint32_t run = 0;
#pragma unroll
                    for (int w = 0; w < kWaves; ++w) {
                        const uint32_t x = s_cnt[w * kBins + b];
                        s_cnt[w * kBins + b] = run;
                        run += x;
                    }
                    s_bstart[b] = block_excl_scan(run, s_tmp, nullptr);
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    if ((wb + i * 64) < L) {
                        const uint32_t d = dg[i];
                        nxt[lp[i] + s_bstart[d] + s_cnt[wave * kBins + d]] = sv[i];
                    }
                }
                __syncthreads();
                uint16_t* tmp = cur;
                cur = nxt;
                nxt = tmp;
            }
        }
        __syncthreads();
        uint16_t pm[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) pm[i] = cur[i * kBlock + tid];
#pragma unroll
        for (int m = 0; m <= R; ++m) {
            if (m < R && m >= r) continue;
            __syncthreads();
            if (m < R) {
                CT* st = (CT*)s_key;
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) st[i * kBlock + tid] = c[m][i];
                __syncthreads();
                CT* dst = (CT*)J.dst_crd[m];
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    const uint32_t j = i * kBlock + tid;
                    if (j < L) dst[j] = st[pm[i]];
                }
            } else {
                VT* st = (VT*)s_key;
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) st[i * kBlock + tid] = v[i];
                __syncthreads();
                VT* dst = (VT*)J.dst_val;
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    const uint32_t j = i * kBlock + tid;
                    if (j < L) dst[j] = st[pm[i]];
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------ validation

template <typename CT>
__global__ void __launch_bounds__(256) k_validate(ValidateArgs a) {
    uint32_t bad = 0;
    for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < a.n; e += gridDim.x * kBlock) {
        for (int m = 0; m < a.r; ++m) {
            const int64_t c = (int64_t)((const CT*)a.crd[m])[e];
            if (c < 0 || c >= a.ext[m]) bad |= 1u;
        }
        if (e > 0) {
            int cmp = 0;
            for (int i = 0; i < a.r && cmp == 0; ++i) {
                const CT* p = (const CT*)a.crd[a.in_order[i]];
                const int64_t x = (int64_t)p[e - 1], y = (int64_t)p[e];
                cmp = (x < y) ? -1 : (x > y ? 1 : 0);
            }
            if (cmp > 0) bad |= 2u;
        }
    }
    if (bad) atomicOr(a.flags, bad);
}

// ------------------------------------------------------------------------------ dispatch helpers

template <typename K>
int resident_blocks(K kernel) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, 0) != hipSuccess || per < 1) per = 1;
    return per * device_cu_count();
}

// One resident grid of a persistent digit-pass kernel (`resident` caches its occupancy).
template <typename K>
hipError_t launch_persistent(K kern, int& resident, const DigitArgs& a, hipStream_t s) {
    if (!resident) resident = resident_blocks(kern);
    const uint32_t grid = (uint32_t)std::max(1, std::min<int>((int)a.ntiles, resident));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int R, typename CT, typename VT, int ITEMS, int MODE, int PK = 0>
hipError_t digit_rs(const DigitArgs& a, hipStream_t s) {
    static int resident = 0;
    // packed words in (R = 1 with 64-bit words, or unpacking), and records of at most 20 bytes
    // in (at most 12 bytes of spill; the 3-mode int32/fp64 packing pass: 895 -> 837 us per
    // launch): three workgroups per CU
    constexpr bool kSmallRec = R * sizeof(CT) + sizeof(VT) <= 20;
    if constexpr (ITEMS == 16 && (PK == 2 || kSmallRec || (R == 1 && sizeof(CT) == 8)))
        return launch_persistent(k_digit3<R, CT, VT, ITEMS, MODE, PK>, resident, a, s);
    else
        return launch_persistent(k_digit<R, CT, VT, ITEMS, MODE, PK>, resident, a, s);
}

template <int R, typename CT, typename VT, int ITEMS>
hipError_t digit_ri(const DigitArgs& a, hipStream_t s) {
    if (a.seg_mode == 2) {
        if (a.pk == 1) return digit_rs<R, CT, VT, ITEMS, 2, 1>(a, s);
        if (a.pk == 2) return digit_rs<R, CT, VT, ITEMS, 2, 2>(a, s);
        return digit_rs<R, CT, VT, ITEMS, 2>(a, s);
    }
    if (a.seg_mode == 1) {
        if constexpr (ITEMS == 16) {  // packed segment passes: 16 records per thread only
            if (a.pk == 1) return digit_rs<R, CT, VT, ITEMS, 1, 1>(a, s);
            if (a.pk == 2) return digit_rs<R, CT, VT, ITEMS, 1, 2>(a, s);
        } else {
            if (a.pk) return hipErrorInvalidValue;
        }
        return digit_rs<R, CT, VT, ITEMS, 1>(a, s);
    }
    if (a.pk == 1) return digit_rs<R, CT, VT, ITEMS, 0, 1>(a, s);
    if (a.pk == 2) return digit_rs<R, CT, VT, ITEMS, 0, 2>(a, s);
    return digit_rs<R, CT, VT, ITEMS, 0>(a, s);
}

template <int R, typename CT, typename VT>
hipError_t digit_r(const DigitArgs& a, int items, hipStream_t s) {
    return items == 16 ? digit_ri<R, CT, VT, 16>(a, s) : digit_ri<R, CT, VT, 8>(a, s);
}

}  // namespace
}  // namespace qsd
