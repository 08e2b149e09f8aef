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
#include "kernels_impl.h"

namespace qsd {

hipError_t digit_launch_u32_u64(const DigitArgs& a, int r, int items, hipStream_t s);
hipError_t digit_launch_u32_u32(const DigitArgs& a, int r, int items, hipStream_t s);
hipError_t digit_launch_u64_u64(const DigitArgs& a, int r, int items, hipStream_t s);
hipError_t digit_launch_u64_u32(const DigitArgs& a, int r, int items, hipStream_t s);

namespace {

int g_cu = 0;

template <typename CT>
hipError_t hist_c(const HistArgs& a, int r, int grid, hipStream_t s) {
#define QSD_HIST_CASE(RR) \
    case RR: hipLaunchKernelGGL((k_hist<RR, CT>), dim3(grid), dim3(kBlock), 0, s, a); break;
    switch (r) {
        QSD_HIST_CASE(1) QSD_HIST_CASE(2) QSD_HIST_CASE(3) QSD_HIST_CASE(4)
        QSD_HIST_CASE(5) QSD_HIST_CASE(6) QSD_HIST_CASE(7) QSD_HIST_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef QSD_HIST_CASE
    return hipGetLastError();
}

}  // namespace

int device_cu_count() {
    if (!g_cu) {
        int dev = 0, cu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
            g_cu = cu;
        else
            g_cu = 256;
    }
    return g_cu;
}

hipError_t launch_zero(const ZeroArgs& a, hipStream_t s) {
    uint64_t mx = a.ctl ? kCtlWords : 0;
    for (int i = 0; i < 4; ++i)
        if (a.ptr[i]) mx = std::max(mx, a.words[i]);
    const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((mx + 255) / 256, 2048));
    hipLaunchKernelGGL(k_zero, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, uint64_t bytes, hipStream_t s) {
    if (!bytes) return hipSuccess;
    const bool aligned = (((uintptr_t)src | (uintptr_t)dst) & 15) == 0;
    const uint64_t n16 = aligned ? bytes / 16 : 0;
    const uint32_t grid = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>((bytes / 16 + 1023) / 1024, (uint64_t)device_cu_count() * 16));
    hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kBlock), 0, s, (const u32x4*)src, (u32x4*)dst, n16,
                       (const uint8_t*)src, (uint8_t*)dst, bytes);
    return hipGetLastError();
}

hipError_t launch_hist(const HistArgs& a, int r, int crd_bytes, int grid, hipStream_t s) {
    return crd_bytes == 8 ? hist_c<uint64_t>(a, r, grid, s) : hist_c<uint32_t>(a, r, grid, s);
}

hipError_t launch_digit(const DigitArgs& a, int r, int crd_bytes, int val_bytes, int items, hipStream_t s) {
    if (crd_bytes == 8)
        return val_bytes == 8 ? digit_launch_u64_u64(a, r, items, s) : digit_launch_u64_u32(a, r, items, s);
    return val_bytes == 8 ? digit_launch_u32_u64(a, r, items, s) : digit_launch_u32_u32(a, r, items, s);
}

hipError_t launch_boundary(const BoundArgs& a, int crd_bytes, hipStream_t s) {
    const uint32_t grid = (a.n + kDiscTile - 1) / kDiscTile;
    if (!grid) return hipSuccess;
    if (crd_bytes == 8)
        hipLaunchKernelGGL(k_boundary<uint64_t>, dim3(grid), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_boundary<uint32_t>, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tile_geo(const ClassArgs& a, uint32_t max_tiles, hipStream_t s) {
    if (!max_tiles) return hipSuccess;
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((max_tiles + kBlock - 1) / kBlock, (uint32_t)device_cu_count() * 4));
    hipLaunchKernelGGL(k_tile_geo, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_classify(const ClassArgs& a, uint32_t max_segments, hipStream_t s) {
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((max_segments + kBlock - 1) / kBlock, 4096));
    hipLaunchKernelGGL(k_classify, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <typename CT, typename VT>
hipError_t small_cv(const SmallArgs& a, uint32_t grid, hipStream_t s) {
#define QSD_SMALL_CASE(RR)                                                                                  \
    case RR:                                                                                                \
        hipLaunchKernelGGL((k_small<RR, CT, VT, small_waves<RR, CT, VT>()>), dim3(grid), dim3(kBlock), 0, s, a); \
        break;
    switch (a.r) {
        QSD_SMALL_CASE(1) QSD_SMALL_CASE(2) QSD_SMALL_CASE(3) QSD_SMALL_CASE(4)
        QSD_SMALL_CASE(5) QSD_SMALL_CASE(6) QSD_SMALL_CASE(7) QSD_SMALL_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef QSD_SMALL_CASE
    return hipGetLastError();
}

hipError_t launch_small(const SmallArgs& a, int crd_bytes, int val_bytes, uint32_t max_items, hipStream_t s) {
    if (!max_items) return hipSuccess;
    const int cu = device_cu_count();
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(max_items, (uint32_t)cu * 8));
    if (crd_bytes == 8)
        return val_bytes == 8 ? small_cv<uint64_t, uint64_t>(a, grid, s) : small_cv<uint64_t, uint32_t>(a, grid, s);
    return val_bytes == 8 ? small_cv<uint32_t, uint64_t>(a, grid, s) : small_cv<uint32_t, uint32_t>(a, grid, s);
}

hipError_t launch_digit_batch(const DigitArgs& a, int rmax, int crd_bytes, int val_bytes, int items,
                              hipStream_t s) {
    if (!a.ntiles) return hipSuccess;
    // batch mode reads r from the table; the template's R fixes the register footprint
    DigitArgs b = a;
    b.seg_mode = 2;
    return launch_digit(b, rmax, crd_bytes, val_bytes, items, s);
}

template <typename CT>
hipError_t hist_batch_c(const BatchHistArgs& a, int rmax, int grid, hipStream_t s) {
#define QSD_HB_CASE(RR) \
    case RR: hipLaunchKernelGGL((k_hist_batch<RR, CT>), dim3(grid), dim3(kBlock), 0, s, a); break;
    switch (rmax) {
        QSD_HB_CASE(1) QSD_HB_CASE(2) QSD_HB_CASE(3) QSD_HB_CASE(4)
        QSD_HB_CASE(5) QSD_HB_CASE(6) QSD_HB_CASE(7) QSD_HB_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef QSD_HB_CASE
    return hipGetLastError();
}

hipError_t launch_hist_batch(const BatchHistArgs& a, int rmax, int crd_bytes, int grid, hipStream_t s) {
    if (!a.ntiles) return hipSuccess;
    return crd_bytes == 8 ? hist_batch_c<uint64_t>(a, rmax, grid, s) : hist_batch_c<uint32_t>(a, rmax, grid, s);
}

hipError_t launch_hist_prefix(uint32_t* hist, uint32_t blocks, hipStream_t s) {
    if (!blocks) return hipSuccess;
    hipLaunchKernelGGL(k_hist_prefix, dim3(blocks), dim3(kBlock), 0, s, hist);
    return hipGetLastError();
}

hipError_t launch_hist_prefix_seg(uint32_t* hist, const uint64_t* large_ctl, uint32_t rows_per_seg,
                                  uint32_t max_rows, hipStream_t s) {
    if (!max_rows) return hipSuccess;
    const uint32_t grid = std::min<uint32_t>(max_rows, (uint32_t)device_cu_count() * 8);
    hipLaunchKernelGGL(k_hist_prefix_seg, dim3(grid), dim3(kBlock), 0, s, hist, large_ctl, rows_per_seg);
    return hipGetLastError();
}

template <typename CT, typename VT>
hipError_t small_batch_cv(const BatchSmallJob* jobs, uint32_t njobs, int rmax, hipStream_t s) {
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(njobs, (uint32_t)device_cu_count() * 8));
#define QSD_SB_CASE(RR) \
    case RR: hipLaunchKernelGGL((k_small_batch<RR, CT, VT>), dim3(grid), dim3(kBlock), 0, s, jobs, njobs); break;
    switch (rmax) {
        QSD_SB_CASE(1) QSD_SB_CASE(2) QSD_SB_CASE(3) QSD_SB_CASE(4)
        QSD_SB_CASE(5) QSD_SB_CASE(6) QSD_SB_CASE(7) QSD_SB_CASE(8)
        default: return hipErrorInvalidValue;
    }
#undef QSD_SB_CASE
    return hipGetLastError();
}

hipError_t launch_small_batch(const BatchSmallJob* jobs, uint32_t njobs, int rmax, int crd_bytes,
                              int val_bytes, hipStream_t s) {
    if (!njobs) return hipSuccess;
    if (crd_bytes == 8)
        return val_bytes == 8 ? small_batch_cv<uint64_t, uint64_t>(jobs, njobs, rmax, s)
                              : small_batch_cv<uint64_t, uint32_t>(jobs, njobs, rmax, s);
    return val_bytes == 8 ? small_batch_cv<uint32_t, uint64_t>(jobs, njobs, rmax, s)
                          : small_batch_cv<uint32_t, uint32_t>(jobs, njobs, rmax, s);
}

hipError_t launch_validate(const ValidateArgs& a, int crd_bytes, hipStream_t s) {
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((a.n + kBlock - 1) / kBlock, 4096));
    if (crd_bytes == 8)
        hipLaunchKernelGGL(k_validate<int64_t>, dim3(grid), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_validate<int32_t>, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace qsd
