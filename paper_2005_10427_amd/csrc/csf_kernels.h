// Compressed sparse fiber (CSF) kernels: packing a sorted coordinate list into CSF, and
// expanding a CSF tensor back into coordinates (the two ends of a CSF -> CSF transposition).
//
// Layout (levels 1..r, level d holds the F_d fibers of the prefix sigma_1..sigma_d, F_0 = 1,
// F_r = nnz): crd[d-1] has F_d entries, the coordinate of each level-d fiber in mode sigma_d;
// pos[d-1] has F_{d-1} + 1 entries, and the children of level-(d-1) fiber p are the level-d
// fibers pos[d-1][p] .. pos[d-1][p+1]-1.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace qsd {

// records per tile of the CSF pack (the smallest tile: the look-back words are sized by it)
constexpr int kCsfTile = 2048;

struct CsfArgs {
    const void* crd[8];         // sorted coordinates in level order: crd[d] is mode sigma_{d+1}
    int32_t r;
    uint32_t n;
    void* pos[8];
    void* out_crd[8];
    int64_t* fiber_counts;      // F_0 .. F_r
    uint32_t* status;           // 8 words per tile (one per counted level), zeroed beforehand
    uint32_t* tile_counter;
    uint32_t* err;
};

// Expansion of a CSF tensor to coordinate arrays, one level per launch pair.  F_d is read from
// the arrays themselves: F_d = pos[d-1][F_{d-1}].
struct CsfExpandArgs {
    const void* pos[8];
    const void* crd[8];
    int32_t r;
    int32_t level;              // d: the level this launch expands (1 <= d < r)
    uint32_t n;                 // leaves
    uint8_t* flags;             // n bytes: 1 where a leaf is the first leaf of a level-d fiber
    uint32_t* status;           // one word per tile of kBoundTile leaves, zeroed beforehand
    uint32_t* tile_counter;
    void* out;                  // the level's coordinate of every leaf
    uint32_t* err;
};

// flags[first leaf of every level-d fiber] = 1 (flags zeroed beforehand)
hipError_t launch_csf_mark(const CsfExpandArgs& a, int crd_bytes, hipStream_t s);
// out[j] = crd[d-1][number of flags at or before j, minus 1]
hipError_t launch_csf_expand(const CsfExpandArgs& a, int crd_bytes, hipStream_t s);
// the CSF form of n sorted records of order r (1 <= r <= 8)
hipError_t launch_csf(const CsfArgs& a, int crd_bytes, hipStream_t s);

}  // namespace qsd
