// Kernel argument blocks and launchers (host side).  All positions are 32-bit: nnz is
// limited to QSD_MAX_NNZ = 2^30 so that a scan status word can hold a 30-bit count.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace qsd {

constexpr int kBlock = 256;        // threads per workgroup (4 wave64)
constexpr int kBins = 256;         // 8-bit digits: one bin per thread
constexpr int kSmallCap = 4096;    // records one workgroup sorts in LDS
constexpr int kTinyLen = 2048;     // segments up to this length are packed by region
constexpr int kRegion = 2048;      // region width for packing tiny segments
constexpr int kBoundTile = 4096;   // elements per tile of the boundary scan
constexpr int kDiscTile = 32768;   // records per tile of bucket discovery
constexpr int kCtlWords = 1024;    // control block (counters, sizes, flags), 4 KB

// control block word offsets (uint32 unless noted)
enum CtlSlot {
    kCtlErr = 0,        // device status bits
    kCtlValid = 1,      // validation result bits
    kCtlNb = 2,         // number of segments
    kCtlNMed = 3,       // medium segments
    kCtlLarge = 4,      // uint64 at words 4-5: (large segments << 32) | large tiles
    kCtlBoundCnt = 8,   // tile counter of the boundary scan
    kCtlMagic = 9,      // kCtlStickyMagic once kCtlErr holds accumulated status bits
    kCtlPassCnt = 16,   // tile counters, kPassCounters per digit pass launch
};
constexpr int kPassCounters = 8;  // a global pass's tile queues
// The status bits of kCtlErr accumulate over calls (the library clears them when the host reads
// them).  A fresh workspace holds arbitrary bytes: the first call that finds the magic word
// missing clears the bits and writes it.
constexpr uint32_t kCtlStickyMagic = 0x51534431u;

struct DevKey {
    uint64_t mask[8];
    int32_t src_lo[8];
    int32_t dst[8];
};

// Items per thread of the digit pass (8 or 16): a whole record per item lives in registers,
// so wide records take fewer items.  `pref` (0 = automatic) is a tuning override.
inline int digit_items(int r, int crd_bytes, int val_bytes, int pref = 0) {
    if (pref == 8 || pref == 16) return pref;
    const int words = r * (crd_bytes / 4) + val_bytes / 4;
    return words <= 6 ? 16 : 8;
}

// The part of one key mode inside a digit window.  The mode's field occupies bits
// [dst, dst + width) of the composite key and comes from bits [src_lo, src_lo + width) of the
// coordinate; the digit is bits [lo, lo + nbits) of the key.  Their overlap is coordinate bits
// [rs, rs + ln), which land at digit bit ls (ln = 0: the mode adds nothing to this digit).
struct DigitSlice {
    uint32_t rs, ln, ls;
};
__host__ __device__ inline DigitSlice digit_slice(int dst, int src_lo, int width, int lo, int nbits) {
    const int a = dst > lo ? dst : lo;
    const int e = (dst + width) < (lo + nbits) ? (dst + width) : (lo + nbits);
    if (e <= a) return DigitSlice{0u, 0u, 0u};
    return DigitSlice{(uint32_t)(src_lo + a - dst), (uint32_t)(e - a), (uint32_t)(a - lo)};
}

// One tensor's digit pass inside a batched launch (device table, one entry per tensor).
struct BatchPass {
    const void* src_crd[8];
    const void* src_val;
    void* dst_crd[8];
    void* dst_val;
    DevKey key;
    int32_t lo, bits;
    int32_t r;
    uint32_t n;
    const uint32_t* hist;       // exclusive prefix of this pass's 256 digit counts over the tensor
    uint32_t tile0;             // first (stable) tile id of the tensor
    int32_t active;             // 0: the tensor has no pass in this launch
    uint32_t pad[2];
    // packed records: the layout of the 64-bit words (as DigitArgs::pk_pos / pk_mask)
    int32_t pk_pos[8];
    uint64_t pk_mask[8];
};

struct DigitArgs {
    const void* src_crd[8];
    const void* src_val;
    void* dst_crd[8];
    void* dst_val;
    DevKey key;
    int32_t lo, bits;           // digit = (key >> lo) & ((1 << bits) - 1)
    uint32_t n;                 // global mode: number of records
    uint32_t ntiles;            // global mode: tiles; segment mode: upper bound (grid sizing)
    int32_t seg_mode;           // 0: one segment [0, n); 1: the large-segment list
    uint32_t hist_stride;       // segment mode: words between two segments' histograms
    const uint32_t* hist;       // this pass's digit histogram (segment mode: of segment 0)
    uint32_t* status;           // look-back words of this pass, kBins per tile
    uint32_t* status_next;      // zeroed for the next pass (may be null)
    uint32_t* tile_counter;     // kPassCounters tile queues (one queue below 2048 tiles)
    const uint64_t* large_ctl;  // segment mode
    const uint32_t* tile_map;   // four words per tile, 16-byte aligned.  Segment mode: first
                                // record, records, the segment's first tile, large segment;
                                // batch mode, per launch tile: stable tile id, tensor, first
                                // record, records
    const BatchPass* batch;     // batch mode: this launch's table
    uint32_t* err;
    // Packed records (global and batch modes).  pk = 1: read the r coordinate arrays, write one
    // array of 64-bit words sum_m (crd_m & pk_mask[m]) << pk_pos[m] (dst_crd[0]); pk = 2:
    // read such words (src_crd[0]; the digit is taken from the word directly) and write the r
    // coordinate arrays back.  pk = 0: records as given.  In batch mode pk is the record layout
    // of every tensor in the launch and the word layout comes from each tensor's table entry.
    int32_t pk;
    int32_t pk_pos[8];
    uint64_t pk_mask[8];
};

// Upfront histograms of a batch: one job per (tensor, sub-key), a static tile range each.
struct BatchHistJob {
    const void* crd[8];
    DevKey key[2];              // sub-keys, least significant first
    int32_t r, nsub, npass;
    int32_t lo[16];
    int32_t bits[16];
    int32_t sub[16];            // sub-key of every pass
    uint32_t n;
    uint32_t tile0;             // first stable tile of the tensor
    uint32_t* hist;             // npass * 256 counts
};

struct BatchHistArgs {
    const BatchHistJob* jobs;
    const uint32_t* tile_job;   // stable tile -> job
    uint32_t ntiles;
    uint32_t tile;              // records per tile
    uint32_t* status_zero;      // look-back words of the first launch, zeroed here
};

// A whole small tensor sorted in LDS by its flattened key (up to 2 sub-keys).
struct BatchSmallJob {
    const void* src_crd[8];
    const void* src_val;
    void* dst_crd[8];
    void* dst_val;
    DevKey key[2];
    int32_t key_bits[2];
    int32_t nsub;
    int32_t r;
    uint32_t n;
    uint32_t pad;
};

struct HistArgs {
    const void* crd[8];
    DevKey key;
    int32_t npass;
    int32_t lo[16];
    int32_t bits[16];
    uint32_t n;                 // global mode
    int32_t seg_mode;
    uint32_t tile;              // segment mode: records per tile
    uint32_t* hist;             // global: npass*kBins; segment: per large segment
    uint32_t hist_stride;
    uint32_t* status_zero;      // status words of the first pass, zeroed here
    uint32_t status_words;      // global mode: words to zero
    const uint64_t* large_ctl;
    const uint4* tile_geo;      // segment mode: as written by k_classify
};

struct BoundArgs {
    const void* crd[8];
    int32_t nprefix;
    int32_t prefix[8];
    // Bucket reuse: when the previous group kept a prefix that this group's prefix extends,
    // its segment starts are still segment starts here.  prev_bits (one bit per record, set at
    // the previous group's segment starts) stands for the comparison of the first nskip prefix
    // modes.  bits_out (may alias prev_bits) receives this group's starts the same way.
    const uint64_t* prev_bits;
    int32_t nskip;
    uint64_t* bits_out;
    uint32_t n;
    uint32_t* seg_start;        // nb + 1 entries written (seg_start[nb] = n)
    uint32_t* region_seg;       // first segment starting in each kRegion-wide region (+ nb)
    uint32_t* status;           // one word per tile, zeroed beforehand
    uint32_t* tile_counter;
    uint32_t* nb_out;
    uint32_t* err;
};

struct ClassArgs {
    const uint32_t* seg_start;
    const uint32_t* nb;
    uint32_t tile;              // digit-pass tile of the large path
    uint32_t* nmed;
    uint4* geo;                 // per work item of the LDS sort: first record, records, first and
                                // end segment (regions first, then the medium segments)
    const uint32_t* region_seg;
    uint32_t nregions;
    uint64_t* large_ctl;
    uint4* large;               // per large segment: first record, records, first tile
    uint4* tile_geo;            // per large-segment tile: first record, records, the segment's
                                // first tile, large segment
    uint32_t* seg_hist;         // zeroed per large segment
    uint32_t hist_stride;
};

struct SmallArgs {
    const void* src_crd[8];
    const void* src_val;
    void* dst_crd[8];
    void* dst_val;
    int32_t r;
    DevKey key;                 // whole group key (<= 52 bits)
    int32_t key_bits;
    uint32_t n;
    uint32_t nregions;
    const uint32_t* seg_start;
    const uint32_t* nmed;
    const uint4* geo;           // work items as written by k_classify
};

struct ZeroArgs {
    uint32_t* ptr[4];
    uint64_t words[4];
    uint32_t* ctl;              // control block: every word cleared except kCtlErr / kCtlMagic
};

struct ValidateArgs {
    const void* crd[8];
    int32_t r;
    int64_t ext[8];
    int32_t in_order[8];
    uint32_t n;
    uint32_t* flags;            // bit 0: out of range, bit 1: unsorted
};

hipError_t launch_zero(const ZeroArgs& a, hipStream_t s);
hipError_t launch_copy(const void* src, void* dst, uint64_t bytes, hipStream_t s);
hipError_t launch_hist(const HistArgs& a, int r, int crd_bytes, int grid, hipStream_t s);
hipError_t launch_digit(const DigitArgs& a, int r, int crd_bytes, int val_bytes, int items, hipStream_t s);
hipError_t launch_digit_batch(const DigitArgs& a, int rmax, int crd_bytes, int val_bytes, int items,
                              hipStream_t s);
hipError_t launch_hist_batch(const BatchHistArgs& a, int rmax, int crd_bytes, int grid, hipStream_t s);
// counts -> exclusive prefix, in place, for `blocks` consecutive blocks of 256 words
hipError_t launch_hist_prefix(uint32_t* hist, uint32_t blocks, hipStream_t s);
hipError_t launch_hist_prefix_seg(uint32_t* hist, const uint64_t* large_ctl, uint32_t rows_per_seg,
                                  uint32_t max_rows, hipStream_t s);
hipError_t launch_small_batch(const BatchSmallJob* jobs, uint32_t njobs, int rmax, int crd_bytes,
                              int val_bytes, hipStream_t s);
hipError_t launch_boundary(const BoundArgs& a, int crd_bytes, hipStream_t s);
hipError_t launch_classify(const ClassArgs& a, uint32_t max_segments, hipStream_t s);
hipError_t launch_tile_geo(const ClassArgs& a, uint32_t max_tiles, hipStream_t s);
hipError_t launch_small(const SmallArgs& a, int crd_bytes, int val_bytes, uint32_t max_items,
                        hipStream_t s);
hipError_t launch_validate(const ValidateArgs& a, int crd_bytes, hipStream_t s);

int device_cu_count();

}  // namespace qsd
