// Device-wide exclusive scan and stable LSD radix sort of (u64 key, u32 value)
// pairs whose count lives in device memory (no host synchronisation).
#pragma once
#include "common.h"

namespace xgs {

constexpr int kScanItems = 2048;   // elements per scan block (256 threads x 8)
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;     // rounds of 256 items per sort block (2, 4, 6, 12, 16 measured slower)
constexpr int kSortItems = kSortThreads * kSortRounds;

// Inclusive prefix sum of v over the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

inline int64_t scan_blocks(int64_t n) { return (n + kScanItems - 1) / kScanItems; }
inline int64_t sort_blocks(int64_t cap) { return (cap + kSortItems - 1) / kSortItems; }

// Exclusive scan of in[0..n) (u32) into out (u64); *total = sum, and when
// cap >= 0: *count = sum (0 if sum > cap), *status = sum > cap.
// partials must hold scan_blocks(n) + 1 entries.  zero_p (optional): zero_n
// u32 words to clear, done by the scan's own launches when possible.
xgs_status exclusive_scan_u32(const uint32_t* in, int64_t n, uint64_t* out, uint64_t* partials,
                              int64_t* total, int64_t cap, int64_t* count, int32_t* status,
                              uint32_t* zero_p, int64_t zero_n, hipStream_t stream);

// Up to this many scan blocks the apply pass sums the block totals before
// its own block itself (no separate partials pass).
constexpr int64_t kFusedScanBlocks = 4096;

// The first pass of exclusive_scan_u32 alone: partials[b] = the sum of block
// b (kScanItems values), zero_p[0..zero_n) cleared by the same launch; for a
// caller that applies the prefix itself.
xgs_status scan_block_totals(const uint32_t* in, int64_t n, uint64_t* partials, uint32_t* zero_p, int64_t zero_n,
                             hipStream_t stream);

// Stable LSD radix sort of the first *count pairs (count <= cap) on key bits
// [0, key_bits), in passes of radix_digit_bits(key_bits, cap) bits: 9 when
// that takes fewer passes than 8 (5 instead of 6 at 41-45 bits) and cap needs
// at most kRadix9MaxBlocks sort blocks, else 8 (past that size the 9-bit
// scatter's shorter write runs per digit cost more than the pass they save:
// 1M keys 0.168 -> 0.159 ms, 3M keys 0.359 -> 0.384 ms for the tile sort).
// Pairs start in (k0, v0); the sorted result is left in (k0, v0) if
// radix_passes is even, otherwise in (k1, v1); hist must hold
// radix_hist_words(cap) u32.
constexpr int64_t kRadix9MaxBlocks = 768;
int radix_digit_bits(int key_bits, int64_t cap);
int radix_passes(int key_bits, int64_t cap);
constexpr int64_t kRadixBinsMax = 512;
inline int64_t radix_hist_words(int64_t cap) {
    int64_t nb = sort_blocks(cap) > 0 ? sort_blocks(cap) : 1;
    return kRadixBinsMax * (nb + 1);
}
xgs_status radix_sort(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1,
                      const int64_t* count, int64_t cap, int key_bits, uint32_t* hist,
                      hipStream_t stream);

// Fills n u32 with a value (used instead of hipMemsetAsync so that the calls
// stay safe to record into graphs).
xgs_status fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t stream);
xgs_status fill_f32(float* p, int64_t n, float v, hipStream_t stream);

// Zeroes k <= 4 ranges of n[j] 32-bit words at p[j] (any 4-byte alignment) in
// one launch; ranges with n[j] = 0 are skipped.
struct ZeroRanges {
    uint32_t* p[4];
    int64_t n[4];
    int k;
};
xgs_status zero_ranges(const ZeroRanges& r, hipStream_t stream);

// ranges[2 s] = first, ranges[2 s + 1] = last + 1 position of segment
// s = keys[i] >> shift among the first *count sorted keys; segments absent
// from the keys keep whatever the caller filled in.
xgs_status segment_ranges(const uint64_t* keys, const int64_t* count, int64_t cap, int shift,
                          uint32_t* ranges, hipStream_t stream);

}  // namespace xgs
