// Stable LSD radix sort of (uint64 key, uint32 value) pairs on the device.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace emst {

constexpr int kRadixMaxBlocks = 1024;

struct RadixPlan {
    int blocks;
    int64_t tiles_per_block;
};

RadixPlan radix_plan(int64_t n);

// Count table the sort needs: uint32[256 * kRadixMaxBlocks] plus 256 row totals.
constexpr size_t radix_hist_elems() { return (size_t)256 * kRadixMaxBlocks + 256; }

// From kRadixOneMin keys on, a pass is one launch with decoupled look-back
// (the one-sweep scheme); it needs per-tile digit counts as scratch after the
// count table.
constexpr int64_t kRadixOneMin = (int64_t)1 << 22;
constexpr int kRadixOneTile = 256 * 16;
// uint32 elements of the scratch `hist` must hold for n keys (every caller
// passes at least this many).
inline size_t radix_scratch_elems(int64_t n) {
    if (n < kRadixOneMin) return radix_hist_elems();
    const size_t tiles = (size_t)((n + kRadixOneTile - 1) / kRadixOneTile);
    return radix_hist_elems() + 3 * 8 * 256 + 64 + 2 * tiles * 256;
}

// Sort n pairs stably by the 8-bit digits at `shifts` (least significant
// digit first).  Input in (k0, v0); (k1, v1) is scratch of the same size.
// On return *result_in_1 says whether the sorted pairs are in (k1, v1).
hipError_t radix_sort_pairs(hipStream_t stream, uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1,
                            uint32_t* hist, int64_t n, const int* shifts, int nshifts, int* result_in_1);

}  // namespace emst
