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

// Sort n pairs stably by the 8-bit digits at `shifts` (least significant
// digit first).  Input in (k0, v0); (k1, v1) is scratch of the same size.
// On return *result_in_1 says whether the sorted pairs are in (k1, v1).
hipError_t radix_sort_pairs(hipStream_t stream, uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1,
                            uint32_t* hist, int64_t n, const int* shifts, int nshifts, int* result_in_1);

}  // namespace emst
