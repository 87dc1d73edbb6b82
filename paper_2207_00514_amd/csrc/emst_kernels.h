// Kernels of the single-tree Boruvka EMST (gfx950).  Every kernel is a
// template over the dimension so coordinate loops unroll.
#pragma once

#include "emst_common.h"

namespace emst {

// Device control block: reductions, counters and flags of one build.
struct Ctrl {
    uint32_t bb_min[3];      // order-preserving encoding of float (see ord_enc)
    uint32_t bb_max[3];
    uint32_t nonfinite;
    uint32_t root;
    uint32_t height;
    uint32_t ncomp_next;
    uint32_t edge_count;
    uint32_t error;          // kErr* bits
    uint64_t key_or;
    uint64_t key_and;
    unsigned long long internal_tests;
    unsigned long long leaf_tests;
    unsigned long long dist_evals;
    unsigned long long touched;     // counting runs: node records the traversals loaded, each once per round
    uint32_t long_ties;      // the edge order met a run of equal keys too long to fix in place
    uint32_t dup_codes;      // sorted positions whose Morton code equals the previous one
    uint32_t done;           // the round loop has reached its target: later round kernels return at once
    uint32_t qcount;         // length of this round's query list
    uint32_t rounds_run;     // rounds that ran before the loop reached its target
    uint32_t pad;
};

// Search radius of a round from the second on (traversal variant 13): the
// component bound, lowered to the shortest candidate already offered to the
// component while components are small (fewer than kTightSize points on
// average).  Any radius at least the component's shortest outgoing edge
// gives the same tree; a point that finds nothing keeps its radius as proof
// for later rounds, and once components are large their radii grow round by
// round, so the looser bound keeps such points from searching again every
// round.  The count of the round's components is the one k_relabel left in
// the control block.
constexpr uint64_t kTightSize = 2048;

constexpr uint32_t kErrStack = 1u;
constexpr uint32_t kErrNoEdge = 2u;
constexpr uint32_t kErrJump = 4u;

// float <-> uint32 whose unsigned order equals the float order (finite values)
__device__ __forceinline__ uint32_t ord_enc(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float ord_dec(uint32_t u) {
    uint32_t b = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
    float f;
    __builtin_memcpy(&f, &b, 4);
    return f;
}

__device__ __forceinline__ bool tight_radius(const Ctrl* ctrl, int64_t n) {
    return (uint64_t)ctrl->ncomp_next * kTightSize > (uint64_t)n;
}

}  // namespace emst
