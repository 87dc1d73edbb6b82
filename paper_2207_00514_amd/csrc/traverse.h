// Nearest-other-component traversal (Algorithm 2 of the paper, with the
// subtree skipping of Optimization 1 and the component bound of
// Optimization 2), followed by stage A of the per-component minimum.
//
// For the query point i (Morton order) of component C the traversal finds
// the point j outside C minimising (D(i, j), j) -- for a fixed i this order
// equals the edge key (D, min(i, j), max(i, j)) -- among the points within
// the radius, which starts at the component bound ub[C] and shrinks to the
// best D found.  A child is skipped if its label is C (all its leaves are in
// C) or its box distance exceeds the radius; a deferred child is re-checked
// against the radius when it is taken back.  At the end the point offers
// (D bits, min(orig i, orig j)) to its component with a 64-bit atomicMin.
//
// Two launch shapes compute the same result:
//   variant 0  one lane per query, private stack (nearer child first);
//   variant 1  wavefront-cooperative: the 64 Morton-adjacent queries of a
//              wave walk the tree together, the wave visits a node if any of
//              its lanes needs it, node records are read once per wave
//              (uniform address), and the stack of (node, lane mask, box) is
//              shared by the wave in LDS.
#pragma once

#include "emst_kernels.h"

namespace emst {

template <int DIM>
struct TraverseArgs {
    const float* spts;
    const uint32_t* labels;
    const uint32_t* orig;
    const uint32_t* ub;
    const Rec<DIM>* recs;
    uint32_t root;
    int64_t n;
    uint32_t* cand_d;
    uint32_t* cand_j;
    uint64_t* compkey;
    uint32_t* compmax;
    Ctrl* ctrl;
    bool first;  // first round: every point is its own component
};

// Candidate order of Algorithm 2's leaf update, made strict: (D, j).
__device__ __forceinline__ bool better(float d, uint32_t j, float best_d, uint32_t best_j) {
    return d < best_d || (d == best_d && j < best_j);
}

template <bool COUNT>
__device__ __forceinline__ void flush_counts(Ctrl* ctrl, uint64_t internal, uint64_t leaf, uint64_t evals) {
    if (!COUNT) return;
    for (int off = 32; off > 0; off >>= 1) {
        internal += __shfl_xor(internal, off);
        leaf += __shfl_xor(leaf, off);
        evals += __shfl_xor(evals, off);
    }
    if (lane_id() == 0) {
        atomicAdd(&ctrl->internal_tests, (unsigned long long)internal);
        atomicAdd(&ctrl->leaf_tests, (unsigned long long)leaf);
        atomicAdd(&ctrl->dist_evals, (unsigned long long)evals);
    }
}

// Stage A of the component minimum.  In the first round the point is the
// whole component, so it writes the component's key (and, being the only
// candidate, its max index) directly.  Later the queries of a run of equal
// labels within the wave combine first and one lane per run updates the
// component with a 64-bit atomicMin.  Every lane of the wave must call it.
template <int DIM>
__device__ __forceinline__ void finish_query(const TraverseArgs<DIM>& a, int64_t i, uint32_t c, float best_d,
                                             uint32_t best_j) {
    const bool valid = i < a.n;
    const bool found = valid && best_j != kNone;
    uint64_t key = kKeyMax;
    if (valid) {
        const uint32_t oi = a.orig[i];
        const uint32_t db = found ? fbits(best_d) : kNone;
        a.cand_d[i] = db;
        a.cand_j[i] = best_j;
        if (found) key = ((uint64_t)db << 32) | (uint64_t)min(oi, best_j);
        if (a.first) {
            a.compkey[c] = key;
            a.compmax[c] = found ? max(oi, best_j) : kNone;
        }
    }
    if (a.first) return;
    bool run_end;
    key = wave_seg_min<uint64_t>(valid ? c : kNone, key, &run_end);
    if (valid && run_end && key != kKeyMax && key < load_relaxed64(&a.compkey[c]))
        atomicMin((unsigned long long*)&a.compkey[c], (unsigned long long)key);
}

// ---------------------------------------------------------------------------
// variant 0: one lane per query

template <int DIM, int STACK, bool COUNT>
__global__ __launch_bounds__(256) void k_traverse_lane(TraverseArgs<DIM> a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t n_int = 0, n_leaf = 0, n_eval = 0;
    uint32_t c_out = kNone, bj_out = kNone;
    float bd_out = INFINITY;
    if (i < a.n) {
        float p[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) p[k] = a.spts[i * DIM + k];
        const uint32_t c = a.labels[i];
        float radius = bitsf(a.ub[c]);
        float best_d = INFINITY;
        uint32_t best_j = kNone;
        uint32_t st_node[STACK];
        float st_d[STACK];
        int sp = 0;
        uint32_t node = a.root;
        // a query visits every internal node at most once
        for (int64_t guard = 0;; ++guard) {
            if (guard >= a.n) {
                atomicOr(&a.ctrl->error, kErrStack);
                break;
            }
            const Rec<DIM> r = a.recs[node];
            Child<DIM> ch[2];
            unpack<DIM>(r, ch[0], ch[1]);
            bool go[2] = {false, false};
            float dd[2] = {0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const bool leaf = (ch[s].ref & kLeafFlag) != 0u;
                if (COUNT) { if (leaf) ++n_leaf; else ++n_int; }
                if (ch[s].lab == c) continue;
                const float d = boxdist<DIM>(p, ch[s].lo, ch[s].hi);
                if (COUNT && leaf) ++n_eval;
                if (d > radius) continue;
                if (leaf) {
                    const uint32_t j = ch[s].ref & ~kLeafFlag;
                    if (better(d, j, best_d, best_j)) { best_d = d; best_j = j; radius = d; }
                } else {
                    go[s] = true;
                    dd[s] = d;
                }
            }
            if (go[0] && go[1]) {
                const int near = (dd[1] < dd[0]) ? 1 : 0;
                if (sp >= STACK) {
                    atomicOr(&a.ctrl->error, kErrStack);
                    break;
                }
                st_node[sp] = ch[1 - near].ref;
                st_d[sp] = dd[1 - near];
                ++sp;
                node = ch[near].ref;
            } else if (go[0]) {
                node = ch[0].ref;
            } else if (go[1]) {
                node = ch[1].ref;
            } else {
                bool found = false;
                while (sp > 0) {
                    --sp;
                    if (st_d[sp] <= radius) {
                        node = st_node[sp];
                        found = true;
                        break;
                    }
                }
                if (!found) break;
            }
        }
        c_out = c;
        bd_out = best_d;
        bj_out = best_j;
    }
    finish_query<DIM>(a, i, c_out, bd_out, bj_out);
    flush_counts<COUNT>(a.ctrl, n_int, n_leaf, n_eval);
}

// ---------------------------------------------------------------------------
// variant 1: wavefront-cooperative

template <int DIM, int STACK, bool COUNT>
__global__ __launch_bounds__(256) void k_traverse_wave(TraverseArgs<DIM> a) {
    constexpr int W = 4;  // waves per block
    __shared__ uint32_t s_node[W][STACK];
    __shared__ uint64_t s_mask[W][STACK];
    __shared__ float s_box[W][STACK][2 * DIM];
    const int w = threadIdx.x / 64, lane = lane_id();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < a.n;
    uint64_t n_int = 0, n_leaf = 0, n_eval = 0;
    float p[DIM];
    uint32_t c = kInvalid;
    float radius = -1.f;
#pragma unroll
    for (int k = 0; k < DIM; ++k) p[k] = 0.f;
    if (valid) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) p[k] = a.spts[i * DIM + k];
        c = a.labels[i];
        radius = bitsf(a.ub[c]);
    }
    float best_d = INFINITY;
    uint32_t best_j = kNone;
    uint64_t mask = __ballot(valid);
    uint32_t node = a.root;
    int sp = 0;
    const uint64_t me = 1ull << lane;
    for (int64_t guard = 0; mask; ++guard) {
        if (guard >= a.n) {
            if (lane == 0) atomicOr(&a.ctrl->error, kErrStack);
            break;
        }
        node = __builtin_amdgcn_readfirstlane(node);
        const Rec<DIM> r = a.recs[node];
        Child<DIM> ch[2];
        unpack<DIM>(r, ch[0], ch[1]);
        const bool in = (mask & me) != 0ull;
        bool go[2] = {false, false};
        float dd[2] = {0.f, 0.f};
        if (in) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const bool leaf = (ch[s].ref & kLeafFlag) != 0u;
                if (COUNT) { if (leaf) ++n_leaf; else ++n_int; }
                if (ch[s].lab == c) continue;
                const float d = boxdist<DIM>(p, ch[s].lo, ch[s].hi);
                if (COUNT && leaf) ++n_eval;
                if (d > radius) continue;
                if (leaf) {
                    const uint32_t j = ch[s].ref & ~kLeafFlag;
                    if (better(d, j, best_d, best_j)) { best_d = d; best_j = j; radius = d; }
                } else {
                    go[s] = true;
                    dd[s] = d;
                }
            }
        }
        const uint64_t m0 = __ballot(go[0]), m1 = __ballot(go[1]);
        if (m0 && m1) {
            // nearer-first by majority of the lanes that want both
            const uint64_t v0 = __ballot(go[0] && go[1] && dd[0] <= dd[1]);
            const uint64_t both = m0 & m1;
            const int first = (2 * __popcll(v0) >= __popcll(both)) ? 0 : 1;
            const Child<DIM>& f = ch[first];
            const Child<DIM>& o = ch[1 - first];
            if (sp >= STACK) {
                if (lane == 0) atomicOr(&a.ctrl->error, kErrStack);
                break;
            }
            if (lane == 0) {
                s_node[w][sp] = o.ref;
                s_mask[w][sp] = first ? m0 : m1;
#pragma unroll
                for (int k = 0; k < DIM; ++k) { s_box[w][sp][k] = o.lo[k]; s_box[w][sp][DIM + k] = o.hi[k]; }
            }
            ++sp;
            node = f.ref;
            mask = first ? m1 : m0;
        } else if (m0) {
            node = ch[0].ref;
            mask = m0;
        } else if (m1) {
            node = ch[1].ref;
            mask = m1;
        } else {
            mask = 0ull;
            while (sp > 0) {
                --sp;
                __builtin_amdgcn_wave_barrier();
                const uint64_t pm = s_mask[w][sp];
                float lo[DIM], hi[DIM];
#pragma unroll
                for (int k = 0; k < DIM; ++k) { lo[k] = s_box[w][sp][k]; hi[k] = s_box[w][sp][DIM + k]; }
                const bool keep = ((pm & me) != 0ull) && boxdist<DIM>(p, lo, hi) <= radius;
                const uint64_t km = __ballot(keep);
                if (km) {
                    node = s_node[w][sp];
                    mask = km;
                    break;
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    finish_query<DIM>(a, i, c, best_d, best_j);
    flush_counts<COUNT>(a.ctrl, n_int, n_leaf, n_eval);
}

// ---------------------------------------------------------------------------

template <int DIM, int STACK>
hipError_t launch_traverse_s(const TraverseArgs<DIM>& a, int variant, bool count, hipStream_t st) {
    const unsigned grid = (unsigned)((a.n + 255) / 256);
    if (variant == 1) {
        if (count) k_traverse_wave<DIM, STACK, true><<<grid, 256, 0, st>>>(a);
        else k_traverse_wave<DIM, STACK, false><<<grid, 256, 0, st>>>(a);
    } else {
        if (count) k_traverse_lane<DIM, STACK, true><<<grid, 256, 0, st>>>(a);
        else k_traverse_lane<DIM, STACK, false><<<grid, 256, 0, st>>>(a);
    }
    return hipGetLastError();
}

// The stack holds at most one deferred node per level below the root, so a
// capacity >= the tree height always suffices; the height of a binary radix
// tree over 64-bit codes and 31-bit indices is at most 96.
template <int DIM>
hipError_t launch_traverse(const TraverseArgs<DIM>& a, int height, int variant, bool count, hipStream_t st) {
    if (height <= 32) return launch_traverse_s<DIM, 32>(a, variant, count, st);
    if (height <= 64) return launch_traverse_s<DIM, 64>(a, variant, count, st);
    return launch_traverse_s<DIM, 96>(a, variant, count, st);
}

}  // namespace emst
