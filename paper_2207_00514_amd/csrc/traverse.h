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
// Three launch shapes compute the same result:
//   variant 0  one lane per query, private stack (nearer child first);
//   variant 2  one lane per query, walking UP from the query's own leaf:
//              at every ancestor the other child's subtree is searched
//              top-down as in variant 0, and the walk stops at the first
//              ancestor whose Morton cell contains the ball of the current
//              radius (every point within the radius is then a leaf of that
//              ancestor, all of which have been searched);
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
    uint32_t* ub;  // written only by variant 11 (atomicMin)
    const Rec<DIM>* recs;
    uint32_t root;
    int64_t n;
    uint32_t* cand_d;
    uint32_t* cand_j;
    uint64_t* compkey;
    uint32_t* compmax;
    Ctrl* ctrl;
    bool first;  // first round: every point is its own component
    const uint32_t* leaf_parent;
    const Up* up;
    // batches: cloud of every sorted position and subtree root of every
    // cloud (kNone for a cloud of one point); null for one cloud
    const uint32_t* cloud_of;
    const uint32_t* cloud_root;
    const uint2* lab2;  // per record: component labels of its two children (rewritten every round)
    // per wave of 64 Morton-consecutive queries: the lowest common ancestor
    // of their leaves (one cloud only)
    const uint32_t* wave_lca;
    // mutual reachability: squared core distances by sorted position and by
    // original index (null for the Euclidean tree)
    const float* core_s;
    const float* core_o;
    const uint32_t* pos;  // sorted position of every original index
    // this round's query list (the points that still search, in Morton
    // order; length ctrl->qcount)
    const uint32_t* qlist;
};

// Where a top-down search of query i starts.
template <int DIM>
__device__ __forceinline__ uint32_t start_node(const TraverseArgs<DIM>& a, int64_t i) {
    return a.cloud_root ? a.cloud_root[a.cloud_of[i]] : a.root;
}

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
// Without a candidate the point stores `miss` as its cand_d (cand_j is
// kNone either way).
template <int DIM>
__device__ __forceinline__ void finish_query(const TraverseArgs<DIM>& a, int64_t i, uint32_t c, float best_d,
                                             uint32_t best_j, uint32_t miss = kNone) {
    const bool valid = i < a.n;
    const bool found = valid && best_j != kNone;
    uint64_t key = kKeyMax;
    if (valid) {
        const uint32_t oi = a.orig[i];
        const uint32_t db = found ? fbits(best_d) : miss;
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

// Top-down search of the subtree below internal node `node` (nearer child
// first, deferred children re-checked against the radius when popped).
template <int DIM, int STACK, bool COUNT>
__device__ __forceinline__ void descend(const TraverseArgs<DIM>& a, uint32_t node, const float* p, uint32_t c,
                                        float& radius, float& best_d, uint32_t& best_j, uint64_t& n_int,
                                        uint64_t& n_leaf, uint64_t& n_eval) {
    uint32_t st_node[STACK];
    float st_d[STACK];
    int sp = 0;
    // a search visits every internal node at most once
    for (int64_t guard = 0;; ++guard) {
        if (guard >= a.n) {
            atomicOr(&a.ctrl->error, kErrStack);
            return;
        }
        const Rec<DIM> r = a.recs[node];
        Child<DIM> ch[2];
        unpack<DIM>(r, ch[0], ch[1]);
        {
            const uint2 L = a.lab2[node];
            ch[0].lab = L.x;
            ch[1].lab = L.y;
        }
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
                return;
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
            if (!found) return;
        }
    }
}

template <int DIM, int STACK, bool COUNT>
__global__ __launch_bounds__(256) void k_traverse_lane(TraverseArgs<DIM> a) {
    if (a.ctrl->done) return;  // the round loop has already finished
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    uint64_t n_int = 0, n_leaf = 0, n_eval = 0;
    uint32_t c = kNone, best_j = kNone;
    float best_d = INFINITY;
    if (i < a.n) {
        float p[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) p[k] = a.spts[i * DIM + k];
        c = a.labels[i];
        float radius = bitsf(a.ub[c]);
        const uint32_t root = start_node<DIM>(a, i);
        if (root != kNone) descend<DIM, STACK, COUNT>(a, root, p, c, radius, best_d, best_j, n_int, n_leaf, n_eval);
    }
    finish_query<DIM>(a, i, c, best_d, best_j);
    flush_counts<COUNT>(a.ctrl, n_int, n_leaf, n_eval);
}

// ---------------------------------------------------------------------------
// variant 2: upward walk from the query's leaf with the Morton-cell stop

template <int DIM, int STACK, bool COUNT>
__global__ __launch_bounds__(256) void k_traverse_up(TraverseArgs<DIM> a) {
    if (a.ctrl->done) return;  // the round loop has already finished
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    uint64_t n_int = 0, n_leaf = 0, n_eval = 0;
    uint32_t c = kNone, best_j = kNone;
    float best_d = INFINITY;
    if (i < a.n) {
        float p[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) p[k] = a.spts[i * DIM + k];
        c = a.labels[i];
        float radius = bitsf(a.ub[c]);
        uint32_t st_node[STACK];
        float st_d[STACK];
        int sp = 0;
        // One flat loop; every iteration processes one record.  Climbing,
        // the record is the current ancestor's and only the child off the
        // walked path is tested (mask); descending, both children are.
        uint32_t link = a.leaf_parent[i];
        uint32_t anc = link >> 1;              // current ancestor
        uint32_t node = anc;                   // record processed next
        uint32_t mask = 2u >> (link & 1u);     // child 1 - side
        Up u = a.up[anc];                      // cell + parent of the ancestor, loaded with its record
        for (int64_t guard = 0;; ++guard) {
            if (guard >= 2 * a.n + 128) {
                atomicOr(&a.ctrl->error, kErrStack);
                break;
            }
            const Rec<DIM> r = a.recs[node];
            Child<DIM> ch[2];
            unpack<DIM>(r, ch[0], ch[1]);
            {
                const uint2 L = a.lab2[node];
                ch[0].lab = L.x;
                ch[1].lab = L.y;
            }
            bool go[2] = {false, false};
            float dd[2] = {0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                if (!((mask >> s) & 1u)) continue;
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
            mask = 3u;
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
                continue;
            }
            if (go[0] || go[1]) {
                node = go[0] ? ch[0].ref : ch[1].ref;
                continue;
            }
            bool found = false;
            while (sp > 0) {
                --sp;
                if (st_d[sp] <= radius) {
                    node = st_node[sp];
                    found = true;
                    break;
                }
            }
            if (found) continue;
            // The subtree off the path at `anc` is done, so every leaf of
            // `anc` has been searched.  A candidate j with D(p, j) <= radius
            // lies within sqrt(radius) (1 + 2^-22) of p on every axis, or
            // within ~5e-23 where squares underflow; r covers both and the
            // rounding of sqrtf.  If that ball lies in the Morton cell of
            // `anc`, every candidate is a leaf of `anc`: stop.
            const float rr = sqrtf(radius) * 1.000001f + 1e-22f;
            bool inside = (p[0] - rr >= u.a.x) && (p[0] + rr <= u.b.x);
            if (DIM > 1) inside = inside && (p[1 % DIM] - rr >= u.a.y) && (p[1 % DIM] + rr <= u.b.y);
            if (DIM > 2) inside = inside && (p[2 % DIM] - rr >= u.a.z) && (p[2 % DIM] + rr <= u.b.z);
            if (inside) break;
            link = fbits(u.a.w);
            if (link == kNone) break;
            anc = link >> 1;
            node = anc;
            mask = 2u >> (link & 1u);
            u = a.up[anc];
        }
    }
    finish_query<DIM>(a, i, c, best_d, best_j);
    flush_counts<COUNT>(a.ctrl, n_int, n_leaf, n_eval);
}

// ---------------------------------------------------------------------------
// variant 1: wavefront-cooperative

template <int DIM, int STACK, bool COUNT>
__global__ __launch_bounds__(256) void k_traverse_wave(TraverseArgs<DIM> a) {
    if (a.ctrl->done) return;  // the round loop has already finished
    constexpr int W = 4;  // waves per block
    __shared__ uint32_t s_node[W][STACK];
    __shared__ uint64_t s_mask[W][STACK];
    __shared__ float s_box[W][STACK][2 * DIM];
    const int w = threadIdx.x / 64, lane = lane_id();
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
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
        {
            const uint2 L = a.lab2[node];
            ch[0].lab = L.x;
            ch[1].lab = L.y;
        }
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
// variants 3 and 4: persistent waves with per-lane refill
//
// A query's cost varies a lot (how far its walk climbs, how many subtrees it
// opens), and a wave runs as long as its slowest lane.  Here a wave takes
// chunks of consecutive (Morton-ordered) queries and a lane that finishes
// takes the next query of the chunk at once, so lanes stay busy until the
// queue is empty.  Variant 3 searches top-down from the root (as variant 0),
// variant 4 walks up from the query's leaf (as variant 2).

template <int DIM>
__device__ __forceinline__ void finish_one(const TraverseArgs<DIM>& a, int64_t i, uint32_t c, float best_d,
                                           uint32_t best_j) {
    const uint32_t oi = a.orig[i];
    const bool found = best_j != kNone;
    const uint32_t db = found ? fbits(best_d) : kNone;
    a.cand_d[i] = db;
    a.cand_j[i] = best_j;
    const uint64_t key = found ? (((uint64_t)db << 32) | (uint64_t)min(oi, best_j)) : kKeyMax;
    if (a.first) {
        a.compkey[c] = key;
        a.compmax[c] = found ? max(oi, best_j) : kNone;
    } else if (found && key < load_relaxed64(&a.compkey[c])) {
        atomicMin((unsigned long long*)&a.compkey[c], (unsigned long long)key);
    }
}

template <int DIM, int STACK, bool COUNT, bool UPWARD>
__global__ __launch_bounds__(256) void k_traverse_pool(TraverseArgs<DIM> a) {
    if (a.ctrl->done) return;  // the round loop has already finished
    constexpr int64_t kChunk = 512;
    const int lane = lane_id();
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint64_t n_int = 0, n_leaf = 0, n_eval = 0;
    int64_t cpos = 0, cend = 0;    // wave-uniform: the current chunk of queries
    bool drained = false;          // wave-uniform: no chunk left
    bool active = false;
    int64_t i = 0;
    float p[DIM];
    uint32_t c = kNone, best_j = kNone, anc = 0, node = 0, mask = 3u;
    float radius = 0.f, best_d = INFINITY;
    uint32_t st_node[STACK];
    float st_d[STACK];
    int sp = 0;
    int64_t steps = 0;
    Up u;
    u.a = u.b = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < DIM; ++k) p[k] = 0.f;
    while (true) {
        // ---- refill idle lanes from the chunk
        const uint64_t idle = __ballot(!active);
        if (idle && !drained) {
            if (cpos >= cend) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(&a.ctrl->trav_next, (unsigned long long)kChunk);
                base = __shfl(base, 0);
                cpos = (int64_t)base;
                cend = min((int64_t)base + kChunk, a.n);
                drained = cpos >= a.n;
            }
            if (!drained) {
                const int64_t take = min((int64_t)__popcll(idle), cend - cpos);
                const int64_t rank = __popcll(idle & lt);
                if (!active && rank < take) {
                    i = cpos + rank;
#pragma unroll
                    for (int k = 0; k < DIM; ++k) p[k] = a.spts[i * DIM + k];
                    c = a.labels[i];
                    radius = bitsf(a.ub[c]);
                    best_d = INFINITY;
                    best_j = kNone;
                    sp = 0;
                    steps = 0;
                    if (UPWARD) {
                        const uint32_t link = a.leaf_parent[i];
                        anc = link >> 1;
                        node = anc;
                        mask = 2u >> (link & 1u);
                        u = a.up[anc];
                    } else {
                        node = a.root;
                        mask = 3u;
                    }
                    active = true;
                }
                cpos += take;
            }
        }
        if (__ballot(active) == 0ull) {
            if (drained) break;
            continue;
        }
        if (!active) continue;
        // a query processes every record at most twice (once climbing, once
        // descending), so this bound only trips on a malformed tree
        if (++steps > 2 * a.n + 256) {
            atomicOr(&a.ctrl->error, kErrStack);
            finish_one<DIM>(a, i, c, best_d, best_j);
            active = false;
            continue;
        }
        // ---- one record
        const Rec<DIM> r = a.recs[node];
        Child<DIM> ch[2];
        unpack<DIM>(r, ch[0], ch[1]);
        {
            const uint2 L = a.lab2[node];
            ch[0].lab = L.x;
            ch[1].lab = L.y;
        }
        bool go[2] = {false, false};
        float dd[2] = {0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (!((mask >> s) & 1u)) continue;
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
        mask = 3u;
        bool done = false;
        if (go[0] && go[1]) {
            const int near = (dd[1] < dd[0]) ? 1 : 0;
            if (sp >= STACK) {
                atomicOr(&a.ctrl->error, kErrStack);
                done = true;
            } else {
                st_node[sp] = ch[1 - near].ref;
                st_d[sp] = dd[1 - near];
                ++sp;
                node = ch[near].ref;
            }
        } else if (go[0] || go[1]) {
            node = go[0] ? ch[0].ref : ch[1].ref;
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
            if (!found) {
                if (!UPWARD) {
                    done = true;
                } else {
                    // the subtree off the path at `anc` is done: stop if the
                    // ball of the radius lies in the Morton cell of `anc`
                    const float rr = sqrtf(radius) * 1.000001f + 1e-22f;
                    bool inside = (p[0] - rr >= u.a.x) && (p[0] + rr <= u.b.x);
                    if (DIM > 1) inside = inside && (p[1 % DIM] - rr >= u.a.y) && (p[1 % DIM] + rr <= u.b.y);
                    if (DIM > 2) inside = inside && (p[2 % DIM] - rr >= u.a.z) && (p[2 % DIM] + rr <= u.b.z);
                    const uint32_t link = fbits(u.a.w);
                    if (inside || link == kNone) {
                        done = true;
                    } else {
                        anc = link >> 1;
                        node = anc;
                        mask = 2u >> (link & 1u);
                        u = a.up[anc];
                    }
                }
            }
        }
        if (done) {
            finish_one<DIM>(a, i, c, best_d, best_j);
            active = false;
        }
    }
    flush_counts<COUNT>(a.ctrl, n_int, n_leaf, n_eval);
}

// ---------------------------------------------------------------------------
// variants 5 and 6: the same searches as 0 and 2 with a tighter loop
//
// One record per iteration; both child distances are computed without
// branching, leaf updates and the choice of the next node are selects, and
// the stack lives in LDS (kLdsDepth entries per lane, laid out [depth][lane]
// so a wave's accesses fall in distinct banks) with the deeper entries
// spilled to a private array only when a search nests deeper than that.
//
// With WSTART (variant 10) the whole wave starts its top-down searches below
// the root, at one node S: from the lowest common ancestor of the wave's 64
// leaves it climbs until the Morton cell of S contains the ball of every
// lane's starting radius.  Every point a lane can admit lies in its ball,
// hence in that cell, hence among the leaves of S (a code-split node holds
// every point of its cell), so each search below S finds the candidate the
// search from the root finds.  The climb reads one uniform cell per step;
// the lanes stay in lockstep and skip the shared descent from the root.

// The ball of radius sqrt(radius) around p lies inside the (shrunk) Morton
// cell u; the radius is widened by more than the rounding of D and of the
// square root, so no point with D <= radius lies outside.
template <int DIM>
__device__ __forceinline__ bool ball_in_cell(const float* p, float rr, const Up& u) {
    bool inside = (p[0] - rr >= u.a.x) && (p[0] + rr <= u.b.x);
    if (DIM > 1) inside = inside && (p[1 % DIM] - rr >= u.a.y) && (p[1 % DIM] + rr <= u.b.y);
    if (DIM > 2) inside = inside && (p[2 % DIM] - rr >= u.a.z) && (p[2 % DIM] + rr <= u.b.z);
    return inside;
}

__device__ __forceinline__ float widen(float radius) { return sqrtf(radius) * 1.000001f + 1e-22f; }

// With MREACH the leaf metric is the mutual reachability M = max(core2(p),
// core2(q), D) (Section 3, "Non-Euclidean metrics"): candidates are
// admitted and ordered by (M, j), the radius follows the best M, and boxes
// are still pruned by their Euclidean distance, a lower bound of M.  A
// query whose own core distance exceeds the radius has no candidate.
//
// With SHARED (variant 11) the component bound is shared while the round
// runs (the dynamic form of Optimization 2): a lane that improves its best
// candidate lowers ub[C] with an atomicMin, and every lane re-reads ub[C]
// at every node.  ub[C] only ever holds D values of real outgoing edges of
// C, so it never drops below C's shortest one, whose point still admits it.
//
// With REUSE (variant 13) a point keeps last round's result where it still
// holds.  The components only grow, so the points outside a point's
// component only get fewer: if its candidate j is still outside, j is
// still the nearest in (D, j) order and the point skips the search; if it
// found nothing within last round's radius R, nothing outside lies within
// R, and it skips the search whenever the new radius does not exceed R.
// Such a point stores R in cand_d (with cand_j = kNone).  With LIST the
// lanes take the points of the query list, which holds exactly the points
// that must search (k_reuse_mark), so waves run full.  A wave of the list
// spans more than 64 positions; its climb starts at the start node of the
// 64 positions around its first point, an ancestor of that point's leaf,
// and the climb's stopping rule (every lane's ball inside the cell) still
// puts every lane's search region below the node it stops at.
template <int DIM, int STACK, bool COUNT, bool UPWARD, int kLdsDepth = 16, bool WSTART = false, bool MREACH = false,
          bool SHARED = false, bool REUSE = false, bool LIST = false>
__global__ __launch_bounds__(256) void k_traverse_fast(TraverseArgs<DIM> a) {
    if (a.ctrl->done) return;  // the round loop has already finished
    __shared__ uint2 lds[kLdsDepth][256];
    const int t = threadIdx.x;
    int64_t i;
    uint32_t first = 0;  // LIST: the wave's first point (its lane 0 holds the smallest position)
    if (LIST) {
        // the grid covers every point; only the blocks the list needs run
        const int64_t cnt = a.ctrl->qcount;
        const int64_t active = ((cnt + 255) / 256 + kXcds - 1) / kXcds * kXcds;
        if ((int64_t)blockIdx.x >= active) return;
        const int64_t li = xcd_block(blockIdx.x, active) * blockDim.x + t;
        i = li < cnt ? (int64_t)a.qlist[li] : a.n;
        first = __builtin_amdgcn_readfirstlane((uint32_t)i);
    } else {
        i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + t;
    }
    uint64_t n_int = 0, n_leaf = 0, n_eval = 0;
    uint32_t c = kNone, best_j = kNone, miss = kNone;
    float best_d = INFINITY;
    if (i < a.n) {
        float p[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) p[k] = a.spts[i * DIM + k];
        c = a.labels[i];
        float radius = bitsf(a.ub[c]);
        const float core_p = MREACH ? a.core_s[i] : 0.f;
        bool search = true;
        if (REUSE) {
            miss = fbits(radius);
            if (!a.first && !LIST) {
                const uint32_t pj = a.cand_j[i], pd = a.cand_d[i];
                if (pj != kNone) {
                    if (a.labels[a.pos[pj]] != c) {
                        best_d = bitsf(pd);
                        best_j = pj;
                        search = false;
                    }
                } else if (miss <= pd) {
                    miss = pd;
                    search = false;
                }
            }
        }
        uint2 spill[STACK];
        int sp = 0, base = 0;  // entries [0, base) spilled, [base, sp) in the LDS ring
        uint32_t node, mask, anc = 0;
        Up u;
        if (UPWARD) {
            const uint32_t link = a.leaf_parent[i];
            anc = link >> 1;
            node = anc;
            mask = 2u >> (link & 1u);
            u = a.up[anc];
        } else {
            node = start_node<DIM>(a, i);
            mask = (node == kNone || (MREACH && core_p > radius) || !search) ? 0u : 3u;
            if (WSTART && mask) {
                // wave-uniform climb; lanes past the end take no part
                const float rr = widen(radius);
                uint32_t s = a.wave_lca[(LIST ? (int64_t)first : i) >> 6];
                for (int h = 0; h < 160 && s != node; ++h) {
                    const Up cu = a.up[s];
                    if (__all(ball_in_cell<DIM>(p, rr, cu))) break;
                    const uint32_t link = fbits(cu.a.w);
                    s = link == kNone ? node : link >> 1;
                }
                node = s;
            }
        }
        for (int64_t guard = 0; mask; ++guard) {
            if (guard > 2 * a.n + 256) {
                atomicOr(&a.ctrl->error, kErrStack);
                break;
            }
            const Rec<DIM> r = a.recs[node];
            Child<DIM> c0, c1;
            unpack<DIM>(r, c0, c1);
            if (a.first) {
                // first round: every leaf is its own component, labelled by
                // its sorted position (the left leaf of record k is k, the
                // right one k + 1), and every internal node holds several
                c0.lab = (c0.ref & kLeafFlag) ? node : kInvalid;
                c1.lab = (c1.ref & kLeafFlag) ? node + 1u : kInvalid;
            } else {
                const uint2 L = a.lab2[node];
                c0.lab = L.x;
                c1.lab = L.y;
            }
            if (SHARED) radius = fminf(radius, bitsf(load_relaxed(&a.ub[c])));
            const float d0 = boxdist<DIM>(p, c0.lo, c0.hi);
            const float d1 = boxdist<DIM>(p, c1.lo, c1.hi);
            const bool in0 = (mask & 1u) && c0.lab != c;
            const bool in1 = (mask & 2u) && c1.lab != c;
            const bool l0 = (c0.ref & kLeafFlag) != 0u, l1 = (c1.ref & kLeafFlag) != 0u;
            if (COUNT) {
                n_leaf += ((mask & 1u) && l0) + ((mask & 2u) && l1);
                n_int += ((mask & 1u) && !l0) + ((mask & 2u) && !l1);
                n_eval += (in0 && l0) + (in1 && l1);
            }
            // leaf candidates: (D, j) order, radius follows the best.  D >= 0,
            // so (D bits, j) as one 64-bit integer has the same order.
            {
                float m0 = d0, m1 = d1;
                if (MREACH) {  // a leaf box is its point, so d0 / d1 are the exact D
                    const uint32_t j0 = c0.ref & ~kLeafFlag, j1 = c1.ref & ~kLeafFlag;
                    const float q0 = (in0 & l0 & (d0 <= radius)) ? a.core_o[j0] : 0.f;
                    const float q1 = (in1 & l1 & (d1 <= radius)) ? a.core_o[j1] : 0.f;
                    m0 = fmaxf(fmaxf(core_p, q0), d0);
                    m1 = fmaxf(fmaxf(core_p, q1), d1);
                }
                const uint64_t k0 = ((uint64_t)fbits(m0) << 32) | (c0.ref & ~kLeafFlag);
                const uint64_t k1 = ((uint64_t)fbits(m1) << 32) | (c1.ref & ~kLeafFlag);
                const bool b0 = in0 & l0 & (m0 <= radius);
                const bool b1 = in1 & l1 & (m1 <= radius);
                uint64_t bk = ((uint64_t)fbits(best_d) << 32) | best_j;
                bk = (b0 & (k0 < bk)) ? k0 : bk;
                bk = (b1 & (k1 < bk)) ? k1 : bk;
                const float nd = bitsf((uint32_t)(bk >> 32));
                if (SHARED && nd < radius) atomicMin(&a.ub[c], fbits(nd));
                best_d = nd;
                best_j = (uint32_t)bk;
                radius = fminf(radius, best_d);
            }
            const bool go0 = in0 && !l0 && d0 <= radius;
            const bool go1 = in1 && !l1 && d1 <= radius;
            mask = 3u;
            if (go0 && go1) {
                const bool near1 = d1 < d0;
                const uint2 far = make_uint2(near1 ? c0.ref : c1.ref, fbits(near1 ? d0 : d1));
                node = near1 ? c1.ref : c0.ref;
                if (sp - base == kLdsDepth) {  // ring full: move its oldest entry out
                    if (base >= STACK) {
                        atomicOr(&a.ctrl->error, kErrStack);
                        break;
                    }
                    spill[base] = lds[base % kLdsDepth][t];
                    ++base;
                }
                lds[sp % kLdsDepth][t] = far;
                ++sp;
                continue;
            }
            if (go0 || go1) {
                node = go0 ? c0.ref : c1.ref;
                continue;
            }
            bool found = false;
            while (sp > 0) {
                if (sp == base) {
                    // ring empty: move spilled entries back first (rare), so
                    // that every pop is a plain LDS read
                    const int back = base < kLdsDepth ? base : kLdsDepth;
                    for (int q = 1; q <= back; ++q) lds[(base - q) % kLdsDepth][t] = spill[base - q];
                    base -= back;
                }
                --sp;
                const uint2 e = lds[sp % kLdsDepth][t];
                if (bitsf(e.y) <= radius) {
                    node = e.x;
                    found = true;
                    break;
                }
            }
            if (found) continue;
            if (!UPWARD) break;
            // every leaf of `anc` has been searched: stop if the ball of the
            // radius lies in its Morton cell (see variant 2)
            const bool inside = ball_in_cell<DIM>(p, widen(radius), u);
            const uint32_t link = fbits(u.a.w);
            if (inside || link == kNone) break;
            anc = link >> 1;
            node = anc;
            mask = 2u >> (link & 1u);
            u = a.up[anc];
        }
    }
    finish_query<DIM>(a, i, c, best_d, best_j, miss);
    flush_counts<COUNT>(a.ctrl, n_int, n_leaf, n_eval);
}

// ---------------------------------------------------------------------------
// variant 12: two nodes per step
//
// The search of variant 10 (per-wave start, LDS ring stack) with a lane
// holding up to two pending nodes: it loads both records together, tests
// up to four children, keeps the two nearest admissible internal children
// as its next pair and defers the others (the farther first).  A step
// issues the loads of two nodes at once, so the chain of dependent record
// loads of the slowest lane, which sets the wave's time, is about half as
// long; the price is that the second node of a pair is opened before the
// first one's leaves could shrink the radius.  Every step pushes at most
// two entries and descends both nodes one level, so twice the tree height
// bounds the stack.

// Compare-exchange of (key, ref) pairs so that the smaller key comes first.
__device__ __forceinline__ void cmpx(uint32_t& ka, uint32_t& ra, uint32_t& kb, uint32_t& rb) {
    const bool sw = kb < ka;
    const uint32_t k = sw ? kb : ka, r = sw ? rb : ra;
    kb = sw ? ka : kb;
    rb = sw ? ra : rb;
    ka = k;
    ra = r;
}

template <int DIM, int STACK, bool COUNT, int kLdsDepth>
__global__ __launch_bounds__(256) void k_traverse_dual(TraverseArgs<DIM> a) {
    if (a.ctrl->done) return;  // the round loop has already finished
    __shared__ uint2 lds[kLdsDepth][256];
    const int t = threadIdx.x;
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + t;
    uint64_t n_int = 0, n_leaf = 0, n_eval = 0;
    uint32_t c = kNone, best_j = kNone;
    float best_d = INFINITY;
    if (i < a.n) {
        float p[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) p[k] = a.spts[i * DIM + k];
        c = a.labels[i];
        float radius = bitsf(a.ub[c]);
        constexpr int kCap = 2 * STACK + 4;
        uint2 spill[kCap];
        int sp = 0, base = 0;  // entries [0, base) spilled, [base, sp) in the LDS ring
        bool overflow = false;
        auto push = [&](uint32_t ref, uint32_t dbits) {
            if (sp - base == kLdsDepth) {  // ring full: move its oldest entry out
                if (base >= kCap) {
                    overflow = true;
                    return;
                }
                spill[base] = lds[base % kLdsDepth][t];
                ++base;
            }
            lds[sp % kLdsDepth][t] = make_uint2(ref, dbits);
            ++sp;
        };
        // the nearest deferred node still within the radius, or kNone
        auto pop = [&]() -> uint32_t {
            while (sp > 0) {
                if (sp == base) {  // ring empty: move spilled entries back first
                    const int back = base < kLdsDepth ? base : kLdsDepth;
                    for (int q = 1; q <= back; ++q) lds[(base - q) % kLdsDepth][t] = spill[base - q];
                    base -= back;
                }
                --sp;
                const uint2 e = lds[sp % kLdsDepth][t];
                if (bitsf(e.y) <= radius) return e.x;
            }
            return kNone;
        };
        uint32_t n0 = start_node<DIM>(a, i), n1 = kNone;
        if (n0 != kNone) {
            // per-wave start as in variant 10; lanes past the end take no part
            const uint32_t root = n0;
            const float rr = widen(radius);
            uint32_t s = a.wave_lca[i >> 6];
            for (int h = 0; h < 160 && s != root; ++h) {
                const Up cu = a.up[s];
                if (__all(ball_in_cell<DIM>(p, rr, cu))) break;
                const uint32_t link = fbits(cu.a.w);
                s = link == kNone ? root : link >> 1;
            }
            n0 = s;
        }
        for (int64_t guard = 0; n0 != kNone; ++guard) {
            if (guard > 2 * a.n + 256 || overflow) {
                atomicOr(&a.ctrl->error, kErrStack);
                break;
            }
            const bool two = n1 != kNone;
            Child<DIM> ch[4];
            {
                const Rec<DIM> r0 = a.recs[n0];
                const uint2 l0 = a.lab2[n0];
                unpack<DIM>(r0, ch[0], ch[1]);
                ch[0].lab = l0.x;
                ch[1].lab = l0.y;
                Rec<DIM> r1 = r0;
                uint2 l1 = l0;
                if (two) {
                    r1 = a.recs[n1];
                    l1 = a.lab2[n1];
                }
                unpack<DIM>(r1, ch[2], ch[3]);
                ch[2].lab = l1.x;
                ch[3].lab = l1.y;
            }
            float d[4];
            bool in[4], lf[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                d[q] = boxdist<DIM>(p, ch[q].lo, ch[q].hi);
                in[q] = (q < 2 || two) && ch[q].lab != c;
                lf[q] = (ch[q].ref & kLeafFlag) != 0u;
                if (COUNT) {
                    const bool v = q < 2 || two;
                    n_leaf += v && lf[q];
                    n_int += v && !lf[q];
                    n_eval += in[q] && lf[q];
                }
            }
            // leaf candidates in (D, j) order (a leaf box is its point)
            {
                uint64_t bk = ((uint64_t)fbits(best_d) << 32) | best_j;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint64_t kq = ((uint64_t)fbits(d[q]) << 32) | (ch[q].ref & ~kLeafFlag);
                    bk = (in[q] & lf[q] & (d[q] <= radius) & (kq < bk)) ? kq : bk;
                }
                best_d = bitsf((uint32_t)(bk >> 32));
                best_j = (uint32_t)bk;
                radius = fminf(radius, best_d);
            }
            // admissible internal children, nearest first
            uint32_t k[4], r[4];
            int cnt = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool go = in[q] && !lf[q] && d[q] <= radius;
                cnt += go;
                k[q] = go ? fbits(d[q]) : 0xFFFFFFFFu;
                r[q] = ch[q].ref;
            }
            cmpx(k[0], r[0], k[1], r[1]);
            cmpx(k[2], r[2], k[3], r[3]);
            cmpx(k[0], r[0], k[2], r[2]);
            cmpx(k[1], r[1], k[3], r[3]);
            cmpx(k[1], r[1], k[2], r[2]);
            if (cnt == 4) push(r[3], k[3]);
            if (cnt >= 3) push(r[2], k[2]);
            if (cnt >= 2) {
                n0 = r[0];
                n1 = r[1];
            } else if (cnt == 1) {
                n0 = r[0];
                n1 = pop();
            } else {
                n0 = pop();
                n1 = n0 == kNone ? kNone : pop();
            }
        }
    }
    finish_query<DIM>(a, i, c, best_d, best_j);
    flush_counts<COUNT>(a.ctrl, n_int, n_leaf, n_eval);
}

// ---------------------------------------------------------------------------
// Core distances (Section 4, "Mutual reachability distance"): for every
// sorted position i the k-th smallest D(i, j) over all j, the point itself
// (D = 0) included.  The k-th smallest D to the sorted positions within k-1
// of i (at least k points) bounds it from above; the search then keeps the
// K smallest D of every leaf it reaches in registers (K >= k, only the
// first k matter), prunes boxes farther than the running k-th value, and
// starts every wave below the root as variant 10 does.

template <int K>
__device__ __forceinline__ void knn_insert(float (&best)[K], float d) {
    if (!(d < best[K - 1])) return;
#pragma unroll
    for (int q = K - 1; q > 0; --q) best[q] = (d < best[q - 1]) ? best[q - 1] : ((d < best[q]) ? d : best[q]);
    best[0] = (d < best[0]) ? d : best[0];
}

template <int K>
__device__ __forceinline__ float knn_kth(const float (&best)[K], int k) {
    float r = best[0];
#pragma unroll
    for (int q = 1; q < K; ++q) r = (q == k - 1) ? best[q] : r;
    return r;
}

template <int DIM, int STACK, int K>
__global__ __launch_bounds__(256) void k_core_dist(TraverseArgs<DIM> a, int k, float* __restrict__ core_s,
                                                   float* __restrict__ core_o, float* __restrict__ core_out) {
    constexpr int kDepth = 8;
    __shared__ uint2 lds[kDepth][256];
    const int t = threadIdx.x;
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + t;
    if (i >= a.n) return;
    float p[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) p[c] = a.spts[i * DIM + c];
    float best[K];
#pragma unroll
    for (int q = 0; q < K; ++q) best[q] = INFINITY;
    {
        const int64_t w0 = i - (k - 1) > 0 ? i - (k - 1) : 0;
        const int64_t w1 = i + (k - 1) < a.n - 1 ? i + (k - 1) : a.n - 1;
        for (int64_t q = w0; q <= w1; ++q) {
            float o[DIM];
#pragma unroll
            for (int c = 0; c < DIM; ++c) o[c] = a.spts[q * DIM + c];
            knn_insert<K>(best, sqdist<DIM>(p, o));
        }
    }
    float radius = knn_kth<K>(best, k);
#pragma unroll
    for (int q = 0; q < K; ++q) best[q] = INFINITY;
    uint32_t node = a.root;
    {  // wave-uniform climb from the wave's leaf LCA (lanes past the end take no part)
        const float rr = widen(radius);
        uint32_t s = a.wave_lca[i >> 6];
        for (int h = 0; h < 160 && s != node; ++h) {
            const Up cu = a.up[s];
            if (__all(ball_in_cell<DIM>(p, rr, cu))) break;
            const uint32_t link = fbits(cu.a.w);
            s = link == kNone ? node : link >> 1;
        }
        node = s;
    }
    uint2 spill[STACK];
    int sp = 0, base = 0;
    for (int64_t guard = 0;; ++guard) {
        if (guard > 2 * a.n + 256) {
            atomicOr(&a.ctrl->error, kErrStack);
            break;
        }
        const Rec<DIM> r = a.recs[node];
        Child<DIM> c0, c1;
        unpack<DIM>(r, c0, c1);
        const float d0 = boxdist<DIM>(p, c0.lo, c0.hi);
        const float d1 = boxdist<DIM>(p, c1.lo, c1.hi);
        const bool l0 = (c0.ref & kLeafFlag) != 0u, l1 = (c1.ref & kLeafFlag) != 0u;
        if (l0 && d0 <= radius) knn_insert<K>(best, d0);
        if (l1 && d1 <= radius) knn_insert<K>(best, d1);
        radius = fminf(radius, knn_kth<K>(best, k));
        const bool go0 = !l0 && d0 <= radius;
        const bool go1 = !l1 && d1 <= radius;
        if (go0 && go1) {
            const bool near1 = d1 < d0;
            const uint2 far = make_uint2(near1 ? c0.ref : c1.ref, fbits(near1 ? d0 : d1));
            node = near1 ? c1.ref : c0.ref;
            if (sp - base == kDepth) {
                if (base >= STACK) {
                    atomicOr(&a.ctrl->error, kErrStack);
                    break;
                }
                spill[base] = lds[base % kDepth][t];
                ++base;
            }
            lds[sp % kDepth][t] = far;
            ++sp;
            continue;
        }
        if (go0 || go1) {
            node = go0 ? c0.ref : c1.ref;
            continue;
        }
        bool found = false;
        while (sp > 0) {
            if (sp == base) {  // as in k_traverse_fast
                const int back = base < kDepth ? base : kDepth;
                for (int q = 1; q <= back; ++q) lds[(base - q) % kDepth][t] = spill[base - q];
                base -= back;
            }
            --sp;
            const uint2 e = lds[sp % kDepth][t];
            if (bitsf(e.y) <= radius) {
                node = e.x;
                found = true;
                break;
            }
        }
        if (!found) break;
    }
    const float core = knn_kth<K>(best, k);
    const uint32_t oi = a.orig[i];
    core_s[i] = core;
    core_o[oi] = core;
    if (core_out) core_out[oi] = core;
}

template <int DIM, int STACK>
hipError_t launch_core_s(const TraverseArgs<DIM>& a, int k, float* core_s, float* core_o, float* core_out,
                         hipStream_t st) {
    const unsigned grid = (unsigned)(((a.n + 255) / 256 + kXcds - 1) / kXcds * kXcds);
    if (k <= 4) k_core_dist<DIM, STACK, 4><<<grid, 256, 0, st>>>(a, k, core_s, core_o, core_out);
    else if (k <= 8) k_core_dist<DIM, STACK, 8><<<grid, 256, 0, st>>>(a, k, core_s, core_o, core_out);
    else if (k <= 16) k_core_dist<DIM, STACK, 16><<<grid, 256, 0, st>>>(a, k, core_s, core_o, core_out);
    else if (k <= 32) k_core_dist<DIM, STACK, 32><<<grid, 256, 0, st>>>(a, k, core_s, core_o, core_out);
    else k_core_dist<DIM, STACK, 64><<<grid, 256, 0, st>>>(a, k, core_s, core_o, core_out);
    return hipGetLastError();
}

template <int DIM>
hipError_t launch_core(const TraverseArgs<DIM>& a, int height, int k, float* core_s, float* core_o, float* core_out,
                       hipStream_t st) {
    if (height <= 32) return launch_core_s<DIM, 32>(a, k, core_s, core_o, core_out, st);
    if (height <= 64) return launch_core_s<DIM, 64>(a, k, core_s, core_o, core_out, st);
    return launch_core_s<DIM, 96>(a, k, core_s, core_o, core_out, st);
}

// ---------------------------------------------------------------------------

template <int DIM, int STACK>
hipError_t launch_traverse_s(const TraverseArgs<DIM>& a, int variant, bool count, hipStream_t st) {
    // a multiple of the XCD count, for the XCD-contiguous block mapping
    const unsigned grid = (unsigned)(((a.n + 255) / 256 + kXcds - 1) / kXcds * kXcds);
    if (a.core_s) {  // mutual reachability: the loop and start of variant 10 (with the reuse of 13)
        if (variant == 13 && a.qlist) {
            if (count) k_traverse_fast<DIM, STACK, true, false, 8, true, true, false, true, true><<<grid, 256, 0, st>>>(a);
            else k_traverse_fast<DIM, STACK, false, false, 8, true, true, false, true, true><<<grid, 256, 0, st>>>(a);
        } else if (variant == 13) {
            if (count) k_traverse_fast<DIM, STACK, true, false, 8, true, true, false, true><<<grid, 256, 0, st>>>(a);
            else k_traverse_fast<DIM, STACK, false, false, 8, true, true, false, true><<<grid, 256, 0, st>>>(a);
        } else {
            if (count) k_traverse_fast<DIM, STACK, true, false, 8, true, true><<<grid, 256, 0, st>>>(a);
            else k_traverse_fast<DIM, STACK, false, false, 8, true, true><<<grid, 256, 0, st>>>(a);
        }
        return hipGetLastError();
    }
    if (variant == 1) {
        if (count) k_traverse_wave<DIM, STACK, true><<<grid, 256, 0, st>>>(a);
        else k_traverse_wave<DIM, STACK, false><<<grid, 256, 0, st>>>(a);
    } else if (variant == 2) {
        if (count) k_traverse_up<DIM, STACK, true><<<grid, 256, 0, st>>>(a);
        else k_traverse_up<DIM, STACK, false><<<grid, 256, 0, st>>>(a);
    } else if (variant == 5) {
        if (count) k_traverse_fast<DIM, STACK, true, false><<<grid, 256, 0, st>>>(a);
        else k_traverse_fast<DIM, STACK, false, false><<<grid, 256, 0, st>>>(a);
    } else if (variant == 6) {
        if (count) k_traverse_fast<DIM, STACK, true, true><<<grid, 256, 0, st>>>(a);
        else k_traverse_fast<DIM, STACK, false, true><<<grid, 256, 0, st>>>(a);
    } else if (variant == 7) {
        if (count) k_traverse_fast<DIM, STACK, true, false, 8><<<grid, 256, 0, st>>>(a);
        else k_traverse_fast<DIM, STACK, false, false, 8><<<grid, 256, 0, st>>>(a);
    } else if (variant == 8) {
        if (count) k_traverse_fast<DIM, STACK, true, false, 4><<<grid, 256, 0, st>>>(a);
        else k_traverse_fast<DIM, STACK, false, false, 4><<<grid, 256, 0, st>>>(a);
    } else if (variant == 9) {
        if (count) k_traverse_fast<DIM, STACK, true, true, 8><<<grid, 256, 0, st>>>(a);
        else k_traverse_fast<DIM, STACK, false, true, 8><<<grid, 256, 0, st>>>(a);
    } else if (variant == 10) {
        if (count) k_traverse_fast<DIM, STACK, true, false, 8, true><<<grid, 256, 0, st>>>(a);
        else k_traverse_fast<DIM, STACK, false, false, 8, true><<<grid, 256, 0, st>>>(a);
    } else if (variant == 13 && a.cloud_of) {
        // batches: the start of variant 7 (each cloud's root) with the reuse
        if (a.qlist) {
            if (count) k_traverse_fast<DIM, STACK, true, false, 8, false, false, false, true, true><<<grid, 256, 0, st>>>(a);
            else k_traverse_fast<DIM, STACK, false, false, 8, false, false, false, true, true><<<grid, 256, 0, st>>>(a);
        } else {
            if (count) k_traverse_fast<DIM, STACK, true, false, 8, false, false, false, true><<<grid, 256, 0, st>>>(a);
            else k_traverse_fast<DIM, STACK, false, false, 8, false, false, false, true><<<grid, 256, 0, st>>>(a);
        }
    } else if (variant == 13 && a.qlist) {
        if (count) k_traverse_fast<DIM, STACK, true, false, 8, true, false, false, true, true><<<grid, 256, 0, st>>>(a);
        else k_traverse_fast<DIM, STACK, false, false, 8, true, false, false, true, true><<<grid, 256, 0, st>>>(a);
    } else if (variant == 13) {
        if (count) k_traverse_fast<DIM, STACK, true, false, 8, true, false, false, true><<<grid, 256, 0, st>>>(a);
        else k_traverse_fast<DIM, STACK, false, false, 8, true, false, false, true><<<grid, 256, 0, st>>>(a);
    } else if (variant == 12) {
        if (count) k_traverse_dual<DIM, STACK, true, 8><<<grid, 256, 0, st>>>(a);
        else k_traverse_dual<DIM, STACK, false, 8><<<grid, 256, 0, st>>>(a);
    } else if (variant == 11) {
        if (count) k_traverse_fast<DIM, STACK, true, false, 8, true, false, true><<<grid, 256, 0, st>>>(a);
        else k_traverse_fast<DIM, STACK, false, false, 8, true, false, true><<<grid, 256, 0, st>>>(a);
    } else if (variant == 3 || variant == 4) {
        // persistent: enough waves to fill every CU several times over
        const unsigned pgrid = std::min<unsigned>(grid, 2048u);
        if (variant == 3) {
            if (count) k_traverse_pool<DIM, STACK, true, false><<<pgrid, 256, 0, st>>>(a);
            else k_traverse_pool<DIM, STACK, false, false><<<pgrid, 256, 0, st>>>(a);
        } else {
            if (count) k_traverse_pool<DIM, STACK, true, true><<<pgrid, 256, 0, st>>>(a);
            else k_traverse_pool<DIM, STACK, false, true><<<pgrid, 256, 0, st>>>(a);
        }
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
