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
// Launch shapes (emst_set_traversal) compute the same result; the kept ones
// are variant 0 (one lane per query, private stack, nearer child first)
// and the tighter loop of k_traverse_fast below (variants 5, 7, 8, 10,
// 11 and 13, the default).
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
    // each point's candidate: its sorted position (the leaf children of
    // record k are positions k and k + 1), written with cand_d / cand_j
    uint32_t* cand_p;
    // the first round: the successor of every component (the component of
    // its one point's candidate), written by the traversal itself
    uint32_t* succ;
    // this round's query list (the points that still search, in Morton
    // order; length ctrl->qcount)
    const uint32_t* qlist;
    // counting runs: one flag per node record, set when a search loads it
    uint8_t* touched;
    // variant 13 without a list from the third round on: per point, 1 if
    // it keeps last round's candidate (already offered to its component by
    // k_round_prep); null otherwise
    const uint8_t* kept;
    // the second round: every point's last candidate (its nearest point)
    // joined its component in the first round
    bool all_absorbed;
    // launch shape (host side): LDS stack ring entries per lane of variant
    // 13 (4, 8 or 16)
    int lds_depth;
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
                                             uint32_t best_j, uint32_t best_p, uint32_t miss = kNone,
                                             bool offer = true) {
    const bool valid = i < a.n;
    const bool found = valid && best_j != kNone;
    uint64_t key = kKeyMax;
    if (valid) {
        const uint32_t oi = a.orig[i];
        const uint32_t db = found ? fbits(best_d) : miss;
        a.cand_d[i] = db;
        a.cand_j[i] = best_j;
        if (found && offer) {  // (a kept candidate's position is already stored)
            key = ((uint64_t)db << 32) | (uint64_t)min(oi, best_j);
            a.cand_p[i] = best_p;
        }
        if (a.first) {
            // the point is its component (label = position = i), and a
            // point's label is its position
            a.compkey[c] = key;
            a.compmax[c] = found ? max(oi, best_j) : kNone;
            a.succ[c] = found ? best_p : c;
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
                                        float& radius, float& best_d, uint32_t& best_j, uint32_t& best_p,
                                        uint64_t& n_int, uint64_t& n_leaf, uint64_t& n_eval) {
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
        if (COUNT) a.touched[node] = 1;
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
                if (better(d, j, best_d, best_j)) {
                    best_d = d;
                    best_j = j;
                    best_p = node + (uint32_t)s;  // leaf children of record k: positions k, k + 1
                    radius = d;
                }
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
    uint32_t c = kNone, best_j = kNone, best_p = kNone;
    float best_d = INFINITY;
    if (i < a.n) {
        float p[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) p[k] = a.spts[i * DIM + k];
        c = a.labels[i];
        float radius = bitsf(a.ub[c]);
        const uint32_t root = start_node<DIM>(a, i);
        if (root != kNone) descend<DIM, STACK, COUNT>(a, root, p, c, radius, best_d, best_j, best_p, n_int, n_leaf,
                                       n_eval);
    }
    finish_query<DIM>(a, i, c, best_d, best_j, best_p);
    flush_counts<COUNT>(a.ctrl, n_int, n_leaf, n_eval);
}

// ---------------------------------------------------------------------------
// variants 5, 7, 8, 10, 11, 13: the search of variant 0 with a tighter loop
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
// Such a point stores R in cand_d (with cand_j = kNone).  If its candidate,
// at D = pd, has joined its component, no point now outside is nearer than
// pd (each was outside before), so when pd exceeds the radius nothing is
// admissible: the point skips the search and stores the float below pd as
// its R.  The radius itself is the component bound, lowered to the
// shortest candidate already offered to the component while components
// are small (tight_radius).  With LIST the
// lanes take the points of the query list, which holds exactly the points
// that must search (k_reuse_mark), so waves run full.  A wave of the list
// spans more than 64 positions; its climb starts at the start node of the
// 64 positions around its first point, an ancestor of that point's leaf,
// and the climb's stopping rule (every lane's ball inside the cell) still
// puts every lane's search region below the node it stops at.
template <int DIM, int STACK, bool COUNT, int kLdsDepth = 16, bool WSTART = false, bool MREACH = false,
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
    uint32_t c = kNone, best_j = kNone, best_p = kNone, miss = kNone;
    bool offer = true;  // false: a kept candidate, already offered
    float best_d = INFINITY;
    if (i < a.n) {
        float p[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) p[k] = a.spts[i * DIM + k];
        c = a.labels[i];
        float radius = bitsf(a.ub[c]);
        if (REUSE && !a.first && tight_radius(a.ctrl, a.n)) {
            // the kept candidates are real outgoing edges of C too: the
            // shortest one offered tightens the radius (k_round_prep offered
            // them before this launch from the third round on; in the second
            // round the key holds what searches have offered so far)
            const uint64_t ck = load_relaxed64(&a.compkey[c]);
            if (ck != kKeyMax) radius = fminf(radius, bitsf((uint32_t)(ck >> 32)));
        }
        const float core_p = MREACH ? a.core_s[i] : 0.f;
        bool search = true;
        if (REUSE) {
            miss = fbits(radius);
            // a listed point searches (k_reuse_mark decided with this radius)
            if (!a.first && !LIST) {
                const uint32_t pj = a.cand_j[i], pd = a.cand_d[i];
                if (pj != kNone) {
                    if (!a.all_absorbed && a.kept[i]) {  // offered by k_round_prep
                        best_d = bitsf(pd);
                        best_j = pj;
                        search = false;
                        offer = false;
                    } else if (pd > miss) {
                        // absorbed, but nothing outside is nearer than pd,
                        // which lies beyond the radius
                        miss = pd - 1u;
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
        uint32_t node = start_node<DIM>(a, i);
        uint32_t mask = (node == kNone || (MREACH && core_p > radius) || !search) ? 0u : 3u;
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
        // Every iteration processes one node or pops one deferred node, so
        // lanes that discard stale entries do not hold the others in a loop
        // of their own.  A search visits each internal node once and pops
        // each deferred node once.
        bool have = mask != 0u;  // a node to process this iteration
        for (int64_t guard = 0;; ++guard) {
            if (guard > 4 * a.n + 256) {
                atomicOr(&a.ctrl->error, kErrStack);
                break;
            }
            if (have) {
            const Rec<DIM> r = a.recs[node];
            if (COUNT) a.touched[node] = 1;
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
            const bool in0 = c0.lab != c;
            const bool in1 = c1.lab != c;
            const bool l0 = (c0.ref & kLeafFlag) != 0u, l1 = (c1.ref & kLeafFlag) != 0u;
            if (COUNT) {
                n_leaf += l0 + l1;
                n_int += !l0 + !l1;
                n_eval += (in0 && l0) + (in1 && l1);
            }
            // leaf candidates: (D, j) order, radius follows the best.  D >= 0,
            // so (D bits, j) as one 64-bit integer has the same order.  (Most
            // nodes a search visits have no leaf child: the whole block is
            // skipped unless some lane of the wave meets one.)
            if ((in0 & l0) | (in1 & l1)) {
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
                const bool t0 = b0 & (k0 < bk);
                bk = t0 ? k0 : bk;
                const bool t1 = b1 & (k1 < bk);
                bk = t1 ? k1 : bk;
                // the leaf children of record k are sorted positions k, k + 1
                best_p = t1 ? node + 1u : (t0 ? node : best_p);
                const float nd = bitsf((uint32_t)(bk >> 32));
                if (SHARED && nd < radius) atomicMin(&a.ub[c], fbits(nd));
                best_d = nd;
                best_j = (uint32_t)bk;
                radius = nd < radius ? nd : radius;  // (no NaN: every coordinate is finite)
            }
            const bool go0 = in0 && !l0 && d0 <= radius;
            const bool go1 = in1 && !l1 && d1 <= radius;
            // the next node is a select; only deferring the farther child
            // of two branches (few branches keep the wave's scalar
            // instructions, which manage the lane masks, down)
            const bool both = go0 && go1;
            const bool near1 = d1 < d0;
            const uint2 far = make_uint2(near1 ? c0.ref : c1.ref, fbits(near1 ? d0 : d1));
            node = both ? (near1 ? c1.ref : c0.ref) : (go0 ? c0.ref : c1.ref);
            have = go0 || go1;
            if (both) {
                if (sp - base == kLdsDepth) {  // ring full: move its oldest entry out
                    if (base < STACK) {
                        spill[base] = lds[(unsigned)base % kLdsDepth][t];
                        ++base;
                    } else {  // (cannot happen: the stack holds a tree's height) end the search
                        atomicOr(&a.ctrl->error, kErrStack);
                        have = false;
                        sp = base = 0;
                    }
                }
                if (have) {
                    lds[(unsigned)sp % kLdsDepth][t] = far;
                    ++sp;
                }
            }
            }
            if (!have) {
                if (sp == 0) break;
                if (sp == base) {
                    // ring empty: move spilled entries back first (rare), so
                    // that every pop is a plain LDS read
                    const int back = base < kLdsDepth ? base : kLdsDepth;
                    for (int q = 1; q <= back; ++q) lds[(unsigned)(base - q) % kLdsDepth][t] = spill[base - q];
                    base -= back;
                }
                --sp;
                const uint2 e = lds[(unsigned)sp % kLdsDepth][t];
                // else the next iteration pops again
                have = bitsf(e.y) <= radius;
                node = have ? e.x : node;
            }
        }
    }
    finish_query<DIM>(a, i, c, best_d, best_j, best_p, miss, offer);
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
                spill[base] = lds[(unsigned)base % kDepth][t];
                ++base;
            }
            lds[(unsigned)sp % kDepth][t] = far;
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
                for (int q = 1; q <= back; ++q) lds[(unsigned)(base - q) % kDepth][t] = spill[base - q];
                base -= back;
            }
            --sp;
            const uint2 e = lds[(unsigned)sp % kDepth][t];
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
#define EMST_FAST(...)                                                                  \
    do {                                                                                \
        if (count) k_traverse_fast<DIM, STACK, true, __VA_ARGS__><<<grid, 256, 0, st>>>(a);  \
        else k_traverse_fast<DIM, STACK, false, __VA_ARGS__><<<grid, 256, 0, st>>>(a);       \
    } while (0)
    //            kLdsDepth, WSTART, MREACH, SHARED, REUSE, LIST
    if (a.core_s) {  // mutual reachability: the loop and start of variant 10 (with the reuse of 13)
        if (variant == 13 && a.qlist) EMST_FAST(8, true, true, false, true, true);
        else if (variant == 13) EMST_FAST(8, true, true, false, true, false);
        else EMST_FAST(8, true, true);
    } else if (variant == 5) {
        EMST_FAST(16);
    } else if (variant == 7) {
        EMST_FAST(8);
    } else if (variant == 8) {
        EMST_FAST(4);
    } else if (variant == 10) {
        EMST_FAST(8, true);
    } else if (variant == 11) {
        EMST_FAST(8, true, false, true);
    } else if (variant == 13 && a.cloud_of) {
        // batches: the start of variant 7 (each cloud's root) with the reuse
        if (a.lds_depth == 4) {
            if (a.qlist) EMST_FAST(4, false, false, false, true, true);
            else EMST_FAST(4, false, false, false, true, false);
        } else if (a.lds_depth == 16) {
            if (a.qlist) EMST_FAST(16, false, false, false, true, true);
            else EMST_FAST(16, false, false, false, true, false);
        } else {
            if (a.qlist) EMST_FAST(8, false, false, false, true, true);
            else EMST_FAST(8, false, false, false, true, false);
        }
    } else if (variant == 13) {
        if (a.lds_depth == 4) {
            if (a.qlist) EMST_FAST(4, true, false, false, true, true);
            else EMST_FAST(4, true, false, false, true, false);
        } else if (a.lds_depth == 16) {
            if (a.qlist) EMST_FAST(16, true, false, false, true, true);
            else EMST_FAST(16, true, false, false, true, false);
        } else {
            if (a.qlist) EMST_FAST(8, true, false, false, true, true);
            else EMST_FAST(8, true, false, false, true, false);
        }
    } else {
        if (count) k_traverse_lane<DIM, STACK, true><<<grid, 256, 0, st>>>(a);
        else k_traverse_lane<DIM, STACK, false><<<grid, 256, 0, st>>>(a);
    }
#undef EMST_FAST
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
