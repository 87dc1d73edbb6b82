// Single-tree Boruvka EMST on one gfx950 GPU: kernels and the C ABI.
//
// Pipeline of emst_build (Section 3, Figure 3):
//   tree      bbox + validation -> Morton codes -> radix sort ->
//             gather into Morton order -> bottom-up hierarchy + boxes
//   round     label propagation -> component bounds -> traversal (+ stage-A
//             component minimum) -> stage-B resolve -> merge (successor,
//             roots + edge emission, pointer jumping, relabel)
//   finalize  canonical edge order by (D bits, u, v), weights = sqrtf(D)
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/emst.h"
#include "../../include/emst_test.h"
#include "emst_kernels.h"
#include "radix_sort.h"
#include "traverse.h"
#include "tune_table.h"

namespace emst {

// ===========================================================================
// tree construction

// Workgroups of 256 threads covering n items (at least one).
static inline unsigned grid_for(int64_t n, int threads = 256) {
    int64_t g = (n + threads - 1) / threads;
    return (unsigned)(g < 1 ? 1 : g);
}

// Device-scope atomics on one address from many workgroups serialise at the
// memory side (the XCDs' L2s are not coherent with each other), a few ns
// each; kernels that reduce to a single value therefore leave one partial
// per workgroup in `part` (at most kPartBlocks of them) and a small kernel
// or the next kernel folds them.
constexpr int kPartBlocks = 2048;

// Scene box and non-finite check: workgroup b leaves (ord_enc of min x,y,z,
// ord_enc of max x,y,z, non-finite flag) in part[8b .. 8b+6].
template <int DIM>
__global__ __launch_bounds__(256) void k_bbox(const float* __restrict__ pts, int64_t n, uint32_t* part) {
    __shared__ float s_lo[4][DIM], s_hi[4][DIM];
    __shared__ uint32_t s_bad[4];
    float lo[DIM], hi[DIM];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < DIM; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const float x = pts[i * DIM + k];
            bad |= !isfinite(x);
            lo[k] = fminf(lo[k], x);
            hi[k] = fmaxf(hi[k], x);
        }
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k)
        for (int off = 32; off > 0; off >>= 1) {
            lo[k] = fminf(lo[k], __shfl_xor(lo[k], off));
            hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off));
        }
    const bool any_bad = __ballot(bad) != 0ull;
    const int w = threadIdx.x / 64;
    if (lane_id() == 0) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) { s_lo[w][k] = lo[k]; s_hi[w][k] = hi[k]; }
        s_bad[w] = any_bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t b = 0;
        for (int v = 0; v < 4; ++v) {
            b |= s_bad[v];
#pragma unroll
            for (int k = 0; k < DIM; ++k) { lo[k] = fminf(lo[k], s_lo[v][k]); hi[k] = fmaxf(hi[k], s_hi[v][k]); }
        }
        uint32_t* o = part + 8 * (int64_t)blockIdx.x;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const bool some = k < DIM && lo[k % DIM] <= hi[k % DIM];
            o[k] = some ? ord_enc(lo[k % DIM]) : 0xFFFFFFFFu;
            o[3 + k] = some ? ord_enc(hi[k % DIM]) : 0u;
        }
        o[6] = b;
    }
}

// Folds the nb partials of k_bbox into the control block (one workgroup).
__global__ __launch_bounds__(256) void k_bbox_final(const uint32_t* __restrict__ part, int nb, Ctrl* ctrl) {
    __shared__ uint32_t s[4][7];
    uint32_t v[7] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u, 0u};
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            v[k] = min(v[k], part[8 * b + k]);
            v[3 + k] = max(v[3 + k], part[8 * b + 3 + k]);
        }
        v[6] |= part[8 * b + 6];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            v[k] = min(v[k], (uint32_t)__shfl_xor(v[k], off));
            v[3 + k] = max(v[3 + k], (uint32_t)__shfl_xor(v[3 + k], off));
        }
        v[6] |= (uint32_t)__shfl_xor(v[6], off);
    }
    const int w = threadIdx.x / 64;
    if (lane_id() == 0)
        for (int k = 0; k < 7; ++k) s[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int u = 1; u < (int)blockDim.x / 64; ++u) {
            for (int k = 0; k < 3; ++k) {
                v[k] = min(v[k], s[u][k]);
                v[3 + k] = max(v[3 + k], s[u][3 + k]);
            }
            v[6] |= s[u][6];
        }
        for (int k = 0; k < 3; ++k) {
            ctrl->bb_min[k] = v[k];
            ctrl->bb_max[k] = v[3 + k];
        }
        ctrl->nonfinite = v[6] ? 1u : 0u;
    }
}

template <int DIM>
hipError_t launch_bbox(const float* pts, int64_t n, uint32_t* part, Ctrl* ctrl, hipStream_t st) {
    const int nb = (int)std::min<unsigned>(grid_for(n), 1024);
    k_bbox<DIM><<<nb, 256, 0, st>>>(pts, n, part);
    k_bbox_final<<<1, 256, 0, st>>>(part, nb, ctrl);
    return hipGetLastError();
}

__global__ void k_init_ctrl(Ctrl* ctrl) {
    if (threadIdx.x == 0) {
        for (int k = 0; k < 3; ++k) { ctrl->bb_min[k] = 0xFFFFFFFFu; ctrl->bb_max[k] = 0u; }
        ctrl->nonfinite = 0; ctrl->root = kNone; ctrl->height = 0;
        ctrl->ncomp_next = 0; ctrl->edge_count = 0; ctrl->error = 0;
        ctrl->key_or = 0ull; ctrl->key_and = ~0ull;
        ctrl->internal_tests = 0; ctrl->leaf_tests = 0; ctrl->dist_evals = 0; ctrl->touched = 0;
        ctrl->long_ties = 0; ctrl->dup_codes = 0; ctrl->done = 0; ctrl->rounds_run = 0;
    }
}

__device__ __forceinline__ uint64_t spread3(uint64_t x) {
    x &= 0x1FFFFFull;
    x = (x | x << 32) & 0x1F00000000FFFFull;
    x = (x | x << 16) & 0x1F0000FF0000FFull;
    x = (x | x << 8) & 0x100F00F00F00F00Full;
    x = (x | x << 4) & 0x10C30C30C30C30C3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}
__device__ __forceinline__ uint64_t spread2(uint64_t x) {
    x &= 0xFFFFFFFFull;
    x = (x | x << 16) & 0x0000FFFF0000FFFFull;
    x = (x | x << 8) & 0x00FF00FF00FF00FFull;
    x = (x | x << 4) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | x << 2) & 0x3333333333333333ull;
    x = (x | x << 1) & 0x5555555555555555ull;
    return x;
}

struct MortonParams {
    double lo[3];
    double scale[3];
    double qmax;
};

// Quantisation of the scene box [lo, hi] to `bits` bits per axis.  Host and
// device evaluate the same IEEE double operations, so a kernel that derives
// the parameters from the control block gets the ones the host derives from
// its mirror.
__host__ __device__ inline MortonParams morton_params(const float* lo, const float* hi, int dim, int bits) {
    MortonParams mp;
    mp.qmax = (double)((1ull << bits) - 1ull);
    for (int k = 0; k < 3; ++k) {
        mp.lo[k] = k < dim ? (double)lo[k] : 0.0;
        const double ext = k < dim ? (double)hi[k] - (double)lo[k] : 0.0;
        mp.scale[k] = ext > 0.0 ? mp.qmax / ext : 0.0;
    }
    return mp;
}

__host__ __device__ inline MortonParams morton_params_of(const Ctrl& c, int dim) {
    float lo[3] = {0.f, 0.f, 0.f}, hi[3] = {0.f, 0.f, 0.f};
    for (int k = 0; k < dim; ++k) {
        lo[k] = ord_dec(c.bb_min[k]);
        hi[k] = ord_dec(c.bb_max[k]);
    }
    return morton_params(lo, hi, dim, dim == 3 ? 21 : 32);
}

// Z-curve code of every point: 21 bits per coordinate in 3D (63-bit code),
// 32 bits per coordinate in 2D (64-bit code).  The quantisation only shapes
// the tree; the EMST does not depend on it.  With `box` set, the parameters
// come from the scene box in that control block instead of `mp`, so the
// codes need no host read-back of the box.
template <int DIM>
__global__ __launch_bounds__(256) void k_morton(const float* __restrict__ pts, int64_t n, MortonParams mp,
                                                const Ctrl* __restrict__ box, uint64_t* __restrict__ keys,
                                                uint32_t* __restrict__ vals) {
    if (box) mp = morton_params_of(*box, DIM);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t q[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double t = ((double)pts[i * DIM + k] - mp.lo[k]) * mp.scale[k];
            t = fmin(fmax(t, 0.0), mp.qmax);
            q[k] = (uint64_t)t;
        }
        uint64_t code;
        if (DIM == 3) code = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2 % DIM]);
        else code = (spread2(q[0]) << 1) | spread2(q[1 % DIM]);
        keys[i] = code;
        vals[i] = (uint32_t)i;
    }
}

// ---------------------------------------------------------------------------
// Rank-space codes.  When many points share a Morton code (a density
// contrast beyond the code's resolution: the scene box is set by a few far
// points and the rest crowd into a handful of cells), equal codes are split
// by index and the tree loses its spatial order.  The codes are then built
// on per-axis ranks instead of coordinates: every axis is sorted once, and
// a point's quantised coordinate on that axis is its rank scaled to the
// code width.  Ranks are monotone in the coordinates, so the Z-curve of the
// ranks is still a spatial order, with resolution where the points are.

// Sorted positions whose code equals the previous one (one atomic per block).
__global__ __launch_bounds__(256) void k_count_dups(const uint64_t* __restrict__ codes, int64_t n, Ctrl* ctrl) {
    __shared__ uint32_t s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool dup = i > 0 && i < n && codes[i] == codes[i - 1];
    const uint64_t b = __ballot(dup);
    if (lane_id() == 0 && b) atomicAdd(&s_cnt, (uint32_t)__popcll(b));
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt) atomicAdd(&ctrl->dup_codes, s_cnt);
}

// keys = order-preserving bits of coordinate `axis`, values = point index
template <int DIM>
__global__ __launch_bounds__(256) void k_axis_keys(const float* __restrict__ pts, int64_t n, int axis,
                                                   uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = ord_enc(pts[i * DIM + axis]);
    vals[i] = (uint32_t)i;
}

// The point at rank r on `axis` gets the quantised coordinate r * 2^bits / n,
// spread into its Morton position; acc collects the axes.
template <int DIM>
__global__ __launch_bounds__(256) void k_axis_rank(const uint32_t* __restrict__ order, int64_t n, int axis, int bits,
                                                   uint64_t* __restrict__ acc) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint64_t q = ((uint64_t)r << bits) / (uint64_t)n;  // r < 2^31, bits <= 32
    const uint64_t part = (DIM == 3 ? spread3(q) : spread2(q)) << (DIM - 1 - axis);
    const uint32_t i = order[r];
    acc[i] = axis == 0 ? part : (acc[i] | part);
}

__global__ __launch_bounds__(256) void k_codes_from(const uint64_t* __restrict__ acc, int64_t n,
                                                    uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = acc[i];
    vals[i] = (uint32_t)i;
}

// Gather the coordinates into Morton order and initialise the per-point and
// per-component state: labels = own sorted position (Figure 3: every vertex
// starts as its own component), bounds = +inf, component keys = max.
template <int DIM>
// (The per-component arrays need no initial values: the first round writes
// every bound and key, and every component id writes its edge slot when it
// merges or resets it while it is a root.)
__global__ __launch_bounds__(256) void k_gather(const float* __restrict__ pts, const uint32_t* __restrict__ perm,
                                                int64_t n, float* __restrict__ spts, uint32_t* __restrict__ orig,
                                                uint32_t* __restrict__ labels, uint64_t* __restrict__ exch) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t o = perm[i];
#pragma unroll
    for (int k = 0; k < DIM; ++k) spts[i * DIM + k] = pts[(int64_t)o * DIM + k];
    orig[i] = o;
    labels[i] = (uint32_t)i;
    if (i + 1 < n) exch[i] = ~0ull;
}

// Highest differing bit between sorted augmented keys (code, index) k and
// k+1: codes that differ rank above any index difference.
__device__ __forceinline__ int split_bit(const uint64_t* __restrict__ codes, int64_t k) {
    const uint64_t x = codes[k] ^ codes[k + 1];
    if (x) return 32 + 63 - __clzll(x);
    return 31 - __clz((uint32_t)k ^ (uint32_t)(k + 1));
}

// Bottom-up construction of the binary radix tree over the sorted codes
// (the agglomerative scheme of Apetrei 2014, one of the two constructions
// the paper's BVH follows).  Internal node k is the node that splits
// between leaves k and k+1.  A node spanning leaves [l, r] becomes the left
// child of node r if its right neighbour pair (r, r+1) shares a longer
// prefix than its left neighbour pair (l-1, l), else the right child of
// node l-1.  The first of the two children to reach a parent parks its range
// end and its height there and stops; the second learns both from that
// exchange and continues upwards.  Only the 64-bit atomic exchange crosses
// between threads (agent-scope acquire/release would write back and
// invalidate the per-XCD L2 caches at every step); every other store is read
// by later kernels only.  The boxes are fitted afterwards (k_fit_tiles,
// k_fit_span).  A node's leaf range, height and parent link go out together
// in one 16-byte NodeInfo once its parent is known (the fit, or
// k_unpack_nodes, spreads them into their arrays): the stores of the climb
// land at scattered nodes, and four separate stores per node each cost a
// whole memory sector.  The child references are written with the boxes by
// the fit (REFS: here as well, for the test hook that reads the hierarchy
// without fitting it).
struct alignas(16) NodeInfo {
    uint32_t lo, hi, link, height;
};

template <int DIM, bool REFS>
__global__ __launch_bounds__(256) void k_build(const uint64_t* __restrict__ codes,
                                               const uint32_t* __restrict__ orig, int64_t n, Rec<DIM>* recs,
                                               uint32_t* __restrict__ leaf_parent, NodeInfo* __restrict__ info,
                                               uint64_t* exch, Ctrl* ctrl) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t l = i, r = i;
    uint32_t h = 0;
    uint32_t self = (uint32_t)i, self_ref = orig[i] | kLeafFlag;
    bool leaf = true;
    // every step climbs one level; a radix tree over 95-bit augmented keys
    // has height <= 96
    for (int step = 0;; ++step) {
        if (step > 128) {
            atomicOr(&ctrl->error, kErrStack);
            return;
        }
        bool left_child;
        if (l == 0) left_child = true;
        else if (r == n - 1) left_child = false;
        else left_child = split_bit(codes, r) < split_bit(codes, l - 1);
        const uint32_t parent = (uint32_t)(left_child ? r : l - 1);
        const int side = left_child ? 0 : 1;
        const uint32_t link = (parent << 1) | (uint32_t)side;
        if (REFS) set_child_ref<DIM>(&recs[parent], side, self_ref);
        if (leaf) leaf_parent[i] = link;
        else info[self] = NodeInfo{(uint32_t)l, (uint32_t)r, link, h};  // self's range and height
        // Two sibling leaves: node k holds leaves k and k+1 exactly when
        // leaf k is a left child and leaf k+1 a right child.  Both leaf
        // threads see this from the split bits of adjacent pairs (which
        // always differ), so the left one continues and the right one stops
        // with no exchange.
        bool pair = false;
        if (leaf) {
            if (left_child) pair = (i + 1 == n - 1) || split_bit(codes, i + 1) > split_bit(codes, i);
            else pair = (i - 1 == 0) || split_bit(codes, i - 1) < split_bit(codes, i - 2);
            if (pair && !left_child) return;
        }
        if (pair) {
            r = i + 1;
            h = 1u;
        } else {
            const uint64_t mine = ((uint64_t)(left_child ? l : r) << 32) | h;
            const uint64_t other = atomicExch((unsigned long long*)&exch[parent], (unsigned long long)mine);
            if (other == ~0ull) return;
            const int64_t oend = (int64_t)(other >> 32);
            if (left_child) r = oend;
            else l = oend;
            h = max(h, (uint32_t)(other & 0xFFFFFFFFu)) + 1u;
        }
        self = parent;
        self_ref = parent;
        leaf = false;
        if (l == 0 && r == n - 1) {
            ctrl->root = parent;
            ctrl->height = h;
            info[parent] = NodeInfo{(uint32_t)l, (uint32_t)r, kNone, h};
            return;
        }
    }
}

__global__ __launch_bounds__(256) void k_unpack_nodes(const NodeInfo* __restrict__ info, int64_t m,
                                                      uint32_t* __restrict__ rlo, uint32_t* __restrict__ rhi,
                                                      uint32_t* __restrict__ node_parent,
                                                      uint8_t* __restrict__ height) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const NodeInfo x = info[k];
    rlo[k] = x.lo;
    rhi[k] = x.hi;
    node_parent[k] = x.link;
    height[k] = (uint8_t)x.height;
}

// Boxes, bottom-up.  One workgroup per tile of kFitTile consecutive leaves
// fits every node whose leaf range lies inside its tile: each leaf's thread
// stores the leaf's box (its point) and reference into the parent's record
// and climbs while the parent lies inside the tile; at each such node the
// first child to arrive parks its box in LDS and stops, the second forms the
// union, stores it with the node's reference into the node's parent's record
// and climbs on.  Only LDS and one workgroup take part, so no thread waits
// on another and no cross-XCD ordering is needed.  The same pass spreads the
// tile's node records (range, parent link, height) into their arrays and
// lists the tile's nodes whose range crosses a tile border; those (a few per
// border and height) are fitted afterwards, one launch per height.
constexpr int kFitTile = 512;  // 256 and 1024 measured slower (LDS per workgroup vs nodes across borders)

template <int DIM>
__global__ __launch_bounds__(256) void k_fit_tiles(const float* __restrict__ spts, const uint32_t* __restrict__ orig,
                                                   const uint32_t* __restrict__ leaf_parent,
                                                   const NodeInfo* __restrict__ info, int64_t n, Rec<DIM>* recs,
                                                   uint32_t* __restrict__ rlo, uint32_t* __restrict__ rhi,
                                                   uint32_t* __restrict__ node_parent, uint8_t* __restrict__ height,
                                                   uint2* __restrict__ span, uint32_t* __restrict__ span_count,
                                                   Ctrl* ctrl) {
    if (ctrl->error) return;  // the build failed: its records are incomplete
    __shared__ uint32_t s_arrive[kFitTile];
    __shared__ float s_box[kFitTile][2][2 * DIM];  // per node of the tile and child side: lo, hi
    __shared__ uint32_t s_lo[kFitTile], s_hi[kFitTile], s_link[kFitTile];
    __shared__ uint2 s_span[kFitTile];
    __shared__ uint32_t s_nspan, s_base;
    const int t = threadIdx.x;
    const int64_t t0 = (int64_t)blockIdx.x * kFitTile;
    const int64_t m = n - 1;
    if (t == 0) s_nspan = 0;
    for (int x = t; x < kFitTile; x += 256) s_arrive[x] = 0;
    __syncthreads();
    for (int x = t; x < kFitTile; x += 256) {
        const int64_t k = t0 + x;
        if (k >= m) break;
        const NodeInfo v = info[k];
        rlo[k] = v.lo;
        rhi[k] = v.hi;
        node_parent[k] = v.link;
        height[k] = (uint8_t)v.height;
        s_lo[x] = v.lo;
        s_hi[x] = v.hi;
        s_link[x] = v.link;
        if (v.lo / kFitTile != v.hi / kFitTile) s_span[atomicAdd(&s_nspan, 1u)] = make_uint2((uint32_t)k, v.height);
    }
    __syncthreads();
    if (t == 0) s_base = s_nspan ? atomicAdd(span_count, s_nspan) : 0u;
    __syncthreads();
    // (the list has room for n - 1 entries, at most 129 per tile border of a
    // valid tree)
    for (uint32_t x = t; x < s_nspan; x += 256) {
        if ((int64_t)s_base + x < m) span[s_base + x] = s_span[x];
        else atomicOr(&ctrl->error, kErrStack);
    }
    const uint32_t lo_in = (uint32_t)t0, hi_in = (uint32_t)min<int64_t>(t0 + kFitTile - 1, n - 1);
    for (int x = t; x < kFitTile; x += 256) {
        const int64_t i = t0 + x;
        if (i >= n) break;
        float lo[DIM], hi[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) lo[k] = hi[k] = spts[i * DIM + k];
        uint32_t link = leaf_parent[i];
        uint32_t ref = orig[i] | kLeafFlag;
        for (int step = 0; step < 160; ++step) {  // a climb passes at most height + 1 <= 129 nodes
            const uint32_t P = link >> 1;
            const int side = (int)(link & 1u);
            if ((int64_t)P >= m) {  // (not from a valid tree)
                atomicOr(&ctrl->error, kErrStack);
                break;
            }
            set_child<DIM>(&recs[P], side, lo, hi, ref);
            const int64_t ps = (int64_t)P - t0;
            if (ps < 0 || ps >= kFitTile) break;                    // P spans the tile's border
            if (s_lo[ps] < lo_in || s_hi[ps] > hi_in) break;         // likewise
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                s_box[ps][side][k] = lo[k];
                s_box[ps][side][DIM + k] = hi[k];
            }
            __threadfence_block();
            if (atomicAdd(&s_arrive[ps], 1u) == 0u) break;  // the sibling completes P
            __threadfence_block();
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                lo[k] = fminf(lo[k], s_box[ps][1 - side][k]);
                hi[k] = fmaxf(hi[k], s_box[ps][1 - side][DIM + k]);
            }
            ref = P;
            link = s_link[ps];
            if (link == kNone) break;  // the root
        }
    }
}

// The listed nodes of height h (ranges across a tile border): box = union
// of the two child boxes in the own record, stored with the node's
// reference in the parent's record.  Their children are leaves and nodes
// fitted by k_fit_tiles, or listed nodes of smaller height.
template <int DIM>
__global__ __launch_bounds__(256) void k_fit_span(const uint2* __restrict__ span,
                                                  const uint32_t* __restrict__ span_count, int64_t cap, uint32_t h,
                                                  const uint32_t* __restrict__ node_parent, Rec<DIM>* recs) {
    const uint32_t cnt = (uint32_t)min<int64_t>(*span_count, cap);
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < cnt; j += gridDim.x * blockDim.x) {
        const uint2 e = span[j];
        if (e.y != h) continue;
        const uint32_t k = e.x;
        const uint32_t link = node_parent[k];
        if (link == kNone) continue;
        Child<DIM> c0, c1;
        unpack<DIM>(recs[k], c0, c1);
        float lo[DIM], hi[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            lo[d] = fminf(c0.lo[d], c1.lo[d]);
            hi[d] = fmaxf(c0.hi[d], c1.hi[d]);
        }
        set_child<DIM>(&recs[link >> 1], (int)(link & 1u), lo, hi, k);
    }
}

__device__ __forceinline__ uint32_t compact3(uint64_t x) {
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10C30C30C30C30C3ull;
    x = (x ^ (x >> 4)) & 0x100F00F00F00F00Full;
    x = (x ^ (x >> 8)) & 0x1F0000FF0000FFull;
    x = (x ^ (x >> 16)) & 0x1F00000000FFFFull;
    x = (x ^ (x >> 32)) & 0x1FFFFFull;
    return (uint32_t)x;
}
__device__ __forceinline__ uint32_t compact2(uint64_t x) {
    x &= 0x5555555555555555ull;
    x = (x ^ (x >> 1)) & 0x3333333333333333ull;
    x = (x ^ (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x ^ (x >> 4)) & 0x00FF00FF00FF00FFull;
    x = (x ^ (x >> 8)) & 0x0000FFFF0000FFFFull;
    x = (x ^ (x >> 16)) & 0x00000000FFFFFFFFull;
    return (uint32_t)x;
}

// Morton cell of every internal node.  A node that splits on a code bit t
// holds exactly the points whose codes agree with its leaves above bit t, so
// its cell is the box of quantised coordinates with those bits fixed.  In
// real coordinates the cell is [lo + Q/scale, lo + (Q + 2^m)/scale) per
// axis (m = free low bits of that axis); the stored box is shrunk by a
// margin far above every rounding in the quantisation, so any point inside
// the stored box has codes with the node's prefix.  Axes at the scene edge
// stay open, nodes that split equal codes get an empty cell.
// With rank-space codes (`ranks`) a cell is not a box of coordinates: every
// cell is left empty, so the climbs run to the top.
template <int DIM>
__global__ __launch_bounds__(256) void k_cells(const uint64_t* __restrict__ codes,
                                               const uint32_t* __restrict__ node_parent, int64_t m,
                                               MortonParams mp, bool ranks, Up* __restrict__ up) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const uint64_t x = codes[k] ^ codes[k + 1];
    if (x && !ranks) {
        const int t = 63 - __clzll(x);  // highest differing code bit = the node's split bit
        const uint64_t code = codes[k];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const int off = DIM - 1 - d;   // bit offset of axis d inside a Morton digit
            const uint32_t q = (DIM == 3) ? compact3(code >> off) : compact2(code >> off);
            const int free_bits = (t >= off) ? (t - off) / DIM + 1 : 0;
            if (mp.scale[d] <= 0.0) {
                clo[d] = -INFINITY;
                chi[d] = INFINITY;
                continue;
            }
            const double Q = (double)(free_bits >= 32 ? 0u : (q >> free_bits) << free_bits);
            const double W = (double)(1ull << free_bits);
            const double ext = mp.qmax / mp.scale[d];
            const double margin = 1e-6 * (fabs(mp.lo[d]) + ext);
            clo[d] = (Q <= 0.0) ? -INFINITY : (float)(mp.lo[d] + Q / mp.scale[d] + margin);
            chi[d] = (Q + W > mp.qmax) ? INFINITY : (float)(mp.lo[d] + (Q + W) / mp.scale[d] - margin);
        }
    }
    Up u;
    u.a = make_float4(clo[0], clo[1], clo[2], __uint_as_float(node_parent[k]));
    u.b = make_float4(chi[0], chi[1], chi[2], 0.f);
    up[k] = u;
}

// For every wave of 64 Morton-consecutive queries [64w, 64w + 63]: the
// lowest node whose leaf range covers them, found by climbing from the first
// leaf.  Written over the exchange words of the build, which are dead once
// the hierarchy exists.
__global__ __launch_bounds__(256) void k_wave_lca(const uint32_t* __restrict__ rlo, const uint32_t* __restrict__ rhi,
                                                  const uint32_t* __restrict__ leaf_parent,
                                                  const uint32_t* __restrict__ node_parent, int64_t n,
                                                  uint32_t* __restrict__ wave_lca) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i0 = 64 * w;
    if (i0 >= n) return;
    const uint32_t i1 = (uint32_t)min<int64_t>(i0 + 63, n - 1);
    uint32_t s = leaf_parent[i0] >> 1;
    for (int h = 0; h < 160; ++h) {
        if (rlo[s] <= (uint32_t)i0 && rhi[s] >= i1) break;
        const uint32_t link = node_parent[s];
        if (link == kNone) break;
        s = link >> 1;
    }
    wave_lca[w] = s;
}

// ===========================================================================
// one Boruvka round

// Optimization 1 (Section 3): every internal node gets its leaves' common
// component label, or kInvalid.  The paper propagates labels bottom-up with
// first/second-arrival threads; here the same labels come from the leaf
// ranges instead.  In Morton order record k holds the leaf ranges [lo, k]
// and [k+1, hi]; the first shares one label exactly when the run of equal
// labels containing k starts at or before lo, the second when the run
// containing k+1 ends at or after hi.  Both tests are local to k once every
// tile of kRunTile positions knows where the run crossing its left edge
// starts and where the run crossing its right edge ends:
//   - per tile, the last position where a run starts and the first where
//     one ends (left by the previous round's relabel kernel, or by
//     k_run_partials for arbitrary labels);
//   - k_tile_carries: an exclusive max-scan and an exclusive suffix
//     min-scan of those over the tiles;
//   - k_round_prep: per tile, the run starts and ends of every position by
//     scans in LDS, then the record labels and, in the same pass, the
//     Morton-neighbour bounds of Optimization 2.
// No thread ever waits on another.

constexpr int kRunPer = 8;                        // positions per thread
constexpr int kRunTile = 256 * kRunPer;           // positions per tile (one workgroup)
constexpr int kRunLds = kRunTile + kRunTile / 16 + 8;

static inline int run_tiles(int64_t n) { return (int)((n + kRunTile - 1) / kRunTile); }

// LDS hash table of the bound pass (k_round_prep), in the run arrays
constexpr int kBoundHashBits = 11;
constexpr int kBoundHash = 1 << kBoundHashBits;
static_assert(kBoundHash <= kRunLds, "the bound hash fits in the run arrays");

// LDS slot of tile-local index x: one pad word per 16 keeps the
// consecutive positions of one thread in distinct banks.
__device__ __forceinline__ int run_lds(int x) { return x + (x >> 4); }

// Reduce (max, min) over the 256 threads of the workgroup; s_w holds 8 words.
__device__ __forceinline__ void block_max_min256(uint32_t& mx, uint32_t& mn, uint32_t* s_w) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        mx = max(mx, (uint32_t)__shfl_xor(mx, off));
        mn = min(mn, (uint32_t)__shfl_xor(mn, off));
    }
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        s_w[w] = mx;
        s_w[4 + w] = mn;
    }
    __syncthreads();
    mx = max(max(s_w[0], s_w[1]), max(s_w[2], s_w[3]));
    mn = min(min(s_w[4], s_w[5]), min(s_w[6], s_w[7]));
}

// Sum of (a, b) over the 256 threads of the workgroup; s_w holds 8 words.
__device__ __forceinline__ void block_sum2_256(uint32_t& a, uint32_t& b, uint32_t* s_w) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += (uint32_t)__shfl_xor(a, off);
        b += (uint32_t)__shfl_xor(b, off);
    }
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        s_w[w] = a;
        s_w[4 + w] = b;
    }
    __syncthreads();
    a = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    b = s_w[4] + s_w[5] + s_w[6] + s_w[7];
}

// Up to this many tiles, a kernel that needs a scan over the per-tile
// partials of the kernel before computes its own entry from all of them
// (at most 2 x 1024 words from L2 per workgroup) instead of waiting for a
// one-workgroup scan kernel, which saves that launch.
constexpr int kFoldTiles = 1024;

// Exclusive max-scan in thread order over the 256 threads (0 for thread 0).
__device__ __forceinline__ uint32_t block_excl_max256(uint32_t x, uint32_t* s_w4) {
    const int lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off);
        if (lane >= off) inc = max(inc, y);
    }
    if (lane == 63) s_w4[w] = inc;
    __syncthreads();
    uint32_t ex = __shfl_up(inc, 1);
    if (lane == 0) ex = 0u;
    for (int k = 0; k < w; ++k) ex = max(ex, s_w4[k]);
    return ex;
}

// Exclusive min-scan in reverse thread order (kNone for thread 255).
__device__ __forceinline__ uint32_t block_excl_min256_rev(uint32_t x, uint32_t* s_w4) {
    const int lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_down(inc, off);
        if (lane + off < 64) inc = min(inc, y);
    }
    if (lane == 0) s_w4[w] = inc;
    __syncthreads();
    uint32_t ex = __shfl_down(inc, 1);
    if (lane == 63) ex = kNone;
    for (int k = w + 1; k < 4; ++k) ex = min(ex, s_w4[k]);
    return ex;
}

// Inclusive max-scan over the block (blockDim.x a multiple of 64, at most
// 1024); s_w holds one slot per wave.
__device__ __forceinline__ uint32_t block_max_scan_incl(uint32_t x, uint32_t* s_w) {
    const int lane = lane_id(), w = threadIdx.x / 64;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x = max(x, y);
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < w; ++k) before = max(before, s_w[k]);
    __syncthreads();
    return max(x, before);
}

// Tile partials of arbitrary labels: part[2t] = the last position p of tile
// t where a run starts (p = 0 or labels[p-1] != labels[p]), 0 if none;
// part[2t+1] = the first position where a run ends (p = n-1 or
// labels[p] != labels[p+1]), kNone if none.
__global__ __launch_bounds__(256) void k_run_partials(const uint32_t* __restrict__ labels, int64_t n,
                                                      uint32_t* __restrict__ part) {
    __shared__ uint32_t s_w[8];
    const int64_t base = (int64_t)blockIdx.x * kRunTile;
    uint32_t hmax = 0u, tmin = kNone;
    for (int q = 0; q < kRunPer; ++q) {
        const int64_t p = base + (int64_t)q * 256 + threadIdx.x;
        if (p >= n) break;
        const uint32_t l = labels[p];
        if (p == 0 || labels[p - 1] != l) hmax = max(hmax, (uint32_t)p);
        if (p == n - 1 || labels[p + 1] != l) tmin = min(tmin, (uint32_t)p);
    }
    block_max_min256(hmax, tmin, s_w);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = hmax;
        part[2 * blockIdx.x + 1] = tmin;
    }
}

// Exclusive scan over the nb tile partials in scan order j (tile j, or tile
// nb-1-j when REV): carry[2t] = max(part[2u], u < t) (0 for the first tile);
// REV: carry[2t+1] = min(part[2u+1], u > t) (kNone for the last tile), as a
// max-scan of complements.
template <bool REV>
__device__ __forceinline__ void tiles_excl_scan(const uint32_t* __restrict__ part, uint32_t* __restrict__ carry,
                                                int nb, uint32_t* s_w, uint32_t* s_incl) {
    uint32_t run = 0u;
    for (int c0 = 0; c0 < nb; c0 += 1024) {
        const int j = c0 + (int)threadIdx.x;
        const int t = REV ? nb - 1 - j : j;
        uint32_t x = 0u;
        if (j < nb) x = REV ? ~part[2 * t + 1] : part[2 * t];
        const uint32_t incl = block_max_scan_incl(x, s_w);
        s_incl[threadIdx.x] = incl;
        __syncthreads();
        const uint32_t ex = max(run, threadIdx.x > 0 ? s_incl[threadIdx.x - 1] : 0u);
        if (j < nb) carry[2 * t + (REV ? 1 : 0)] = REV ? ~ex : ex;
        run = max(run, s_incl[1023]);
        __syncthreads();
    }
}

// One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_tile_carries(const uint32_t* __restrict__ part, int nb,
                                                       uint32_t* __restrict__ carry, const Ctrl* ctrl) {
    if (ctrl->done) return;
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_incl[1024];
    tiles_excl_scan<false>(part, carry, nb, s_w, s_incl);
    tiles_excl_scan<true>(part, carry, nb, s_w, s_incl);
}

// Per tile: the record labels lab2[k] of every record k in the tile and,
// with BOUNDS, the Morton-neighbour bound of every component (Optimization
// 2): a Morton-adjacent pair with different labels bounds the shortest
// outgoing edge of both components by its D.  Every position takes the
// smaller D to its neighbours outside its component (its M under mutual
// reachability, core_s set; pairs in different clouds of a batch bound
// nothing).  FIRST: the first round, where every position is its own
// component: the tests reduce to lo == k and hi == k + 1, and every
// position writes its own bound.  Later the positions of a run of equal
// labels within a wave combine first and one lane per run lowers the
// component's bound.
// Kept candidates (traversal variant 13, from the third round on): a point
// whose last candidate still lies outside its component keeps it (see
// k_traverse_fast, REUSE).  k_round_prep flags such points in `kept` and
// offers their candidates to stage A of their component, so that the
// component key holds a real outgoing edge of the component, hence a bound
// on its shortest one, before the query list is made and the traversal
// runs.  kept = null: no offers.
struct KeepArgs {
    const uint32_t* cand_d;
    const uint32_t* cand_j;
    const uint32_t* cand_p;
    const uint32_t* orig;
    uint64_t* compkey;
    uint8_t* kept;
};

template <int DIM, bool FIRST, bool BOUNDS>
__global__ __launch_bounds__(256) void k_round_prep(const uint32_t* __restrict__ labels,
                                                    const uint32_t* __restrict__ carry,
                                                    const uint32_t* __restrict__ rlo,
                                                    const uint32_t* __restrict__ rhi, uint2* __restrict__ lab2,
                                                    const float* __restrict__ spts,
                                                    const uint32_t* __restrict__ cloud_of,
                                                    const float* __restrict__ core_s, int64_t n, uint32_t* ub,
                                                    Ctrl* ctrl, const uint32_t* __restrict__ fold_part, int nt,
                                                    KeepArgs keep, uint32_t* __restrict__ succ) {
    if (ctrl->done) return;
    __shared__ uint32_t s_lab[kRunLds];               // labels of positions base-1 .. base+kRunTile
    __shared__ uint32_t s_rs[FIRST ? 1 : kRunLds];    // start of the run containing each position
    __shared__ uint32_t s_re[FIRST ? 1 : kRunLds];    // end of the run containing each position
    __shared__ uint32_t s_w[8];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kRunTile;
    // the leaf ranges of the tile's records, loaded before the label scans
    // so that their latency overlaps the scans
    uint32_t rl[kRunPer], rh[kRunPer];
#pragma unroll
    for (int q = 0; q < kRunPer; ++q) {
        const int64_t k = base + q * 256 + tid;
        rl[q] = k < n - 1 ? rlo[k] : 0u;
        rh[q] = k < n - 1 ? rhi[k] : 0u;
    }
    for (int x = tid; x < kRunTile + 2; x += 256) {
        int64_t p = base + x - 1;
        p = p < 0 ? 0 : (p >= n ? n - 1 : p);
        s_lab[run_lds(x)] = FIRST ? (uint32_t)p : labels[p];  // first round: a point's label is its position
    }
    // the tile carries: last run start before the tile, first run end after
    // it (from k_tile_carries, or with fold_part from the tile partials)
    uint32_t carry_l = 0u, carry_r = kNone;
    if (!FIRST) {
        if (fold_part) {
            for (int t = tid; t < nt; t += 256) {
                if (t < (int)blockIdx.x) carry_l = max(carry_l, fold_part[2 * t]);
                if (t > (int)blockIdx.x) carry_r = min(carry_r, fold_part[2 * t + 1]);
            }
            block_max_min256(carry_l, carry_r, s_w);  // (its barrier also covers s_lab)
        } else {
            carry_l = carry[2 * blockIdx.x];
            carry_r = carry[2 * blockIdx.x + 1];
        }
    }
    __syncthreads();
    if (!FIRST) {
        // thread tid owns the local positions [kRunPer tid, kRunPer (tid + 1))
        const int x0 = tid * kRunPer;
        uint32_t agg_h = 0u, agg_t = kNone;
#pragma unroll
        for (int j = 0; j < kRunPer; ++j) {
            const int x = x0 + j;
            const int64_t p = base + x;
            if (p < n) {
                const uint32_t l = s_lab[run_lds(x + 1)];
                if (p == 0 || s_lab[run_lds(x)] != l) agg_h = max(agg_h, (uint32_t)p);
                if (p == n - 1 || s_lab[run_lds(x + 2)] != l) agg_t = min(agg_t, (uint32_t)p);
            }
        }
        uint32_t cur = max(block_excl_max256(agg_h, s_w), carry_l);
        const uint32_t cr = min(block_excl_min256_rev(agg_t, s_w + 4), carry_r);
#pragma unroll
        for (int j = 0; j < kRunPer; ++j) {
            const int x = x0 + j;
            const int64_t p = base + x;
            if (p < n && (p == 0 || s_lab[run_lds(x)] != s_lab[run_lds(x + 1)])) cur = (uint32_t)p;
            s_rs[run_lds(x)] = cur;
        }
        cur = cr;
#pragma unroll
        for (int j = kRunPer - 1; j >= 0; --j) {
            const int x = x0 + j;
            const int64_t p = base + x;
            if (p < n && (p == n - 1 || s_lab[run_lds(x + 2)] != s_lab[run_lds(x + 1)])) cur = (uint32_t)p;
            s_re[run_lds(x)] = cur;
        }
        __syncthreads();
    }
    // record labels; record k has the children [rlo[k], k] and [k+1, rhi[k]]
#pragma unroll
    for (int q = 0; q < kRunPer; ++q) {
        const int x = q * 256 + tid;
        const int64_t k = base + x;
        if (k < n - 1) {
            const uint32_t lo = rl[q], hi = rh[q];
            bool left, right;
            if (FIRST) {
                left = lo == (uint32_t)k;
                right = hi == (uint32_t)(k + 1);
            } else {
                left = s_rs[run_lds(x)] <= lo;
                right = (x + 1 < kRunTile ? s_re[run_lds(x + 1)] : carry_r) >= hi;
            }
            lab2[k] = make_uint2(left ? s_lab[run_lds(x + 1)] : kInvalid,
                                 right ? s_lab[run_lds(x + 2)] : kInvalid);
        }
        // a component's successor is itself until stage B finds its edge
        // (the first round's traversal writes every successor itself)
        if (!FIRST && succ && k < n && s_lab[run_lds(x + 1)] == (uint32_t)k) succ[k] = (uint32_t)k;
    }
    if (!FIRST && keep.kept) {
        uint32_t pj[kRunPer], other[kRunPer];
#pragma unroll
        for (int q = 0; q < kRunPer; ++q) {
            const int64_t k = base + q * 256 + tid;
            pj[q] = k < n ? keep.cand_j[k] : kNone;
        }
#pragma unroll
        for (int q = 0; q < kRunPer; ++q) {
            const int64_t k = base + q * 256 + tid;
            other[q] = pj[q] != kNone ? keep.cand_p[k] : 0u;
        }
#pragma unroll
        for (int q = 0; q < kRunPer; ++q) other[q] = pj[q] != kNone ? labels[other[q]] : kNone;
#pragma unroll
        for (int q = 0; q < kRunPer; ++q) {
            const int x = q * 256 + tid;
            const int64_t k = base + x;
            const bool valid = k < n;
            const uint32_t lab = valid ? s_lab[run_lds(x + 1)] : kNone;
            const bool kp = valid && pj[q] != kNone && other[q] != lab;
            uint64_t key = kKeyMax;
            if (kp) key = ((uint64_t)keep.cand_d[k] << 32) | (uint64_t)min(keep.orig[k], pj[q]);
            if (valid) keep.kept[k] = kp ? 1u : 0u;
            if (base + q * 256 < n) {  // uniform over the workgroup
                bool run_end;
                key = wave_seg_min<uint64_t>(lab, key, &run_end);
                if (valid && run_end && key != kKeyMax && key < load_relaxed64(&keep.compkey[lab]))
                    atomicMin((unsigned long long*)&keep.compkey[lab], (unsigned long long)key);
            }
        }
    }
    if (!BOUNDS) return;
    uint32_t v[kRunPer];
#pragma unroll
    for (int q = 0; q < kRunPer; ++q) {
        const int x = q * 256 + tid;
        const int64_t k = base + x;
        v[q] = kInfBits;
        const uint32_t lab = s_lab[run_lds(x + 1)];
        const uint32_t llab = s_lab[run_lds(x)], rlab = s_lab[run_lds(x + 2)];
        // only a position next to another component reads coordinates
        if (k < n && (llab != lab || rlab != lab)) {
            const int64_t kl = k > 0 ? k - 1 : k, kr = k + 1 < n ? k + 1 : k;
            uint32_t cl = 0u, lcl = 0u, rcl = 0u;
            if (cloud_of) {
                cl = cloud_of[k];
                lcl = cloud_of[kl];
                rcl = cloud_of[kr];
            }
            float pp[DIM], o[DIM], r[DIM];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                pp[c] = spts[k * DIM + c];
                o[c] = spts[kl * DIM + c];
                r[c] = spts[kr * DIM + c];
            }
            // D(k-1, k) is evaluated as position k-1 evaluates D(k-1, k)
            const float ck = core_s ? core_s[k] : 0.f;
            const float cll = core_s ? core_s[kl] : 0.f, crr = core_s ? core_s[kr] : 0.f;
            if (kl != k && llab != lab && lcl == cl)
                v[q] = min(v[q], fbits(fmaxf(fmaxf(cll, ck), sqdist<DIM>(o, pp))));
            if (kr != k && rlab != lab && rcl == cl)
                v[q] = min(v[q], fbits(fmaxf(fmaxf(ck, crr), sqdist<DIM>(pp, r))));
        }
    }
    if constexpr (FIRST) {
#pragma unroll
        for (int q = 0; q < kRunPer; ++q) {
            const int64_t k = base + q * 256 + tid;
            if (k < n) ub[k] = v[q];
        }
    } else {
        // Later rounds: the runs of a wave combine first (segmented min over the
        // lanes), then the tile's components combine in an LDS hash table (the
        // run-start and run-end arrays are free by now), so a component gets
        // one global atomic per tile instead of one per run.  A full probe
        // sequence falls back to the global atomic.
        uint32_t* h_lab = s_rs;
        uint32_t* h_val = s_re;
        bool some = false;
#pragma unroll
        for (int q = 0; q < kRunPer; ++q) some |= v[q] != kInfBits;
        // a tile without a component boundary (most tiles of late rounds)
        // has no bound to give
        if (!__syncthreads_or(some)) return;
        for (int e = tid; e < kBoundHash; e += 256) {
            h_lab[e] = kNone;
            h_val[e] = kInfBits;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kRunPer; ++q) {
            const int x = q * 256 + tid;
            const int64_t k = base + x;
            // uniform over the workgroup; a wave without a bound skips its scan
            if (base + q * 256 < n && __ballot(v[q] != kInfBits) != 0ull) {
                const uint32_t lab = k < n ? s_lab[run_lds(x + 1)] : kNone;
                bool run_end;
                const uint32_t m = wave_seg_min<uint32_t>(lab, v[q], &run_end);
                if (k < n && run_end && m != kInfBits) {
                    uint32_t h = (lab * 2654435761u) >> (32 - kBoundHashBits);
                    bool placed = false;
                    for (int probe = 0; probe < 8; ++probe) {
                        const uint32_t old = atomicCAS(&h_lab[h], kNone, lab);
                        if (old == kNone || old == lab) {
                            atomicMin(&h_val[h], m);
                            placed = true;
                            break;
                        }
                        h = (h + 1) & (kBoundHash - 1);
                    }
                    if (!placed && m < load_relaxed(&ub[lab])) atomicMin(&ub[lab], m);
                }
            }
        }
        __syncthreads();
        for (int e = tid; e < kBoundHash; e += 256) {
            const uint32_t lab = h_lab[e];
            if (lab == kNone) continue;
            const uint32_t m = h_val[e];
            if (m < load_relaxed(&ub[lab])) atomicMin(&ub[lab], m);
        }
    }
}

// ---------------------------------------------------------------------------
// Query lists (traversal variant 13 from the third round on): the points
// that still have to search, in Morton order, so that the traversal's waves
// run full.  A point whose last result still holds (see k_traverse_fast,
// REUSE) offers its kept candidate to its component here instead.

// Per tile of kRunTile positions: qflag[i] = 1 for a point that must
// search, qcnt[t] = their number.  On entry qflag holds the kept flags of
// k_round_prep, whose offers are complete by now, so the radius of every
// component is known: its bound, lowered to the shortest kept candidate
// while components are small (tight_radius).  A
// point searches unless it keeps its candidate, or its last result shows
// that nothing outside its component lies within that radius: an absorbed
// candidate at D = pd (every point now outside was outside then, so none
// is nearer), or a search that found nothing within R.
__global__ __launch_bounds__(256) void k_reuse_mark(const uint32_t* __restrict__ labels,
                                                    const uint32_t* __restrict__ ub,
                                                    const uint64_t* __restrict__ compkey,
                                                    uint32_t* __restrict__ cand_d, uint32_t* __restrict__ cand_j,
                                                    uint8_t* __restrict__ qflag, uint32_t* __restrict__ qcnt,
                                                    int64_t n, const Ctrl* ctrl) {
    if (ctrl->done) return;
    __shared__ uint32_t s_w[4];
    const int64_t base = (int64_t)blockIdx.x * kRunTile;
    uint32_t c[kRunPer], pj[kRunPer], pd[kRunPer], kp[kRunPer], radius[kRunPer];
#pragma unroll
    for (int q = 0; q < kRunPer; ++q) {
        const int64_t i = base + q * 256 + threadIdx.x;
        const bool valid = i < n;
        c[q] = valid ? labels[i] : kNone;
        kp[q] = valid ? qflag[i] : 1u;
        pj[q] = valid ? cand_j[i] : kNone;
        pd[q] = valid ? cand_d[i] : 0u;
    }
    const bool tight = tight_radius(ctrl, n);
#pragma unroll
    for (int q = 0; q < kRunPer; ++q) {
        radius[q] = 0u;
        if (c[q] != kNone && !kp[q]) {
            const uint64_t ck = tight ? compkey[c[q]] : kKeyMax;
            radius[q] = min(ub[c[q]], ck != kKeyMax ? (uint32_t)(ck >> 32) : kInfBits);
        }
    }
    uint32_t cnt = 0;
#pragma unroll
    for (int q = 0; q < kRunPer; ++q) {
        const int64_t i = base + q * 256 + threadIdx.x;
        if (i >= n) continue;
        bool need = false;
        if (!kp[q]) {
            if (pj[q] != kNone) {
                need = pd[q] <= radius[q];
                if (!need) {  // absorbed beyond the radius
                    cand_j[i] = kNone;
                    cand_d[i] = pd[q] - 1u;  // every outside point has D > this
                }
            } else {
                need = radius[q] > pd[q];
            }
        }
        qflag[i] = need ? 1u : 0u;
        cnt += need;
    }
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) qcnt[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// qoff[t] = sum(qcnt[u], u < t); ctrl->qcount = the total.  One workgroup
// of 1024 threads.
__global__ __launch_bounds__(1024) void k_qlist_scan(const uint32_t* __restrict__ qcnt, int nt,
                                                     uint32_t* __restrict__ qoff, Ctrl* ctrl) {
    if (ctrl->done) return;
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_incl[1024];
    uint32_t run = 0;
    for (int c0 = 0; c0 < nt; c0 += 1024) {
        const int t = c0 + (int)threadIdx.x;
        uint32_t x = t < nt ? qcnt[t] : 0u;
        const int lane = lane_id(), w = threadIdx.x / 64;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) s_w[w] = x;
        __syncthreads();
        uint32_t before = 0;
        for (int k = 0; k < w; ++k) before += s_w[k];
        s_incl[threadIdx.x] = x + before;
        __syncthreads();
        const uint32_t ex = run + (threadIdx.x > 0 ? s_incl[threadIdx.x - 1] : 0u);
        if (t < nt) qoff[t] = ex;
        run += s_incl[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) ctrl->qcount = run;
}

// qlist[qoff[t] + k] = the k-th flagged position of tile t, in order.  With
// fold_cnt, a workgroup sums the tile counts before its own tile itself
// (qoff unused), and workgroup 0 stores the total in ctrl->qcount.
__global__ __launch_bounds__(256) void k_qlist_write(const uint8_t* __restrict__ qflag,
                                                     const uint32_t* __restrict__ qoff, int64_t n,
                                                     uint32_t* __restrict__ qlist, Ctrl* ctrl,
                                                     const uint32_t* __restrict__ fold_cnt, int nt) {
    if (ctrl->done) return;
    __shared__ uint32_t s_w[8];
    uint32_t off;
    if (fold_cnt) {
        uint32_t before = 0u, total = 0u;
        for (int t = threadIdx.x; t < nt; t += 256) {
            const uint32_t c = fold_cnt[t];
            total += c;
            if (t < (int)blockIdx.x) before += c;
        }
        block_sum2_256(before, total, s_w);
        if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->qcount = total;
        off = before;
        __syncthreads();  // s_w is reused below
    } else {
        off = qoff[blockIdx.x];
    }
    const int64_t base = (int64_t)blockIdx.x * kRunTile;
    const int64_t x0 = base + (int64_t)threadIdx.x * kRunPer;  // this thread's kRunPer consecutive positions
    uint32_t f[kRunPer];
    uint32_t cnt = 0;
#pragma unroll
    for (int j = 0; j < kRunPer; ++j) {
        f[j] = x0 + j < n ? qflag[x0 + j] : 0u;
        cnt += f[j];
    }
    // exclusive sum over the threads of the workgroup
    const int lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t inc = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off);
        if (lane >= off) inc += y;
    }
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t at = off + inc - cnt;
    for (int k = 0; k < w; ++k) at += s_w[k];
#pragma unroll
    for (int j = 0; j < kRunPer; ++j)
        if (f[j]) qlist[at++] = (uint32_t)(x0 + j);
}

// Stage B of the component minimum: among the points whose candidate matches
// the component's (D bits, min index) key, the smallest max index wins, so
// the component edge is the minimum under (D, min, max).  Every matching
// point also names the component at the other end of that edge, the
// successor of the merge (Section 3, "Merging components together"): if
// two points of a component match, their common min index cannot be one
// of them (the other's candidate lies outside), so it is their common
// candidate; hence all matching points have the same candidate, and write
// the same successor, the label at its sorted position.  PER consecutive
// points per thread: 4 (16-byte loads; the arrays are 256-byte aligned)
// once components span many points, 1 in the round after the first, where
// they are small and a thread's component-key loads mostly miss.
template <int PER>
__global__ __launch_bounds__(256) void k_resolve(const uint32_t* __restrict__ cand_d,
                                                 const uint32_t* __restrict__ cand_j,
                                                 const uint32_t* __restrict__ cand_p,
                                                 const uint32_t* __restrict__ labels,
                                                 const uint32_t* __restrict__ orig,
                                                 const uint64_t* __restrict__ compkey, uint32_t* compmax,
                                                 uint32_t* __restrict__ succ, int64_t n, const Ctrl* ctrl) {
    const int64_t i0 = PER * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (i0 >= n || ctrl->done) return;
    uint32_t j[PER], cd[PER], oi[PER], c[PER];
    if (PER == 4 && i0 + 3 < n) {
        const uint4 J = *reinterpret_cast<const uint4*>(cand_j + i0);
        if ((J.x & J.y & J.z & J.w) == kNone) return;  // none has a candidate
        const uint4 D = *reinterpret_cast<const uint4*>(cand_d + i0);
        const uint4 O = *reinterpret_cast<const uint4*>(orig + i0);
        const uint4 L = *reinterpret_cast<const uint4*>(labels + i0);
        const uint32_t jv[4] = {J.x, J.y, J.z, J.w}, dv[4] = {D.x, D.y, D.z, D.w};
        const uint32_t ov[4] = {O.x, O.y, O.z, O.w}, lv[4] = {L.x, L.y, L.z, L.w};
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            j[k] = jv[k];
            cd[k] = dv[k];
            oi[k] = ov[k];
            c[k] = lv[k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int64_t i = i0 + k;
            j[k] = i < n ? cand_j[i] : kNone;
            cd[k] = j[k] != kNone ? cand_d[i] : 0u;
            oi[k] = j[k] != kNone ? orig[i] : 0u;
            c[k] = j[k] != kNone ? labels[i] : 0u;
        }
    }
    uint64_t ck[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) ck[k] = j[k] != kNone ? compkey[c[k]] : 0ull;  // loads in flight together
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (j[k] == kNone) continue;  // no candidate
        const uint64_t key = ((uint64_t)cd[k] << 32) | (uint64_t)min(oi[k], j[k]);
        if (key == ck[k]) {
            atomicMin(&compmax[c[k]], max(oi[k], j[k]));
            succ[c[k]] = labels[cand_p[i0 + k]];
        }
    }
}

// The components of a round, as a list: k_merge_parent leaves the roots it
// finds (the components of the next round) in its workgroup's segment of
// `out`, `cap` entries from cap * blockIdx.x on, and their number in
// cnt_out[blockIdx.x].  From the second round on the merge kernels run with
// that many workgroups and visit the entries of `in` (the list of the round
// before) instead of testing labels[c] == c at every position.  Order inside
// a segment does not matter: every component's work is independent.
struct RootList {
    const uint32_t* in;
    const uint32_t* cnt_in;
    uint32_t* out;
    uint32_t* cnt_out;
    int64_t cap;
};

// Merge, step 1 (the successors come from stage B, or in the first round
// from the traversal): the chains of successors end in a mutual pair (Section 2);
// the smaller label of that pair becomes the root of the merged component
// ("Merging components together").  Every other component emits its edge,
// so a mutual pair contributes its shared edge once.  Roots reset their
// per-component state for the next round.
// With `first` the workgroups stride over every position (the segment of
// workgroup b then has room for every position it visits); otherwise each
// visits its segment of the root list.
__global__ __launch_bounds__(256) void k_merge_parent(const uint32_t* __restrict__ labels,
                                                      const uint32_t* __restrict__ succ, uint32_t* par,
                                                      uint64_t* compkey, uint32_t* compmax, uint32_t* ub,
                                                      uint4* __restrict__ eud, uint2* __restrict__ part,
                                                      Ctrl* ctrl, int64_t n, bool first, RootList rl,
                                                      bool allow_isolated) {
    if (ctrl->done) return;
    __shared__ uint32_t s_cnt[2];
    if (threadIdx.x < 2) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    uint32_t emitted = 0;
    const uint32_t* seg_in = rl.in + rl.cap * blockIdx.x;
    uint32_t* seg_out = rl.out + rl.cap * blockIdx.x;
    const int64_t cnt = first ? 0 : rl.cnt_in[blockIdx.x];
    // the lanes of a wave take consecutive entries, so the loop is uniform
    // per wave, and a wave appends its roots in lane order (segments stay
    // runs of ascending positions)
    const int lane = lane_id();
    const int64_t w0 = (first ? (int64_t)blockIdx.x * blockDim.x + threadIdx.x : (int64_t)threadIdx.x) - lane;
    const int64_t step = first ? (int64_t)gridDim.x * blockDim.x : (int64_t)blockDim.x;
    const int64_t end = first ? n : cnt;
    for (int64_t w = w0; w < end; w += step) {
        const int64_t i = w + lane;
        int64_t c = 0;
        bool comp = i < end;
        if (comp) {
            c = first ? i : (int64_t)seg_in[i];
            comp = !first || labels[c] == (uint32_t)c;
        }
        bool root = false;
        if (comp) {
            const uint32_t s = succ[c];
            // only a component that is a whole cloud of a batch has no edge
            if (s == (uint32_t)c && !allow_isolated) atomicOr(&ctrl->error, kErrNoEdge);
            root = (s == (uint32_t)c) || (succ[s] == (uint32_t)c && (uint32_t)c < s);
            par[c] = root ? (uint32_t)c : s;
        }
        const uint64_t rm = __ballot(root);
        if (rm) {
            uint32_t at = 0u;
            if (lane == 0) at = atomicAdd(&s_cnt[0], (uint32_t)__popcll(rm));
            at = (uint32_t)__shfl((int)at, 0);
            if (root) seg_out[at + (uint32_t)__popcll(rm & ((1ull << lane) - 1ull))] = (uint32_t)c;
        }
        if (!comp) continue;
        if (root) {
            ub[c] = kInfBits;
            compkey[c] = kKeyMax;
            compmax[c] = kNone;
            eud[c] = make_uint4(kNone, kNone, kNone, 0u);  // a final root's slot keeps this and sorts last
        } else {
            // a component id stops being one once it is merged, so every id
            // emits at most once over the whole run: its slot is its own
            ++emitted;
            const uint64_t key = compkey[c];
            eud[c] = make_uint4((uint32_t)(key & 0xFFFFFFFFu), compmax[c], (uint32_t)(key >> 32), 0u);
        }
    }
    for (int off = 32; off > 0; off >>= 1) emitted += __shfl_xor(emitted, off);
    if (lane_id() == 0 && emitted) atomicAdd(&s_cnt[1], emitted);
    __syncthreads();
    // (new roots, emitted edges) of this workgroup; k_relabel adds them up
    if (threadIdx.x == 0) {
        part[blockIdx.x] = make_uint2(s_cnt[0], s_cnt[1]);
        rl.cnt_out[blockIdx.x] = s_cnt[0];
    }
}

// Merge, step 3: pointer jumping towards the roots.  Concurrent updates only
// ever replace a pointer by one of its ancestors, so any interleaving is
// safe; the loop is capped and the relabel step finishes any remaining hops.
__device__ __forceinline__ void merge_jump_one(int64_t c, uint32_t* par, int steps) {
    uint32_t p = load_relaxed(&par[c]);
    for (int it = 0; it < steps; ++it) {
        const uint32_t pp = load_relaxed(&par[p]);
        if (pp == p) return;
        __hip_atomic_store(&par[c], pp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        p = pp;
    }
}

// First round: one thread per position.  Later rounds: the root list of the
// round (the components that k_merge_parent has just linked).
__global__ __launch_bounds__(256) void k_merge_jump(const uint32_t* __restrict__ labels, uint32_t* par,
                                                    int64_t n, int steps, const Ctrl* ctrl, bool first,
                                                    RootList rl) {
    if (ctrl->done) return;
    if (first) {
        const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (c < n && labels[c] == (uint32_t)c) merge_jump_one(c, par, steps);
        return;
    }
    const uint32_t* seg = rl.in + rl.cap * blockIdx.x;
    const int64_t cnt = rl.cnt_in[blockIdx.x];
    for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) merge_jump_one(seg[i], par, steps);
}

// Merge, step 4: every point takes its component's root as its new label
// (following any hops the jumping step left, up to a cap), and every tile
// leaves the run partials of the new labels for the next round (see
// k_run_partials).  The labels of the two positions just outside the tile
// are read while their own tiles rewrite them; the old and the new value
// lead to the same root, so either serves.  It is the last kernel of a
// round: workgroup 0 also totals k_merge_parent's partials into the new
// component count and raises `done` once that reaches the loop's target,
// so that every kernel of a round already queued behind this one returns
// at once (this kernel itself always runs: on a finished loop it rewrites
// the same labels).
__global__ __launch_bounds__(256) void k_relabel(uint32_t* labels, const uint32_t* __restrict__ par, int64_t n,
                                                 int steps, uint32_t* __restrict__ tile_part,
                                                 const uint2* __restrict__ part, int nparts, Ctrl* ctrl,
                                                 int64_t target) {
    __shared__ uint32_t s_new[kRunLds];
    __shared__ uint32_t s_w[8];
    const int tid = threadIdx.x;
    if (blockIdx.x == 0) {
        // (unless the loop had already finished, when k_merge_parent left
        // its partials untouched)
        const bool was_done = ctrl->done != 0u;
        uint32_t r = 0, e = 0;
        for (int b = tid; b < nparts; b += blockDim.x) {
            r += part[b].x;
            e += part[b].y;
        }
        for (int off = 32; off > 0; off >>= 1) {
            r += __shfl_xor(r, off);
            e += __shfl_xor(e, off);
        }
        if (lane_id() == 0) { s_w[tid / 64] = r; s_w[4 + tid / 64] = e; }
        __syncthreads();
        if (tid == 0 && !was_done) {
            r = s_w[0] + s_w[1] + s_w[2] + s_w[3];
            e = s_w[4] + s_w[5] + s_w[6] + s_w[7];
            ctrl->ncomp_next = r;
            ctrl->edge_count += e;
            ctrl->rounds_run += 1u;
            // the loop ends here (or stops on an error)
            if ((int64_t)r <= target || ctrl->error) ctrl->done = 1u;
        }
        __syncthreads();
    }
    const int64_t base = (int64_t)blockIdx.x * kRunTile;
    // thread 0 also follows position base-1, thread 1 position base+kRunTile
    const int64_t hp = tid == 0 ? base - 1 : (tid == 1 ? base + kRunTile : -1);
    const bool halo = hp >= 0 && hp < n;
    uint32_t r[kRunPer];
    uint32_t h = halo ? labels[hp] : 0u;
#pragma unroll
    for (int q = 0; q < kRunPer; ++q) {
        const int64_t p = base + (int64_t)q * 256 + tid;
        r[q] = p < n ? labels[p] : 0u;
    }
#pragma unroll
    for (int q = 0; q < kRunPer; ++q)
        if (base + (int64_t)q * 256 + tid < n) r[q] = par[r[q]];
    if (halo) h = par[h];
    // finish the chains in lockstep: one batch of independent loads per hop
    bool more = true;
    for (int it = 0; it < steps && more; ++it) {
        more = false;
        uint32_t rr[kRunPer];
#pragma unroll
        for (int q = 0; q < kRunPer; ++q) rr[q] = (base + (int64_t)q * 256 + tid < n) ? par[r[q]] : r[q];
        const uint32_t hh = halo ? par[h] : h;
#pragma unroll
        for (int q = 0; q < kRunPer; ++q) {
            more |= rr[q] != r[q];
            r[q] = rr[q];
        }
        more |= hh != h;
        h = hh;
    }
    if (more) atomicOr(&ctrl->error, kErrJump);
#pragma unroll
    for (int q = 0; q < kRunPer; ++q) {
        const int x = q * 256 + tid;
        if (base + x < n) labels[base + x] = r[q];
        s_new[run_lds(x + 1)] = r[q];
    }
    if (tid == 0) s_new[run_lds(0)] = h;
    if (tid == 1) s_new[run_lds(kRunTile + 1)] = h;
    __syncthreads();
    uint32_t hmax = 0u, tmin = kNone;
#pragma unroll
    for (int q = 0; q < kRunPer; ++q) {
        const int x = q * 256 + tid;
        const int64_t p = base + x;
        if (p < n) {
            const uint32_t l = s_new[run_lds(x + 1)];
            if (p == 0 || s_new[run_lds(x)] != l) hmax = max(hmax, (uint32_t)p);
            if (p == n - 1 || s_new[run_lds(x + 2)] != l) tmin = min(tmin, (uint32_t)p);
        }
    }
    block_max_min256(hmax, tmin, s_w);
    if (tid == 0) {
        tile_part[2 * blockIdx.x] = hmax;
        tile_part[2 * blockIdx.x + 1] = tmin;
    }
}

// ===========================================================================
// finalize

// Canonical edge order (the key K = (D, min, max) of every emitted edge).
// Component slot e holds (u, v, D bits) with u < v; the empty slots (the
// final root of each cloud) hold D = kNone and sort last.
//
// Fast path: sort the slots by the 64-bit key (D bits, u), then put every
// run of equal keys -- edges of exactly equal length at one endpoint u, at
// most a point's MST degree unless points coincide -- in v order in place.
// A run longer than kMaxTieRun raises long_ties and the caller redoes the
// order by the full path: by (u, v), then stably by D.  A batch finally
// sorts stably by cloud (a run never spans two clouds: u fixes the cloud).
// (Sorting by D alone, four passes, and ordering runs of equal D by (u, v)
// was measured and dropped: on the 37M-point cosmology cloud, where many
// short edges in dense halos share one float32 length, runs of equal D
// exceed any small bound and the full path then costs 9 ms more.)
constexpr int kMaxTieRun = 32;

// keys (D bits, u); values: the slot ids, or with v_values the v of every
// edge (one cloud: the sort then carries the whole edge, and the write
// reads it in order)
__global__ __launch_bounds__(256) void k_edge_du_keys(const uint4* __restrict__ eud, int64_t m,
                                                      uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                      bool v_values) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const uint4 s = eud[e];
    keys[e] = ((uint64_t)s.z << 32) | (uint64_t)s.x;
    vals[e] = v_values ? s.y : (uint32_t)e;
}

__global__ __launch_bounds__(256) void k_tie_fix(const uint64_t* __restrict__ keys, uint32_t* __restrict__ order,
                                                 const uint4* __restrict__ eud, int64_t m, Ctrl* ctrl,
                                                 bool v_values) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r + 1 >= m) return;
    const uint64_t k = keys[r];
    // one thread per run of two or more equal keys: its first position
    if (keys[r + 1] != k || (r > 0 && keys[r - 1] == k) || (uint32_t)(k >> 32) == kNone) return;
    int64_t e = r + 2;
    while (e < m && e - r <= kMaxTieRun && keys[e] == k) ++e;
    if (e - r > kMaxTieRun) {
        atomicOr(&ctrl->long_ties, 1u);
        return;
    }
    const int len = (int)(e - r);
    uint32_t id[kMaxTieRun];
    uint64_t uv[kMaxTieRun];
    for (int t = 0; t < len; ++t) {  // insertion sort by (u, v); u is the run's
        const uint32_t x = order[r + t];
        uint64_t y = x;  // v_values: the value is v
        if (!v_values) {
            const uint4 s = eud[x];
            y = ((uint64_t)s.x << 32) | s.y;
        }
        int q = t;
        while (q > 0 && uv[q - 1] > y) {
            uv[q] = uv[q - 1];
            id[q] = id[q - 1];
            --q;
        }
        uv[q] = y;
        id[q] = x;
    }
    for (int t = 0; t < len; ++t) order[r + t] = id[t];
}

// Full path, first pass: (u, v) keys of every slot.
__global__ __launch_bounds__(256) void k_edge_keys(const uint4* __restrict__ eud, int64_t m,
                                                   uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const uint4 s = eud[e];
    keys[e] = ((uint64_t)s.x << 32) | (uint64_t)s.y;
    vals[e] = (uint32_t)e;
}

// keys[i] = D bits of slot perm[i]
__global__ __launch_bounds__(256) void k_edge_dkeys(const uint4* __restrict__ eud, const uint32_t* __restrict__ perm,
                                                    int64_t m, uint64_t* __restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    keys[i] = (uint64_t)eud[perm[i]].z;
}

// keys[i] = src[perm[i]]
__global__ __launch_bounds__(256) void k_perm_keys(const uint32_t* __restrict__ src,
                                                   const uint32_t* __restrict__ perm, int64_t m,
                                                   uint64_t* __restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    keys[i] = (uint64_t)src[perm[i]];
}

// One cloud: edge i is (u, v) = (low word of keys[i], v[i]) with D bits
// the high word, all read in order.
__global__ __launch_bounds__(256) void k_edge_write_kv(const uint64_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ v, int64_t m,
                                                       int32_t* __restrict__ edges, float* __restrict__ w,
                                                       float* __restrict__ d2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint64_t k = keys[i];
    const float d = bitsf((uint32_t)(k >> 32));
    reinterpret_cast<int2*>(edges)[i] = make_int2((int32_t)(uint32_t)k, (int32_t)v[i]);
    w[i] = edge_weight(d);
    if (d2) d2[i] = d;
}

__global__ __launch_bounds__(256) void k_edge_write(const uint4* __restrict__ eud, const uint32_t* __restrict__ perm,
                                                    int64_t m, int32_t* __restrict__ edges, float* __restrict__ w,
                                                    float* __restrict__ d2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint4 s = eud[perm[i]];
    const float d = bitsf(s.z);
    reinterpret_cast<int2*>(edges)[i] = make_int2((int32_t)s.x, (int32_t)s.y);
    w[i] = edge_weight(d);
    if (d2) d2[i] = d;
}

// ===========================================================================
// batches: many independent clouds in one pass
//
// Every cloud gets its own scene box and Morton quantisation, and its cloud
// id becomes the top bits of its codes.  One sort then groups each cloud in
// a contiguous range of sorted positions, and in the one radix tree built
// over all codes every cloud with two or more points is exactly one subtree
// (all keys with the cloud-id prefix, and only those).

struct CloudIn {       // host -> device, per cloud
    int64_t off;       // first point (input order = sorted order per cloud)
    int64_t n;         // points
    int64_t foff;      // first float of the cloud in the input array
    int64_t eoff;      // first output edge
    int32_t dim;
    int32_t pad;
};
struct CloudBox {      // device -> host, per cloud
    uint32_t mn[3], mx[3];
    uint32_t bad;
    uint32_t pad;
};
struct CloudMorton {   // host -> device, per cloud
    double lo[3], scale[3], qmax;
    int32_t dim, bits;
};

// Empty per-cloud boxes for k_batch_unpack to grow (a cloud without points
// keeps the box [0, 0]).
__global__ __launch_bounds__(256) void k_batch_box_init(const CloudIn* __restrict__ cin, int32_t B,
                                                        CloudBox* __restrict__ cbox) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= B) return;
    const bool any = cin[c].n > 0;
    CloudBox cb;
    for (int k = 0; k < 3; ++k) {
        cb.mn[k] = ord_enc(any ? INFINITY : 0.f);
        cb.mx[k] = ord_enc(any ? -INFINITY : 0.f);
    }
    cb.bad = 0;
    cb.pad = 0;
    cbox[c] = cb;
}

// The cloud holding point g: the last cloud whose first point is at or
// before g (an empty cloud shares its first point with the next cloud, so
// the last of them is the one that holds g).
__device__ __forceinline__ int cloud_at(const CloudIn* __restrict__ cin, int32_t B, int64_t g) {
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cin[mid].off <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void box_flush(CloudBox* __restrict__ cb, const float* lo, const float* hi, bool bad) {
    for (int k = 0; k < 3; ++k) {
        atomicMin(&cb->mn[k], ord_enc(lo[k]));
        atomicMax(&cb->mx[k], ord_enc(hi[k]));
    }
    if (bad) atomicOr(&cb->bad, 1u);
}

// Unpack to 3D (z = 0 for 2D clouds; + 0 adds exactly, so D is unchanged),
// record each point's cloud and grow the cloud boxes (min / max ignore a
// NaN; a non-finite coordinate marks the cloud bad).  One workgroup per
// kUnpackPts consecutive points, so a large cloud spreads over many
// workgroups: a workgroup inside one cloud reduces its box in LDS and merges
// it with one set of atomics; one that spans clouds merges per thread at
// every cloud change.
constexpr int64_t kUnpackPts = 4096;
__global__ __launch_bounds__(256) void k_batch_unpack(const float* __restrict__ pts, const CloudIn* __restrict__ cin,
                                                      int32_t B, int64_t n, float* __restrict__ pts3,
                                                      uint32_t* __restrict__ cloud_of, CloudBox* __restrict__ cbox) {
    __shared__ float s_lo[4][3], s_hi[4][3];
    __shared__ uint32_t s_bad[4];
    __shared__ int s_c[2];
    const int64_t base = (int64_t)blockIdx.x * kUnpackPts;
    const int64_t end = base + kUnpackPts < n ? base + kUnpackPts : n;
    if (threadIdx.x == 0) {
        s_c[0] = cloud_at(cin, B, base);
        s_c[1] = cloud_at(cin, B, end - 1);
    }
    __syncthreads();
    const bool one = s_c[0] == s_c[1];
    int c = s_c[0];
    CloudIn ci = cin[c];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false, any = false;
    for (int64_t g = base + threadIdx.x; g < end; g += blockDim.x) {
        if (!one) {
            while (g >= ci.off + ci.n) {  // past this cloud (empty clouds are skipped)
                if (any) box_flush(cbox + c, lo, hi, bad);
                for (int k = 0; k < 3; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
                bad = any = false;
                ci = cin[++c];
            }
        }
        const int64_t q = g - ci.off;
        float x[3] = {0.f, 0.f, 0.f};
        for (int k = 0; k < ci.dim; ++k) x[k] = pts[ci.foff + q * ci.dim + k];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            pts3[3 * g + k] = x[k];
            bad |= !isfinite(x[k]);
            lo[k] = fminf(lo[k], x[k]);
            hi[k] = fmaxf(hi[k], x[k]);
        }
        cloud_of[g] = (uint32_t)c;
        any = true;
    }
    if (!one) {
        if (any) box_flush(cbox + c, lo, hi, bad);
        return;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
        for (int off = 32; off > 0; off >>= 1) {
            lo[k] = fminf(lo[k], __shfl_xor(lo[k], off));
            hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off));
        }
    const bool any_bad = __ballot(bad) != 0ull;
    const int w = threadIdx.x / 64;
    if (lane_id() == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) { s_lo[w][k] = lo[k]; s_hi[w][k] = hi[k]; }
        s_bad[w] = any_bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        bool b = false;
        for (int v = 0; v < 4; ++v) {
            b |= s_bad[v] != 0;
            for (int k = 0; k < 3; ++k) { lo[k] = fminf(lo[k], s_lo[v][k]); hi[k] = fmaxf(hi[k], s_hi[v][k]); }
        }
        box_flush(cbox + c, lo, hi, b);
    }
}

static unsigned unpack_grid(int64_t n) { return (unsigned)((n + kUnpackPts - 1) / kUnpackPts); }

// Per-cloud quantisation from the per-cloud boxes, on the device: the same
// double operations as the host's morton_params, hence the same parameters.
// `avail` = code bits below the cloud id.
__global__ __launch_bounds__(256) void k_batch_mparams(const CloudBox* __restrict__ cbox,
                                                       const CloudIn* __restrict__ cin, int32_t B, int avail,
                                                       CloudMorton* __restrict__ cm) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= B) return;
    float lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = ord_dec(cbox[c].mn[k]);
        hi[k] = ord_dec(cbox[c].mx[k]);
    }
    const int dim = cin[c].dim;
    const int bits = min(dim == 3 ? 21 : 32, avail / dim);
    const MortonParams mp = morton_params(lo, hi, dim, bits);
    CloudMorton m;
    for (int k = 0; k < 3; ++k) {
        m.lo[k] = mp.lo[k];
        m.scale[k] = mp.scale[k];
    }
    m.qmax = mp.qmax;
    m.dim = dim;
    m.bits = bits;
    cm[c] = m;
}

__global__ __launch_bounds__(256) void k_batch_morton(const float* __restrict__ pts3,
                                                      const uint32_t* __restrict__ cloud_of,
                                                      const CloudMorton* __restrict__ cm, int64_t n, int cloud_shift,
                                                      uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                      uint64_t* part) {
    __shared__ uint64_t s_or[4], s_and[4];
    uint64_t kor = 0, kand = ~0ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t b = cloud_of[i];
        const CloudMorton m = cm[b];
        uint64_t q[3];
        for (int k = 0; k < 3; ++k) {
            double t = ((double)pts3[3 * i + k] - m.lo[k]) * m.scale[k];
            t = fmin(fmax(t, 0.0), m.qmax);
            q[k] = (uint64_t)t;
        }
        uint64_t code = (m.dim == 3) ? ((spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]))
                                     : ((spread2(q[0]) << 1) | spread2(q[1]));
        if (cloud_shift < 64) code |= (uint64_t)b << cloud_shift;
        keys[i] = code;
        vals[i] = (uint32_t)i;
        kor |= code;
        kand &= code;
    }
    for (int off = 32; off > 0; off >>= 1) {
        kor |= __shfl_xor(kor, off);
        kand &= __shfl_xor(kand, off);
    }
    const int w = threadIdx.x / 64;
    if (lane_id() == 0) { s_or[w] = kor; s_and[w] = kand; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < 4; ++v) { kor |= s_or[v]; kand &= s_and[v]; }
        part[2 * blockIdx.x] = kor;
        part[2 * blockIdx.x + 1] = kand;
    }
}

// Folds the nb (OR, AND) partials of k_batch_morton into the control block.
__global__ __launch_bounds__(256) void k_or_and_final(const uint64_t* __restrict__ part, int nb, Ctrl* ctrl) {
    __shared__ uint64_t s_or[4], s_and[4];
    uint64_t kor = 0, kand = ~0ull;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        kor |= part[2 * b];
        kand &= part[2 * b + 1];
    }
    for (int off = 32; off > 0; off >>= 1) {
        kor |= __shfl_xor(kor, off);
        kand &= __shfl_xor(kand, off);
    }
    const int w = threadIdx.x / 64;
    if (lane_id() == 0) { s_or[w] = kor; s_and[w] = kand; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < (int)blockDim.x / 64; ++v) { kor |= s_or[v]; kand &= s_and[v]; }
        ctrl->key_or = kor;
        ctrl->key_and = kand;
    }
}

// Cloud of every sorted position (sorting keeps clouds contiguous and in
// order, so it is also the cloud of every component slot).
__global__ __launch_bounds__(256) void k_batch_sorted_cloud(const uint32_t* __restrict__ cloud_of,
                                                            const uint32_t* __restrict__ perm, int64_t n,
                                                            uint32_t* __restrict__ cloud_sorted) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) cloud_sorted[i] = cloud_of[perm[i]];
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(64) void k_fill_u8(uint8_t* __restrict__ p, int64_t n, uint8_t v) {
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

// Counting runs: ctrl->touched += the number of set flags among f[0, m).
__global__ __launch_bounds__(256) void k_count_flags(const uint8_t* __restrict__ f, int64_t m, Ctrl* ctrl) {
    __shared__ uint32_t s_w[4];
    uint32_t cnt = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        cnt += f[i] != 0;
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(&ctrl->touched, (unsigned long long)(s_w[0] + s_w[1] + s_w[2] + s_w[3]));
}

// The subtree root of a cloud is the internal node whose leaf range is
// exactly the cloud's range of sorted positions.
__global__ __launch_bounds__(256) void k_cloud_roots(const uint32_t* __restrict__ rlo, const uint32_t* __restrict__ rhi,
                                                     const uint32_t* __restrict__ cloud_sorted,
                                                     const CloudIn* __restrict__ cin, int64_t m,
                                                     uint32_t* __restrict__ cloud_root) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const uint32_t lo = rlo[k], hi = rhi[k];
    const uint32_t b = cloud_sorted[lo];
    const CloudIn ci = cin[b];
    if ((int64_t)lo == ci.off && (int64_t)hi == ci.off + ci.n - 1) cloud_root[b] = (uint32_t)k;
}

// Sorted slot i -> output edge of its cloud, with cloud-local indices.
__global__ __launch_bounds__(256) void k_batch_edge_write(const uint4* __restrict__ eud,
                                                          const uint32_t* __restrict__ order,
                                                          const uint32_t* __restrict__ cloud_sorted,
                                                          const CloudIn* __restrict__ cin, int64_t n,
                                                          int32_t* __restrict__ edges, float* __restrict__ w,
                                                          float* __restrict__ d2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t e = order[i];
    const uint4 s = eud[e];
    if (s.z == kNone) return;
    const CloudIn ci = cin[cloud_sorted[e]];
    const int64_t o = ci.eoff + (i - ci.off);
    const float d = bitsf(s.z);
    edges[2 * o] = (int32_t)((int64_t)s.x - ci.off);
    edges[2 * o + 1] = (int32_t)((int64_t)s.y - ci.off);
    w[o] = edge_weight(d);
    if (d2) d2[o] = d;
}

// ===========================================================================
// workspace layout

struct Layout {
    size_t ctrl, bpart, k0, k1, v0, v1, hist, spts, orig, cand_p, recs, lab2, height, node_parent, leaf_parent, up, exch, rlo, rhi, run_part, run_carry, qcnt, qoff, qflag, qlist, labels, ub, compkey, compmax, succ, par, cand_d, cand_j, eud, core_s, core_o, total;
};

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct BatchLayout {
    Layout base;
    size_t pts3, cloud_of, cloud_sorted, cin, cbox, cm, croot, total;
};

static BatchLayout make_batch_layout(int64_t n, int64_t clouds);

// Root lists of the merge kernels: one segment per k_merge_parent
// workgroup, with room for every position that workgroup strides over.
static int root_list_blocks(int64_t n) { return (int)std::min<unsigned>(grid_for(n), kPartBlocks); }
static int64_t root_list_cap(int64_t n) {
    const int64_t stride = (int64_t)root_list_blocks(n) * 256;
    return (n + stride - 1) / stride * 256;
}

static Layout make_layout(int64_t n, int dim) {
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += align_up(bytes);
        return r;
    };
    const size_t N = (size_t)(n > 0 ? n : 1), M = (size_t)(n > 1 ? n - 1 : 1);
    L.ctrl = take(sizeof(Ctrl));
    L.bpart = take(32 * (size_t)kPartBlocks);
    // the key buffers also hold the root lists during the rounds
    const size_t keys = std::max<size_t>(8 * N, 4 * (size_t)root_list_blocks(n) * (size_t)root_list_cap(n));
    L.k0 = take(keys);
    L.k1 = take(keys);
    L.v0 = take(4 * N);
    L.v1 = take(4 * N);
    L.hist = take(4 * radix_scratch_elems(n));
    L.spts = take(4 * N * dim);
    L.orig = take(4 * N);
    L.cand_p = take(4 * N);
    L.recs = take(M * (dim == 3 ? sizeof(Rec<3>) : sizeof(Rec<2>)));
    L.lab2 = take(8 * M);
    L.height = take(M);
    L.node_parent = take(4 * M);
    L.leaf_parent = take(4 * N);
    L.up = take(sizeof(Up) * M);
    L.exch = take(8 * M);
    L.rlo = take(4 * M);
    L.rhi = take(4 * M);
    L.run_part = take(8 * (N / kRunTile + 2));
    L.run_carry = take(8 * (N / kRunTile + 2));
    L.qcnt = take(4 * (N / kRunTile + 2));
    L.qoff = take(4 * (N / kRunTile + 2));
    L.qflag = take(N);
    L.qlist = take(4 * N);
    L.labels = take(4 * N);
    L.ub = take(4 * N);
    L.compkey = take(8 * N);
    L.compmax = take(4 * N);
    L.succ = take(4 * N);
    L.par = take(4 * N);
    L.cand_d = take(4 * N);
    L.cand_j = take(4 * N);
    L.eud = take(16 * N);
    L.core_s = take(4 * N);
    L.core_o = take(4 * N);
    L.total = o;
    return L;
}

static BatchLayout make_batch_layout(int64_t n, int64_t clouds) {
    BatchLayout B;
    B.base = make_layout(n, 3);
    size_t o = B.base.total;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += align_up(bytes);
        return r;
    };
    const size_t N = (size_t)(n > 0 ? n : 1), C = (size_t)(clouds > 0 ? clouds : 1);
    B.pts3 = take(12 * N);
    B.cloud_of = take(4 * N);
    B.cloud_sorted = take(4 * N);
    B.cin = take(sizeof(CloudIn) * C);
    B.cbox = take(sizeof(CloudBox) * C);
    B.cm = take(sizeof(CloudMorton) * C);
    B.croot = take(4 * C);
    B.total = o;
    return B;
}

}  // namespace emst

// ===========================================================================
// C ABI

using namespace emst;

// traversal variants: 0, 5, 7, 8, 10, 11 and 13 (the default)
constexpr uint32_t kVariants = (1u << 0) | (1u << 5) | (1u << 7) | (1u << 8) | (1u << 10) | (1u << 11) | (1u << 13);
static inline bool variant_ok(int v) { return v >= 0 && v < 32 && ((kVariants >> v) & 1u); }

// Device memory of the allocation-free entry point (emst_build_noalloc):
// its workspace is this array, which every device the library runs on holds
// from the code object's load until the process ends.  Host code never
// passes its name to a kernel: it takes the device address that
// hipGetSymbolAddress returns for the current device (scratch_address).
static __device__ __align__(256) unsigned char scratch[EMST_NOALLOC_WORKSPACE_BYTES];

// The address of `scratch` on each device, looked up once per device with
// that device current.
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];

static hipError_t scratch_address(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();  // leave no sticky error for the next launch check
            return e != hipSuccess ? e : hipErrorInvalidSymbol;
        }
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

struct emst_ctx {
    int device = 0;
    void* scratch = nullptr;       // this device's `scratch` (null if the lookup failed)
    std::string scratch_err;
    std::string err;
    bool profiling = false;
    bool counting = false;
    int traversal = -1;            // -1: the autotune table, else the built-in choice
    int lds_depth = 0;             // 0: the autotune table, else 4, 8 or 16 (variant 13)
    TuneTable tune;
    emst_stats stats;
    Ctrl* h_ctrl = nullptr;        // pinned host mirror of the control block
    hipEvent_t ev[2 * 64 + 8];
    bool ev_ok = false;
    hipEvent_t sev[2] = {nullptr, nullptr};  // completion of the control copies of two rounds in flight
    void* h_stage = nullptr;       // pinned host staging for per-cloud tables
    size_t h_stage_bytes = 0;
    // captured round pairs of batches (emst_set_graphs): a few instantiated
    // graphs, keyed by everything their launches bake in
    bool graphs = false;
    hipStream_t cap_stream = nullptr;
    struct GraphEntry {
        const void* ws;
        int64_t n, target;
        int variant, height;
        const void* cloud_of;
        uint32_t root;
        int lds_depth;
        hipGraphExec_t exec;
        uint64_t used;
    };
    std::vector<GraphEntry> gcache;
    uint64_t gclock = 0;
};

// Pinned host memory of at least `bytes` (host memory only; the library
// never allocates device memory).
static void* stage(emst_ctx* ctx, size_t bytes) {
    if (ctx->h_stage_bytes >= bytes) return ctx->h_stage;
    if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
    ctx->h_stage = nullptr;
    ctx->h_stage_bytes = 0;
    if (hipHostMalloc(&ctx->h_stage, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
    ctx->h_stage_bytes = bytes;
    return ctx->h_stage;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t _e = (expr);                                                          \
        if (_e != hipSuccess) {                                                          \
            ctx->err = std::string(#expr) + ": " + hipGetErrorString(_e);                \
            return EMST_EHIP;                                                            \
        }                                                                                \
    } while (0)

static int fail(emst_ctx* ctx, int code, const char* msg) {
    if (ctx) ctx->err = msg;
    return code;
}

// The traversal shape of a call: the context's explicit choices, else the
// autotune table's entry for (mode, dim, n), else variant 13 with an 8-deep
// LDS ring.
static void pick_shape(const emst_ctx* ctx, int batched, int dim, int64_t n, int* variant, int* depth) {
    const TuneEntry* e = ctx->tune.pick(batched, dim, n);
    *variant = ctx->traversal >= 0 ? ctx->traversal : (e ? e->variant : 13);
    *depth = ctx->lds_depth > 0 ? ctx->lds_depth : (e ? e->lds_depth : 8);
}

extern "C" int emst_create(emst_ctx** out, int hip_device, const char* autotune_json) {
    if (!out) return EMST_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count) return EMST_EINVAL;
    emst_ctx* ctx = new (std::nothrow) emst_ctx();
    if (!ctx) return EMST_ENOMEM;
    ctx->device = hip_device;
    if (autotune_json && !ctx->tune.parse(autotune_json, kVariants, nullptr)) {
        delete ctx;
        return EMST_EINVAL;
    }
    memset(&ctx->stats, 0, sizeof(ctx->stats));
    if (hipSetDevice(hip_device) != hipSuccess ||
        hipHostMalloc((void**)&ctx->h_ctrl, 2 * sizeof(Ctrl) + 256, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->sev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->sev[1], hipEventDisableTiming) != hipSuccess) {
        for (auto& e : ctx->sev)
            if (e) (void)hipEventDestroy(e);
        if (ctx->h_ctrl) (void)hipHostFree(ctx->h_ctrl);
        delete ctx;
        return EMST_EHIP;
    }
    ctx->ev_ok = true;
    for (auto& e : ctx->ev)
        if (hipEventCreate(&e) != hipSuccess) ctx->ev_ok = false;
    // the allocation-free entry point's workspace on this device (the
    // device is current); a failed lookup only disables that entry point
    if (const hipError_t e = scratch_address(hip_device, &ctx->scratch); e != hipSuccess)
        ctx->scratch_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    *out = ctx;
    return EMST_OK;
}

extern "C" void emst_destroy(emst_ctx* ctx) {
    if (!ctx) return;
    for (auto& g : ctx->gcache) (void)hipGraphExecDestroy(g.exec);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    for (auto& e : ctx->ev) (void)hipEventDestroy(e);
    for (auto& e : ctx->sev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->h_ctrl) (void)hipHostFree(ctx->h_ctrl);
    if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
    delete ctx;
}

extern "C" const char* emst_last_error(const emst_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" size_t emst_workspace_bytes(int64_t n, int dim) {
    if (n < 0 || n > 0x7FFFFFFFll || (dim != 2 && dim != 3)) return 0;
    return make_layout(n, dim).total;
}

extern "C" int emst_set_profiling(emst_ctx* ctx, int on) {
    if (!ctx) return EMST_EINVAL;
    ctx->profiling = on != 0;
    return EMST_OK;
}
extern "C" int emst_set_lds_depth(emst_ctx* ctx, int depth) {
    if (!ctx || (depth != 0 && depth != 4 && depth != 8 && depth != 16)) return EMST_EINVAL;
    ctx->lds_depth = depth;
    return EMST_OK;
}
extern "C" int emst_set_graphs(emst_ctx* ctx, int on) {
    if (!ctx) return EMST_EINVAL;
    ctx->graphs = on != 0;
    return EMST_OK;
}
extern "C" int emst_set_counting(emst_ctx* ctx, int on) {
    if (!ctx) return EMST_EINVAL;
    ctx->counting = on != 0;
    return EMST_OK;
}
extern "C" int emst_set_traversal(emst_ctx* ctx, int variant) {
    if (!ctx || (variant != -1 && !variant_ok(variant))) return EMST_EINVAL;
    ctx->traversal = variant;
    return EMST_OK;
}
extern "C" int emst_set_autotune(emst_ctx* ctx, const char* json) {
    if (!ctx) return EMST_EINVAL;
    ctx->err.clear();
    if (!json) {
        ctx->tune.clear();
        return EMST_OK;
    }
    if (!ctx->tune.parse(json, kVariants, &ctx->err)) return EMST_EINVAL;
    return EMST_OK;
}
extern "C" int emst_get_autotune(const emst_ctx* ctx, char* buf, size_t cap, size_t* len) {
    if (!ctx) return EMST_EINVAL;
    const std::string s = ctx->tune.dump();
    if (len) *len = s.size() + 1;
    if (!buf || cap < s.size() + 1) return buf ? EMST_ENOMEM : EMST_OK;
    memcpy(buf, s.c_str(), s.size() + 1);
    return EMST_OK;
}
extern "C" int emst_get_stats(const emst_ctx* ctx, emst_stats* out) {
    if (!ctx || !out) return EMST_EINVAL;
    *out = ctx->stats;
    return EMST_OK;
}

namespace {

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
    return ms;
}

// Every D is at most the squared extent of the box, evaluated in the same
// order, so a finite squared extent means no D overflows.
bool extent_ok(const float* lo, const float* hi, int dim) {
    volatile float s = 0.f;
    for (int k = 0; k < dim; ++k) {
        volatile float g = hi[k] - lo[k];
        volatile float g2 = g * g;
        s = (k == 0) ? (float)g2 : (float)(s + g2);
    }
    return isfinite((float)s);
}

// The record labels of arbitrary labels (no bounds).
hipError_t propagate_labels(const uint32_t* labels, uint32_t* run_part, uint32_t* run_carry, const uint32_t* rlo,
                            const uint32_t* rhi, uint2* lab2, int64_t n, Ctrl* ctrl, hipStream_t st) {
    const int nb = run_tiles(n);
    k_run_partials<<<nb, 256, 0, st>>>(labels, n, run_part);
    k_tile_carries<<<1, 1024, 0, st>>>(run_part, nb, run_carry, ctrl);
    k_round_prep<3, false, false><<<nb, 256, 0, st>>>(labels, run_carry, rlo, rhi, lab2, nullptr, nullptr, nullptr,
                                                      n, nullptr, ctrl, nullptr, nb, KeepArgs{}, nullptr);
    return hipGetLastError();
}

// All device arrays of one build, carved from the workspace.
template <int DIM>
struct Bufs {
    Ctrl* ctrl;
    uint32_t* bpart;  // per-workgroup partials (kPartBlocks x 32 bytes)
    uint64_t *k0, *k1;
    uint32_t *v0, *v1, *hist;
    float* spts;
    uint32_t *orig, *cand_p;
    Rec<DIM>* recs;
    uint2* lab2;
    uint8_t* height;
    uint32_t *node_parent, *leaf_parent;
    Up* up;
    uint64_t* exch;
    uint32_t *rlo, *rhi, *run_part, *run_carry, *labels, *ub;
    uint32_t *qcnt, *qoff, *qlist;
    uint8_t* qflag;
    uint64_t* compkey;
    uint32_t *compmax, *succ, *par, *cand_d, *cand_j;
    uint4* eud;
    float *core_s, *core_o;
};

template <int DIM>
Bufs<DIM> carve(char* ws, const Layout& L) {
    Bufs<DIM> b;
    b.ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
    b.bpart = reinterpret_cast<uint32_t*>(ws + L.bpart);
    b.k0 = reinterpret_cast<uint64_t*>(ws + L.k0);
    b.k1 = reinterpret_cast<uint64_t*>(ws + L.k1);
    b.v0 = reinterpret_cast<uint32_t*>(ws + L.v0);
    b.v1 = reinterpret_cast<uint32_t*>(ws + L.v1);
    b.hist = reinterpret_cast<uint32_t*>(ws + L.hist);
    b.spts = reinterpret_cast<float*>(ws + L.spts);
    b.orig = reinterpret_cast<uint32_t*>(ws + L.orig);
    b.cand_p = reinterpret_cast<uint32_t*>(ws + L.cand_p);
    b.recs = reinterpret_cast<Rec<DIM>*>(ws + L.recs);
    b.lab2 = reinterpret_cast<uint2*>(ws + L.lab2);
    b.height = reinterpret_cast<uint8_t*>(ws + L.height);
    b.node_parent = reinterpret_cast<uint32_t*>(ws + L.node_parent);
    b.leaf_parent = reinterpret_cast<uint32_t*>(ws + L.leaf_parent);
    b.up = reinterpret_cast<Up*>(ws + L.up);
    b.exch = reinterpret_cast<uint64_t*>(ws + L.exch);
    b.rlo = reinterpret_cast<uint32_t*>(ws + L.rlo);
    b.rhi = reinterpret_cast<uint32_t*>(ws + L.rhi);
    b.run_part = reinterpret_cast<uint32_t*>(ws + L.run_part);
    b.run_carry = reinterpret_cast<uint32_t*>(ws + L.run_carry);
    b.qcnt = reinterpret_cast<uint32_t*>(ws + L.qcnt);
    b.qoff = reinterpret_cast<uint32_t*>(ws + L.qoff);
    b.qflag = reinterpret_cast<uint8_t*>(ws + L.qflag);
    b.qlist = reinterpret_cast<uint32_t*>(ws + L.qlist);
    b.labels = reinterpret_cast<uint32_t*>(ws + L.labels);
    b.ub = reinterpret_cast<uint32_t*>(ws + L.ub);
    b.compkey = reinterpret_cast<uint64_t*>(ws + L.compkey);
    b.compmax = reinterpret_cast<uint32_t*>(ws + L.compmax);
    b.succ = reinterpret_cast<uint32_t*>(ws + L.succ);
    b.par = reinterpret_cast<uint32_t*>(ws + L.par);
    b.cand_d = reinterpret_cast<uint32_t*>(ws + L.cand_d);
    b.cand_j = reinterpret_cast<uint32_t*>(ws + L.cand_j);
    b.eud = reinterpret_cast<uint4*>(ws + L.eud);
    b.core_s = reinterpret_cast<float*>(ws + L.core_s);
    b.core_o = reinterpret_cast<float*>(ws + L.core_o);
    return b;
}

template <int DIM>
TraverseArgs<DIM> traverse_args(const Bufs<DIM>& b, int64_t n, uint32_t root) {
    TraverseArgs<DIM> ta;
    ta.spts = b.spts; ta.labels = b.labels; ta.orig = b.orig; ta.ub = b.ub; ta.recs = b.recs; ta.root = root;
    ta.n = n; ta.cand_d = b.cand_d; ta.cand_j = b.cand_j; ta.compkey = b.compkey; ta.compmax = b.compmax;
    ta.ctrl = b.ctrl; ta.first = true; ta.up = b.up;
    ta.cloud_of = nullptr; ta.cloud_root = nullptr; ta.lab2 = b.lab2;
    ta.wave_lca = reinterpret_cast<const uint32_t*>(b.exch);  // the build's exchange words are free by now
    ta.core_s = nullptr;
    ta.core_o = nullptr;
    ta.cand_p = b.cand_p;
    ta.succ = b.succ;
    ta.qlist = nullptr;
    ta.touched = nullptr;
    ta.kept = nullptr;
    ta.all_absorbed = false;
    ta.lds_depth = 8;
    return ta;
}

int read_ctrl(emst_ctx* ctx, Ctrl* ctrl, hipStream_t st) {
    HIP_TRY(hipMemcpyAsync(ctx->h_ctrl, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return EMST_OK;
}

// Boruvka rounds until the component count reaches `target` (1 for one
// cloud, the number of non-empty clouds for a batch).  With cloud_of set,
// Morton neighbours in different clouds bound nothing, every query searches
// its own cloud's subtree, and a component without an outgoing edge (its
// cloud is finished) becomes a root.
// Variant 13 searches from a query list from the third round on (the
// second keeps nothing: in the first round every point joins its nearest
// neighbour's component).  Below kQlistMinN points the list's extra
// launches per round cost more than the idle lanes they save, and the
// points skip inside the traversal instead (measured crossover between
// 5e5 and 1e6 points).
constexpr int64_t kQlistMinN = (int64_t)3 << 18;
static inline bool uses_qlist(int variant, int round, int64_t n) {
    return variant == 13 && round >= 2 && n >= kQlistMinN;
}

// Test hook support (emst_test_round): the state of a round between stage
// B and the merge, per point in input order.
struct RoundCapture {
    float* bound;       // bound of the point's component
    float* cand_d;      // the point's candidate D, +inf if none
    int32_t* cand_j;    // its original index, -1 if none
    float* comp_d2;     // the component's edge (D, u, v), D = +inf if none
    int32_t* comp_u;
    int32_t* comp_v;
};

__global__ __launch_bounds__(256) void k_test_capture(const uint32_t* __restrict__ labels,
                                                      const uint32_t* __restrict__ orig,
                                                      const uint32_t* __restrict__ ub,
                                                      const uint32_t* __restrict__ cand_d,
                                                      const uint32_t* __restrict__ cand_j,
                                                      const uint64_t* __restrict__ compkey,
                                                      const uint32_t* __restrict__ compmax, int64_t n,
                                                      RoundCapture cap) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t o = orig[p], c = labels[p];
    cap.bound[o] = bitsf(ub[c]);
    const uint32_t j = cand_j[p];
    cap.cand_d[o] = j == kNone ? INFINITY : bitsf(cand_d[p]);
    cap.cand_j[o] = j == kNone ? -1 : (int32_t)j;
    const uint64_t key = compkey[c];
    const uint32_t v = compmax[c];
    const bool has = key != kKeyMax && v != kNone;
    cap.comp_d2[o] = has ? bitsf((uint32_t)(key >> 32)) : INFINITY;
    cap.comp_u[o] = has ? (int32_t)(uint32_t)key : -1;
    cap.comp_v[o] = has ? (int32_t)v : -1;
}

// One Boruvka round, enqueued on st (no host wait).
template <int DIM>
int enqueue_round(emst_ctx* ctx, Bufs<DIM>& b, TraverseArgs<DIM>& ta, int64_t n, int round, int height,
                  int variant, const uint32_t* cloud_of, int64_t target, bool prof, hipStream_t st,
                  const RoundCapture* cap = nullptr) {
    hipEvent_t* E = ctx->ev;
    // record labels and bounds; the run partials of round r > 0 come from
    // the relabel kernel of round r - 1
    const int nt = run_tiles(n);
    const bool fold = nt <= kFoldTiles;  // scans folded into their consumers
    // variant 13 from the third round on: kept candidates are offered here
    // (in round 1 none is kept: every point joined its candidate's
    // component in round 0)
    const bool keep = variant == 13 && round >= 2;
    const KeepArgs ka = keep ? KeepArgs{b.cand_d, b.cand_j, b.cand_p, b.orig, b.compkey, b.qflag} : KeepArgs{};
    if (round == 0) {
        k_round_prep<DIM, true, true><<<nt, 256, 0, st>>>(b.labels, b.run_carry, b.rlo, b.rhi, b.lab2, b.spts,
                                                          cloud_of, ta.core_s, n, b.ub, b.ctrl, nullptr, nt, ka,
                                                          b.succ);
    } else {
        if (!fold) k_tile_carries<<<1, 1024, 0, st>>>(b.run_part, nt, b.run_carry, b.ctrl);
        k_round_prep<DIM, false, true><<<nt, 256, 0, st>>>(b.labels, b.run_carry, b.rlo, b.rhi, b.lab2, b.spts,
                                                           cloud_of, ta.core_s, n, b.ub, b.ctrl,
                                                           fold ? b.run_part : nullptr, nt, ka, b.succ);
    }
    ta.first = round == 0;
    ta.all_absorbed = round == 1;
    ta.kept = keep ? b.qflag : nullptr;
    // variant 13: only the points whose last result no longer holds search
    ta.qlist = nullptr;
    if (uses_qlist(variant, round, n)) {
        ta.kept = nullptr;
        k_reuse_mark<<<nt, 256, 0, st>>>(b.labels, b.ub, b.compkey, b.cand_d, b.cand_j, b.qflag, b.qcnt, n,
                                         b.ctrl);
        if (!fold) k_qlist_scan<<<1, 1024, 0, st>>>(b.qcnt, nt, b.qoff, b.ctrl);
        k_qlist_write<<<nt, 256, 0, st>>>(b.qflag, b.qoff, n, b.qlist, b.ctrl, fold ? b.qcnt : nullptr, nt);
        HIP_TRY(hipGetLastError());
        ta.qlist = b.qlist;
    }
    // counting runs: the node heights (dead after the build) mark the node
    // records this round's searches load
    ta.touched = nullptr;
    const int64_t words = (n - 1) / 4;  // whole words only: the tail is cleared by bytes
    if (ctx->counting) {
        k_fill_u32<<<grid_for(words + 1), 256, 0, st>>>(reinterpret_cast<uint32_t*>(b.height), words, 0u);
        k_fill_u8<<<1, 64, 0, st>>>(b.height + 4 * words, n - 1 - 4 * words, 0u);
        ta.touched = b.height;
    }
    if (prof) HIP_TRY(hipEventRecord(E[8 + 2 * round], st));
    HIP_TRY(launch_traverse<DIM>(ta, height, variant, ctx->counting, st));
    if (prof) HIP_TRY(hipEventRecord(E[9 + 2 * round], st));
    if (ctx->counting) k_count_flags<<<std::min<unsigned>(grid_for(n - 1), 1024), 256, 0, st>>>(b.height, n - 1, b.ctrl);
    if (round == 1)
        k_resolve<1><<<grid_for(n), 256, 0, st>>>(b.cand_d, b.cand_j, b.cand_p, b.labels, b.orig, b.compkey,
                                                  b.compmax, b.succ, n, b.ctrl);
    else if (round > 1)
        k_resolve<4><<<grid_for((n + 3) / 4), 256, 0, st>>>(b.cand_d, b.cand_j, b.cand_p, b.labels, b.orig,
                                                            b.compkey, b.compmax, b.succ, n, b.ctrl);
    if (cap)
        k_test_capture<<<grid_for(n), 256, 0, st>>>(b.labels, b.orig, b.ub, b.cand_d, b.cand_j, b.compkey,
                                                    b.compmax, n, *cap);
    // root lists: segments in the Morton key buffers (free during the
    // rounds), counts behind k_merge_parent's partials in bpart
    const int mp_blocks = root_list_blocks(n);
    const bool first = round == 0;
    RootList rl;
    uint32_t* lists[2] = {reinterpret_cast<uint32_t*>(b.k0), reinterpret_cast<uint32_t*>(b.k1)};
    uint32_t* counts = b.bpart + 4 * kPartBlocks;
    rl.in = lists[round & 1];
    rl.cnt_in = counts + kPartBlocks * (round & 1);
    rl.out = lists[(round + 1) & 1];
    rl.cnt_out = counts + kPartBlocks * ((round + 1) & 1);
    rl.cap = root_list_cap(n);
    const unsigned merge_grid = first ? grid_for(n) : (unsigned)mp_blocks;
    k_merge_parent<<<mp_blocks, 256, 0, st>>>(b.labels, b.succ, b.par, b.compkey, b.compmax, b.ub, b.eud,
                                              reinterpret_cast<uint2*>(b.bpart), b.ctrl, n, first, rl,
                                              cloud_of != nullptr);
    HIP_TRY(hipGetLastError());
    k_merge_jump<<<merge_grid, 256, 0, st>>>(b.labels, b.par, n, 1024, b.ctrl, first, rl);
    k_relabel<<<nt, 256, 0, st>>>(b.labels, b.par, n, 4096, b.run_part, reinterpret_cast<const uint2*>(b.bpart),
                                  mp_blocks, b.ctrl, target);
    HIP_TRY(hipGetLastError());
    return EMST_OK;
}

// The host side of a finished round: consistency checks, counters, and the
// new component count.
int finish_round(emst_ctx* ctx, const Ctrl* h, int round, int64_t target, int64_t& ncomp, emst_stats& S) {
    if (h->error & kErrStack) return fail(ctx, EMST_EINTERNAL, "traversal stack overflow");
    if (h->error & kErrJump) return fail(ctx, EMST_EINTERNAL, "component merge did not converge");
    if (h->error) return fail(ctx, EMST_EINTERNAL, "a component found no outgoing edge");
    if (ctx->counting) {
        const int64_t it = (int64_t)h->internal_tests, lt = (int64_t)h->leaf_tests;
        S.child_tests_round[round] = it - S.child_tests;
        S.leaf_tests_round[round] = lt - S.leaf_tests;
        S.child_tests = it;
        S.leaf_tests = lt;
        S.dist_evals = (int64_t)h->dist_evals;
        int64_t before = 0;
        for (int r = 0; r < round; ++r) before += S.records_touched_round[r];
        S.records_touched_round[round] = (int64_t)h->touched - before;
    }
    const int64_t next = h->ncomp_next;
    if (next >= ncomp || next < target) return fail(ctx, EMST_EINTERNAL, "round made no progress");
    ncomp = next;
    return EMST_OK;
}

// Boruvka rounds until the component count reaches `target` (the number of
// non-empty clouds of a batch).  As for one cloud (job_rounds), round r + 1
// is queued before round r is read back, while the shrink of the last
// round predicts that round r leaves components beyond the target; a round
// queued past the end finds `done` raised and returns at once.
// A graph of two consecutive rounds (an even one and the next) from the
// third round on: those rounds launch the same kernels with the same
// arguments, so one graph serves every pair.  Instantiated graphs are kept
// per context (at most kGraphCache, least recently used replaced).
constexpr int kGraphCache = 4;
template <int DIM>
int round_pair_graph(emst_ctx* ctx, Bufs<DIM>& b, TraverseArgs<DIM>& ta, int64_t n, int64_t target, int height,
                     int variant, const uint32_t* cloud_of, hipGraphExec_t* out) {
    ++ctx->gclock;
    for (auto& g : ctx->gcache)
        if (g.ws == (const void*)b.ctrl && g.n == n && g.target == target && g.variant == variant &&
            g.height == height && g.cloud_of == (const void*)cloud_of && g.root == ta.root &&
            g.lds_depth == ta.lds_depth) {
            g.used = ctx->gclock;
            *out = g.exec;
            return EMST_OK;
        }
    if (!ctx->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_round<DIM>(ctx, b, ta, n, 2, height, variant, cloud_of, target, false, ctx->cap_stream);
    if (rc == EMST_OK)
        rc = enqueue_round<DIM>(ctx, b, ta, n, 3, height, variant, cloud_of, target, false, ctx->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (ec != hipSuccess) return fail(ctx, EMST_EHIP, hipGetErrorString(ec));
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return fail(ctx, EMST_EHIP, hipGetErrorString(ei));
    if ((int)ctx->gcache.size() >= kGraphCache) {
        auto old = std::min_element(ctx->gcache.begin(), ctx->gcache.end(),
                                    [](const emst_ctx::GraphEntry& x, const emst_ctx::GraphEntry& y) {
                                        return x.used < y.used;
                                    });
        (void)hipGraphExecDestroy(old->exec);
        ctx->gcache.erase(old);
    }
    ctx->gcache.push_back({(const void*)b.ctrl, n, target, variant, height, (const void*)cloud_of, ta.root,
                           ta.lds_depth, exec, ctx->gclock});
    *out = exec;
    return EMST_OK;
}

// Rounds 2, 3, ... as replays of the captured pair, the next replay queued
// before the last one is read back while more rounds are predicted.  A
// replay past the end returns at once (`done`).  Per-round statistics are
// kept only at pair boundaries; the round count comes from the device.
template <int DIM>
int graph_rounds(emst_ctx* ctx, Bufs<DIM>& b, TraverseArgs<DIM>& ta, int64_t n, int64_t target, int height,
                 int variant, const uint32_t* cloud_of, emst_stats& S, int64_t ncomp, hipStream_t st) {
    hipGraphExec_t exec = nullptr;
    if (int rc = round_pair_graph<DIM>(ctx, b, ta, n, target, height, variant, cloud_of, &exec)) return rc;
    Ctrl* mirror[2] = {ctx->h_ctrl, ctx->h_ctrl + 1};
    auto launch = [&](int k) -> int {
        HIP_TRY(hipGraphLaunch(exec, st));
        HIP_TRY(hipMemcpyAsync(mirror[k & 1], b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipEventRecord(ctx->sev[k & 1], st));
        return EMST_OK;
    };
    if (int rc = launch(0)) return rc;
    int queued = 0;
    int64_t prev = 0;
    for (int k = 0; 2 + 2 * k < 64; ++k) {
        // components after this pair, predicted from the last one's shrink
        const bool more = prev == 0 || (double)ncomp * (double)ncomp >= 2.0 * (double)prev * (double)target;
        if (queued == k && more) {
            if (int rc = launch(k + 1)) return rc;
            queued = k + 1;
        }
        HIP_TRY(hipEventSynchronize(ctx->sev[k & 1]));
        const Ctrl* h = mirror[k & 1];
        S.components[2 + 2 * k] = ncomp;
        prev = ncomp;
        if (int rc = finish_round(ctx, h, 2 + 2 * k, target, ncomp, S)) {
            (void)hipStreamSynchronize(st);
            return rc;
        }
        if (ncomp <= target) {
            HIP_TRY(hipStreamSynchronize(st));
            *ctx->h_ctrl = *h;
            S.rounds = (int32_t)h->rounds_run;
            S.traversal_launches = S.rounds;
            S.traversal_variant = variant;
            return EMST_OK;
        }
        if (queued == k) {
            if (int rc = launch(k + 1)) return rc;
            queued = k + 1;
        }
    }
    (void)hipStreamSynchronize(st);
    return fail(ctx, EMST_EINTERNAL, "too many rounds");
}

template <int DIM>
int run_rounds(emst_ctx* ctx, Bufs<DIM>& b, TraverseArgs<DIM>& ta, int64_t n, int64_t target, int height,
               int variant, const uint32_t* cloud_of, emst_stats& S, hipStream_t st) {
    const bool prof = ctx->profiling && ctx->ev_ok;
    // with graphs, rounds from the third on run as replays of a captured
    // pair, each followed by one read-back
    const bool graphs = ctx->graphs && !prof && !ctx->counting;
    Ctrl* mirror[2] = {ctx->h_ctrl, ctx->h_ctrl + 1};
    auto queue = [&](int r) -> int {
        if (int rc = enqueue_round<DIM>(ctx, b, ta, n, r, height, variant, cloud_of, target, prof, st)) return rc;
        HIP_TRY(hipMemcpyAsync(mirror[r & 1], b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipEventRecord(ctx->sev[r & 1], st));
        return EMST_OK;
    };
    if (n <= target) {  // every cloud is a single point: no round at all
        S.rounds = 0;
        S.traversal_launches = 0;
        S.traversal_variant = variant;
        return EMST_OK;
    }
    int64_t ncomp = n, prev = 0;
    int queued = -1;
    for (int round = 0;; ++round) {
        if (round >= 64) return fail(ctx, EMST_EINTERNAL, "too many rounds");
        if (graphs && round == 2) return graph_rounds<DIM>(ctx, b, ta, n, target, height, variant, cloud_of, S,
                                                           ncomp, st);
        if (queued < round) {
            if (int rc = queue(round)) return rc;
            queued = round;
        }
        // components entering round + 1, predicted from the last shrink
        const bool more = prev == 0 || (double)ncomp * (double)ncomp >= 2.0 * (double)prev * (double)target;
        if (more && round + 1 < 64 && !(graphs && round + 1 == 2)) {
            if (int rc = queue(round + 1)) return rc;
            queued = round + 1;
        }
        HIP_TRY(hipEventSynchronize(ctx->sev[round & 1]));
        const Ctrl* h = mirror[round & 1];
        S.components[round] = ncomp;
        S.queries_round[round] = uses_qlist(variant, round, n) ? (int64_t)h->qcount : n;
        prev = ncomp;
        if (int rc = finish_round(ctx, h, round, target, ncomp, S)) {
            (void)hipStreamSynchronize(st);
            return rc;
        }
        if (ncomp <= target) {
            // a round queued beyond the last returned at once; wait for it
            HIP_TRY(hipStreamSynchronize(st));
            *ctx->h_ctrl = *h;
            S.rounds = round + 1;
            S.traversal_launches = round + 1;
            S.traversal_variant = variant;
            return EMST_OK;
        }
    }
}

// Canonical edge order over the n component slots (the slots of the final
// roots are empty and sort last).  Writes sorted slot ids to *order.
//   full = false: by (D bits, u), runs of equal keys put in v order in place
//                 (see k_tie_fix; may raise long_ties);
//   full = true:  by (u, v), then stably by D bits;
// then, for a batch, stably by cloud.
template <int DIM>
int sort_edges(emst_ctx* ctx, Bufs<DIM>& b, int64_t n, const uint32_t* slot_cloud, int cloud_bits, bool full,
               const uint32_t** order, hipStream_t st, const uint64_t** keys_out = nullptr) {
    int in1 = 0;
    const int ib = 32 - __builtin_clz((unsigned)(n - 1));  // bits of the largest index
    uint32_t *p, *p_alt;
    uint64_t *kd, *kd_alt;
    // one cloud's fast path sorts the v of every edge as its value
    const bool v_values = !full && !slot_cloud && keys_out;
    if (keys_out) *keys_out = nullptr;
    if (!full) {
        k_edge_du_keys<<<grid_for(n), 256, 0, st>>>(b.eud, n, b.k0, b.v0, v_values);
        int sh[8], q = 0;
        for (int s = 0; s < ib; s += 8) sh[q++] = s;
        for (int s = 32; s < 64; s += 8) sh[q++] = s;
        HIP_TRY(radix_sort_pairs(st, b.k0, b.v0, b.k1, b.v1, b.hist, n, sh, q, &in1));
        p = in1 ? b.v1 : b.v0;
        kd = in1 ? b.k1 : b.k0;
        kd_alt = in1 ? b.k0 : b.k1;
        p_alt = in1 ? b.v0 : b.v1;
        k_tie_fix<<<grid_for(n), 256, 0, st>>>(kd, p, b.eud, n, b.ctrl, v_values);
        if (v_values) *keys_out = kd;
    } else {
        k_edge_keys<<<grid_for(n), 256, 0, st>>>(b.eud, n, b.k0, b.v0);
        int sh[8], q = 0;
        for (int s = 0; s < ib; s += 8) sh[q++] = s;
        for (int s = 0; s < ib; s += 8) sh[q++] = 32 + s;
        HIP_TRY(radix_sort_pairs(st, b.k0, b.v0, b.k1, b.v1, b.hist, n, sh, q, &in1));
        p = in1 ? b.v1 : b.v0;
        kd = in1 ? b.k1 : b.k0;
        kd_alt = in1 ? b.k0 : b.k1;
        p_alt = in1 ? b.v0 : b.v1;
        k_edge_dkeys<<<grid_for(n), 256, 0, st>>>(b.eud, p, n, kd);
        const int dsh[4] = {0, 8, 16, 24};
        HIP_TRY(radix_sort_pairs(st, kd, p, kd_alt, p_alt, b.hist, n, dsh, 4, &in1));
        if (in1) {
            std::swap(p, p_alt);
            std::swap(kd, kd_alt);
        }
    }
    if (slot_cloud && cloud_bits > 0) {
        k_perm_keys<<<grid_for(n), 256, 0, st>>>(slot_cloud, p, n, kd);
        int csh[4], cq = 0;
        for (int s = 0; s < cloud_bits; s += 8) csh[cq++] = s;
        HIP_TRY(radix_sort_pairs(st, kd, p, kd_alt, p_alt, b.hist, n, csh, cq, &in1));
        if (in1) std::swap(p, p_alt);
    }
    HIP_TRY(hipGetLastError());
    *order = p;
    return EMST_OK;
}

// Hierarchy (bottom-up, exchange only) and the boxes of every node inside
// a tile of kFitTile leaves.  The node records live in the cells' array,
// the list of nodes across tile borders in the exchange words (both free
// until the cells and the wave starts are made), its length in the sort's
// histogram (free until the next sort).
template <int DIM>
int build_hierarchy(emst_ctx* ctx, Bufs<DIM>& b, const uint64_t* codes, int64_t n, hipStream_t st) {
    NodeInfo* info = reinterpret_cast<NodeInfo*>(b.up);
    k_build<DIM, false><<<grid_for(n), 256, 0, st>>>(codes, b.orig, n, b.recs, b.leaf_parent, info, b.exch, b.ctrl);
    k_fill_u32<<<1, 64, 0, st>>>(b.hist, 1, 0u);
    const unsigned tiles = (unsigned)((n + kFitTile - 1) / kFitTile);
    k_fit_tiles<DIM><<<tiles, 256, 0, st>>>(b.spts, b.orig, b.leaf_parent, info, n, b.recs, b.rlo, b.rhi,
                                              b.node_parent, b.height, reinterpret_cast<uint2*>(b.exch), b.hist,
                                              b.ctrl);
    HIP_TRY(hipGetLastError());
    return EMST_OK;
}

// The control block after build_hierarchy names a usable root and height.
static int check_hierarchy(emst_ctx* ctx, const Ctrl* h, int64_t n) {
    if (h->root == kNone || h->root >= (uint32_t)(n - 1) || h->error || h->height > 128)
        return fail(ctx, EMST_EINTERNAL, "tree construction failed");
    return EMST_OK;
}

// The boxes of the nodes across tile borders, one launch per height below
// the root H (after build_hierarchy, whose list they come from).
template <int DIM>
int fit_levels(emst_ctx* ctx, Bufs<DIM>& b, const uint64_t* codes, int64_t n, uint32_t H, hipStream_t st) {
    (void)codes;
    // at most 129 listed nodes per tile border (the grid only; the kernel
    // reads the list's length)
    const int64_t cap = ((n + kFitTile - 1) / kFitTile) * 129;
    const unsigned grid = std::min<unsigned>(grid_for(cap), 1024);
    for (uint32_t h = 1; h < H; ++h)
        k_fit_span<DIM><<<grid, 256, 0, st>>>(reinterpret_cast<const uint2*>(b.exch), b.hist, n - 1, h,
                                               b.node_parent, b.recs);
    HIP_TRY(hipGetLastError());
    return EMST_OK;
}

// Hierarchy and boxes in one go (reads the control block back for the root
// and height).
template <int DIM>
int build_tree(emst_ctx* ctx, Bufs<DIM>& b, const uint64_t* codes, int64_t n, hipStream_t st) {
    if (int rc = build_hierarchy<DIM>(ctx, b, codes, n, st)) return rc;
    if (int rc = read_ctrl(ctx, b.ctrl, st)) return rc;
    if (int rc = check_hierarchy(ctx, ctx->h_ctrl, n)) return rc;
    return fit_levels<DIM>(ctx, b, codes, n, ctx->h_ctrl->height, st);
}

void finish_stats(emst_ctx* ctx, emst_stats& S) {
    if (ctx->profiling && ctx->ev_ok) {
        hipEvent_t* E = ctx->ev;
        S.tree_ms = elapsed(E[0], E[1]);
        S.rounds_ms = elapsed(E[1], E[2]);
        S.finalize_ms = elapsed(E[2], E[3]);
        S.total_ms = elapsed(E[0], E[3]);
        for (int r = 0; r < S.rounds; ++r) {
            S.traversal_ms_round[r] = elapsed(E[8 + 2 * r], E[9 + 2 * r]);
            S.traversal_ms += S.traversal_ms_round[r];
        }
    }
    ctx->stats = S;
}

// One cloud's build as a resumable sequence of phases.  Each phase
// enqueues its work and a copy of the control block into the job's pinned
// host mirror; after the stream has drained, advance() reads the mirror and
// picks the next phase.  emst_build, emst_build_mreach and the one-round
// test hook run one job to the end.
//
// k_pts = 0: the EMST.  k_pts >= 1: the MST under mutual reachability with
// core distances of k_pts (k_pts = 1 gives zero cores, hence the EMST);
// core_out (nullable) receives the squared core distances in input order;
// core_only stops after them.
enum JobPhase { kPhTree, kPhRank, kPhFit, kPhRound, kPhFinal, kPhDone };

struct Job {
    int dim = 3;
    int64_t n = 0;
    const float* pts = nullptr;
    char* ws = nullptr;
    int32_t* edges = nullptr;
    float* weights = nullptr;
    float* d2 = nullptr;
    int k_pts = 0;
    float* core_out = nullptr;
    bool core_only = false;
    Ctrl* h = nullptr;     // pinned host mirror of this job's control block
    bool prof = false;     // record the context's phase and traversal events
    int phase = kPhTree;
    int round = 0;
    int64_t ncomp = 0;
    bool ranks = false;
    int full = 0;
    int variant = 10;
    int lds_depth = 8;
    uint32_t root = 0;     // of the finished hierarchy
    int height = 0;
    int codes_in1 = 0;     // which key buffer holds the sorted codes
    MortonParams mp;
    emst_stats S;
};

static Job make_job(emst_ctx* ctx, const float* pts, int64_t n, int dim, char* ws, int32_t* edges, float* weights,
                    float* d2, int k_pts, float* core_out, bool core_only, Ctrl* h, bool prof) {
    Job j;
    j.dim = dim;
    j.n = n;
    j.pts = pts;
    j.ws = ws;
    j.edges = edges;
    j.weights = weights;
    j.d2 = d2;
    j.k_pts = k_pts;
    j.core_out = core_out;
    j.core_only = core_only;
    j.h = h;
    j.prof = prof;
    j.ncomp = n;
    pick_shape(ctx, 0, dim, n, &j.variant, &j.lds_depth);
    memset(&j.S, 0, sizeof(j.S));
    j.S.n = n;
    j.S.dim = dim;
    return j;
}

template <int DIM>
static TraverseArgs<DIM> job_args(const Job& j, const Bufs<DIM>& b) {
    TraverseArgs<DIM> ta = traverse_args<DIM>(b, j.n, j.root);
    ta.lds_depth = j.lds_depth;
    if (j.k_pts >= 2) {
        ta.core_s = b.core_s;
        ta.core_o = b.core_o;
    }
    return ta;
}

// Enqueue the current phase (ending with the control block copy).
template <int DIM>
int job_enqueue(emst_ctx* ctx, Job& j, hipStream_t st) {
    const int64_t n = j.n;
    const Layout L = make_layout(n, DIM);
    Bufs<DIM> b = carve<DIM>(j.ws, L);
    hipEvent_t* E = ctx->ev;  // E[0..3] phases, E[8 + 2r], E[9 + 2r] traversal of round r
    switch (j.phase) {
    case kPhTree: {  // validation + scene box, Morton codes, sort, hierarchy
        if (j.prof) HIP_TRY(hipEventRecord(E[0], st));
        k_init_ctrl<<<1, 64, 0, st>>>(b.ctrl);
        HIP_TRY(launch_bbox<DIM>(j.pts, n, b.bpart, b.ctrl, st));
        // The codes take the box from the control block.  A cloud that fails
        // validation (read back after this phase) still yields codes of some
        // box: any codes make a valid hierarchy, and the job stops there.
        k_morton<DIM><<<std::min<unsigned>(grid_for(n), 1024), 256, 0, st>>>(j.pts, n, j.mp, b.ctrl, b.k0, b.v0);
        const int shifts[8] = {0, 8, 16, 24, 32, 40, 48, 56};
        HIP_TRY(radix_sort_pairs(st, b.k0, b.v0, b.k1, b.v1, b.hist, n, shifts, 8, &j.codes_in1));
        const uint64_t* codes = j.codes_in1 ? b.k1 : b.k0;
        k_count_dups<<<grid_for(n), 256, 0, st>>>(codes, n, b.ctrl);
        k_gather<DIM><<<grid_for(n), 256, 0, st>>>(j.pts, j.codes_in1 ? b.v1 : b.v0, n, b.spts, b.orig,
                                                   b.labels, b.exch);
        if (int rc = build_hierarchy<DIM>(ctx, b, codes, n, st)) return rc;
        break;
    }
    case kPhRank: {
        // many equal codes: rebuild on rank-space codes (the node records
        // are rebuilt afterwards, so they hold the codes meanwhile)
        uint64_t* acc = reinterpret_cast<uint64_t*>(b.recs);
        const int bits = DIM == 3 ? 21 : 32;
        const int ash[4] = {0, 8, 16, 24};
        int in1 = 0;
        for (int axis = 0; axis < DIM; ++axis) {
            k_axis_keys<DIM><<<grid_for(n), 256, 0, st>>>(j.pts, n, axis, b.k0, b.v0);
            HIP_TRY(radix_sort_pairs(st, b.k0, b.v0, b.k1, b.v1, b.hist, n, ash, 4, &in1));
            k_axis_rank<DIM><<<grid_for(n), 256, 0, st>>>(in1 ? b.v1 : b.v0, n, axis, bits, acc);
        }
        k_codes_from<<<grid_for(n), 256, 0, st>>>(acc, n, b.k0, b.v0);
        int csh[8], cq = 0;
        for (int s = 0; s < DIM * bits; s += 8) csh[cq++] = s;
        HIP_TRY(radix_sort_pairs(st, b.k0, b.v0, b.k1, b.v1, b.hist, n, csh, cq, &j.codes_in1));
        const uint64_t* codes = j.codes_in1 ? b.k1 : b.k0;
        k_gather<DIM><<<grid_for(n), 256, 0, st>>>(j.pts, j.codes_in1 ? b.v1 : b.v0, n, b.spts, b.orig,
                                                   b.labels, b.exch);
        if (int rc = build_hierarchy<DIM>(ctx, b, codes, n, st)) return rc;
        break;
    }
    case kPhFit: {  // boxes, Morton cells, wave starts, core distances; then round 0
        const uint64_t* codes = j.codes_in1 ? b.k1 : b.k0;
        if (int rc = fit_levels<DIM>(ctx, b, codes, n, (uint32_t)j.height, st)) return rc;
        k_cells<DIM><<<grid_for(n - 1), 256, 0, st>>>(codes, b.node_parent, n - 1, j.mp, j.ranks, b.up);
        k_wave_lca<<<grid_for((n + 63) / 64), 256, 0, st>>>(b.rlo, b.rhi, b.leaf_parent, b.node_parent, n,
                                                            reinterpret_cast<uint32_t*>(b.exch));
        HIP_TRY(hipGetLastError());
        TraverseArgs<DIM> ta = job_args<DIM>(j, b);
        if (j.k_pts >= 2) {
            HIP_TRY(launch_core<DIM>(ta, j.height, j.k_pts, b.core_s, b.core_o, j.core_out, st));
        } else if (j.k_pts == 1 && j.core_out) {
            k_fill_u32<<<grid_for(n), 256, 0, st>>>(reinterpret_cast<uint32_t*>(j.core_out), n, 0u);
            HIP_TRY(hipGetLastError());
        }
        if (j.prof) HIP_TRY(hipEventRecord(E[1], st));
        if (j.core_only) {
            if (j.prof) {
                HIP_TRY(hipEventRecord(E[2], st));
                HIP_TRY(hipEventRecord(E[3], st));
            }
            break;
        }
        j.phase = kPhRound;  // round 0 goes out with this phase
        j.S.components[0] = n;
        if (int rc = enqueue_round<DIM>(ctx, b, ta, n, 0, j.height, j.variant, nullptr, 1, j.prof, st)) return rc;
        break;
    }
    case kPhRound: {
        TraverseArgs<DIM> ta = job_args<DIM>(j, b);
        j.S.components[j.round] = j.ncomp;
        if (int rc = enqueue_round<DIM>(ctx, b, ta, n, j.round, j.height, j.variant, nullptr, 1, j.prof, st))
            return rc;
        break;
    }
    case kPhFinal: {  // canonical order (the full sort only after a long run of ties)
        const uint32_t* order = nullptr;
        const uint64_t* keys = nullptr;
        if (int rc = sort_edges<DIM>(ctx, b, n, nullptr, 0, j.full != 0, &order, st, &keys)) return rc;
        if (keys)  // the sorted keys and values are the edges
            k_edge_write_kv<<<grid_for(n - 1), 256, 0, st>>>(keys, order, n - 1, j.edges, j.weights, j.d2);
        else
            k_edge_write<<<grid_for(n - 1), 256, 0, st>>>(b.eud, order, n - 1, j.edges, j.weights, j.d2);
        HIP_TRY(hipGetLastError());
        if (j.prof) HIP_TRY(hipEventRecord(E[3], st));
        break;
    }
    default:
        return fail(ctx, EMST_EINTERNAL, "job already finished");
    }
    HIP_TRY(hipMemcpyAsync(j.h, b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    return EMST_OK;
}

// After the stream has drained: read the mirror, choose the next phase.
template <int DIM>
int job_advance(emst_ctx* ctx, Job& j) {
    const Ctrl* h = j.h;
    const int64_t n = j.n;
    switch (j.phase) {
    case kPhTree:
    case kPhRank:
        if (j.phase == kPhTree) {
            if (h->nonfinite) return fail(ctx, EMST_ENONFINITE, "non-finite coordinate");
            float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
            for (int k = 0; k < DIM; ++k) {
                lo[k] = ord_dec(h->bb_min[k]);
                hi[k] = ord_dec(h->bb_max[k]);
            }
            if (!extent_ok(lo, hi, DIM))
                return fail(ctx, EMST_ERANGE, "squared extent of the cloud overflows float32");
            j.mp = morton_params_of(*h, DIM);  // the parameters k_morton derived on the device
        }
        if (int rc = check_hierarchy(ctx, h, n)) return rc;
        if (j.phase == kPhTree && (int64_t)h->dup_codes * 64 > n) {
            j.ranks = true;
            j.phase = kPhRank;
        } else {
            j.S.rank_codes = j.ranks ? 1 : 0;
            j.S.tree_height = (int32_t)h->height;
            j.root = h->root;
            j.height = (int)h->height;
            j.phase = kPhFit;
        }
        return EMST_OK;
    case kPhFit:  // core distances only
        if (h->error) return fail(ctx, EMST_EINTERNAL, "core distance search failed");
        j.phase = kPhDone;
        return EMST_OK;
    case kPhRound: {
        if (j.round >= 64) return fail(ctx, EMST_EINTERNAL, "too many rounds");
        j.S.queries_round[j.round] = uses_qlist(j.variant, j.round, n) ? (int64_t)h->qcount : n;
        if (int rc = finish_round(ctx, h, j.round, 1, j.ncomp, j.S)) return rc;
        ++j.round;
        if (j.ncomp == 1) {
            j.S.rounds = j.round;
            j.S.traversal_launches = j.round;
            j.S.traversal_variant = j.variant;
            j.S.traversal_lds_depth = j.variant == 13 ? j.lds_depth : 0;
            if (h->edge_count != (uint32_t)(n - 1)) return fail(ctx, EMST_EINTERNAL, "wrong edge count");
            j.phase = kPhFinal;
        }
        return EMST_OK;
    }
    case kPhFinal:
        if (h->long_ties && !j.full) j.full = 1;
        else j.phase = kPhDone;
        return EMST_OK;
    default:
        return fail(ctx, EMST_EINTERNAL, "job already finished");
    }
}

// The rounds of one job, with the next round queued before the host reads
// the last one back, so that the device does not idle while the host
// checks a round: round r's control block goes to mirror r % 2 and an event
// marks its arrival.  A round queued past the end finds `done` raised and
// returns at once, but still costs its launches, so round r + 1 is queued
// early only while the shrink of the last round predicts that round r
// leaves at least two components.  Round 0 is already queued (by the fit
// phase) with its copy going to mirror 0.
template <int DIM>
int job_rounds(emst_ctx* ctx, Job& j, hipStream_t st) {
    Ctrl* mirror[2] = {ctx->h_ctrl, ctx->h_ctrl + 1};
    HIP_TRY(hipEventRecord(ctx->sev[0], st));
    const Layout L = make_layout(j.n, DIM);
    Bufs<DIM> b = carve<DIM>(j.ws, L);
    TraverseArgs<DIM> ta = job_args<DIM>(j, b);
    auto queue = [&](int r) -> int {
        if (int rc = enqueue_round<DIM>(ctx, b, ta, j.n, r, j.height, j.variant, nullptr, 1, j.prof, st)) return rc;
        HIP_TRY(hipMemcpyAsync(mirror[r & 1], b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipEventRecord(ctx->sev[r & 1], st));
        return EMST_OK;
    };
    int queued = 0;      // last round on the stream
    int64_t prev = 0;    // components entering the previous round (0: none yet)
    for (int r = 0;; ++r) {
        const int64_t now = j.ncomp;  // components entering round r
        const bool more = prev == 0 || (double)now * (double)now >= 2.0 * (double)prev;
        if (queued == r && r + 1 < 64 && more) {
            if (int rc = queue(r + 1)) return rc;
            queued = r + 1;
        }
        HIP_TRY(hipEventSynchronize(ctx->sev[r & 1]));
        j.h = mirror[r & 1];
        j.round = r;
        j.S.components[r] = now;
        const int rc = job_advance<DIM>(ctx, j);
        j.h = mirror[0];
        if (rc) return rc;
        if (j.phase != kPhRound) return EMST_OK;
        prev = now;
        if (queued == r) {
            if (r + 1 >= 64) return fail(ctx, EMST_EINTERNAL, "too many rounds");
            if (int rc2 = queue(r + 1)) return rc2;
            queued = r + 1;
        }
    }
}

// E[2] (end of the rounds) sits between the last round and the final sort.
template <int DIM>
int job_run(emst_ctx* ctx, Job& j, hipStream_t st) {
    while (j.phase != kPhDone) {
        if (j.prof && j.phase == kPhFinal && !j.full) HIP_TRY(hipEventRecord(ctx->ev[2], st));
        const bool to_rounds = j.phase == kPhFit && !j.core_only;
        int rc = job_enqueue<DIM>(ctx, j, st);
        if (rc == EMST_OK && to_rounds) {
            rc = job_rounds<DIM>(ctx, j, st);
            if (rc) {
                (void)hipStreamSynchronize(st);
                return rc;
            }
            continue;
        }
        const hipError_t w = hipStreamSynchronize(st);
        if (rc) return rc;
        if (w != hipSuccess) return fail(ctx, EMST_EHIP, hipGetErrorString(w));
        if (int rc2 = job_advance<DIM>(ctx, j)) return rc2;
    }
    return EMST_OK;
}

template <int DIM>
int build_impl(emst_ctx* ctx, const float* pts, int64_t n, int32_t* edges, float* weights, float* d2, char* ws,
               hipStream_t st, int k_pts = 0, float* core_out = nullptr, bool core_only = false) {
    Job j = make_job(ctx, pts, n, DIM, ws, edges, weights, d2, k_pts, core_out, core_only, ctx->h_ctrl,
                     ctx->profiling && ctx->ev_ok);
    if (int rc = job_run<DIM>(ctx, j, st)) return rc;
    finish_stats(ctx, j.S);
    return EMST_OK;
}


int batched_impl(emst_ctx* ctx, const float* pts, const int64_t* h_offsets, const int32_t* h_dims, int32_t B,
                 int32_t* edges, float* weights, float* d2, int64_t* h_edge_offsets, char* ws, hipStream_t st) {
    const int64_t n = h_offsets[B];
    const BatchLayout BL = make_batch_layout(n, B);
    Bufs<3> b = carve<3>(ws, BL.base);
    float* pts3 = reinterpret_cast<float*>(ws + BL.pts3);
    uint32_t* cloud_of = reinterpret_cast<uint32_t*>(ws + BL.cloud_of);
    uint32_t* cloud_sorted = reinterpret_cast<uint32_t*>(ws + BL.cloud_sorted);
    CloudIn* d_cin = reinterpret_cast<CloudIn*>(ws + BL.cin);
    CloudBox* d_cbox = reinterpret_cast<CloudBox*>(ws + BL.cbox);
    CloudMorton* d_cm = reinterpret_cast<CloudMorton*>(ws + BL.cm);
    uint32_t* d_croot = reinterpret_cast<uint32_t*>(ws + BL.croot);
    emst_stats S;
    memset(&S, 0, sizeof(S));
    S.n = n;
    S.dim = 3;
    const bool prof = ctx->profiling && ctx->ev_ok;
    hipEvent_t* E = ctx->ev;

    // ---- per-cloud table (host) -> device
    const size_t tbl = std::max(sizeof(CloudIn), std::max(sizeof(CloudBox), sizeof(CloudMorton))) * (size_t)B;
    char* h = reinterpret_cast<char*>(stage(ctx, tbl));
    if (!h) return fail(ctx, EMST_EHIP, "hipHostMalloc failed");
    CloudIn* cin = reinterpret_cast<CloudIn*>(h);
    int64_t foff = 0, eoff = 0, nonempty = 0;
    for (int32_t c = 0; c < B; ++c) {
        cin[c].off = h_offsets[c];
        cin[c].n = h_offsets[c + 1] - h_offsets[c];
        cin[c].foff = foff;
        cin[c].eoff = eoff;
        cin[c].dim = h_dims[c];
        cin[c].pad = 0;
        foff += cin[c].n * h_dims[c];
        if (h_edge_offsets) h_edge_offsets[c] = eoff;
        eoff += cin[c].n > 1 ? cin[c].n - 1 : 0;
        nonempty += cin[c].n > 0;
    }
    if (h_edge_offsets) h_edge_offsets[B] = eoff;
    if (prof) HIP_TRY(hipEventRecord(E[0], st));
    HIP_TRY(hipMemcpyAsync(d_cin, cin, sizeof(CloudIn) * B, hipMemcpyHostToDevice, st));
    // ---- unpack + per-cloud boxes, validation
    k_init_ctrl<<<1, 64, 0, st>>>(b.ctrl);
    k_batch_box_init<<<grid_for(B), 256, 0, st>>>(d_cin, B, d_cbox);
    k_batch_unpack<<<unpack_grid(n), 256, 0, st>>>(pts, d_cin, B, n, pts3, cloud_of, d_cbox);
    HIP_TRY(hipGetLastError());
    CloudBox* cbox = reinterpret_cast<CloudBox*>(h);  // reuses the staging area
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipMemcpyAsync(cbox, d_cbox, sizeof(CloudBox) * B, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int cloud_bits = B > 1 ? 64 - __builtin_clzll((unsigned long long)(B - 1)) : 0;
    const int avail = 64 - cloud_bits;
    std::vector<CloudMorton> cm(B);
    for (int32_t c = 0; c < B; ++c) {
        if (cbox[c].bad) {
            ctx->err = "non-finite coordinate in cloud " + std::to_string(c);
            return EMST_ENONFINITE;
        }
        float lo[3], hi[3];
        for (int k = 0; k < 3; ++k) { lo[k] = ord_dec(cbox[c].mn[k]); hi[k] = ord_dec(cbox[c].mx[k]); }
        if (!extent_ok(lo, hi, 3)) {
            ctx->err = "squared extent of cloud " + std::to_string(c) + " overflows float32";
            return EMST_ERANGE;
        }
        const int dim = h_dims[c];
        const int bits = std::min(dim == 3 ? 21 : 32, avail / dim);
        const MortonParams mp = morton_params(lo, hi, dim, bits);
        for (int k = 0; k < 3; ++k) { cm[c].lo[k] = mp.lo[k]; cm[c].scale[k] = mp.scale[k]; }
        cm[c].qmax = mp.qmax;
        cm[c].dim = dim;
        cm[c].bits = bits;
    }
    memcpy(h, cm.data(), sizeof(CloudMorton) * B);
    HIP_TRY(hipMemcpyAsync(d_cm, h, sizeof(CloudMorton) * B, hipMemcpyHostToDevice, st));
    // ---- codes (cloud id on top) + sort
    {
        const int nb = (int)std::min<unsigned>(grid_for(n), kPartBlocks);
        uint64_t* part = reinterpret_cast<uint64_t*>(b.bpart);
        k_batch_morton<<<nb, 256, 0, st>>>(pts3, cloud_of, d_cm, n, avail, b.k0, b.v0, part);
        k_or_and_final<<<1, 256, 0, st>>>(part, nb, b.ctrl);
    }
    HIP_TRY(hipGetLastError());
    if (int rc = read_ctrl(ctx, b.ctrl, st)) return rc;
    int shifts[8], ns = 0;
    {
        const uint64_t vary = ctx->h_ctrl->key_or ^ ctx->h_ctrl->key_and;
        for (int s = 0; s < 64; s += 8)
            if ((vary >> s) & 0xFFull) shifts[ns++] = s;
    }
    int in1 = 0;
    HIP_TRY(radix_sort_pairs(st, b.k0, b.v0, b.k1, b.v1, b.hist, n, shifts, ns, &in1));
    const uint64_t* codes = in1 ? b.k1 : b.k0;
    const uint32_t* perm = in1 ? b.v1 : b.v0;
    // ---- one tree over all clouds
    k_gather<3><<<grid_for(n), 256, 0, st>>>(pts3, perm, n, b.spts, b.orig, b.labels, b.exch);
    // a batch of single points runs no round, so every edge slot starts empty
    k_fill_u32<<<grid_for(4 * n), 256, 0, st>>>(reinterpret_cast<uint32_t*>(b.eud), 4 * n, kNone);
    k_batch_sorted_cloud<<<grid_for(n), 256, 0, st>>>(cloud_of, perm, n, cloud_sorted);
    if (int rc = build_tree<3>(ctx, b, codes, n, st)) return rc;
    k_fill_u32<<<grid_for(B), 256, 0, st>>>(d_croot, B, kNone);
    k_cloud_roots<<<grid_for(n - 1), 256, 0, st>>>(b.rlo, b.rhi, cloud_sorted, d_cin, n - 1, d_croot);
    HIP_TRY(hipGetLastError());
    S.tree_height = (int32_t)ctx->h_ctrl->height;
    if (prof) HIP_TRY(hipEventRecord(E[1], st));

    // ---- rounds, every query inside its own cloud's subtree (top-down)
    TraverseArgs<3> ta = traverse_args<3>(b, n, ctx->h_ctrl->root);
    ta.cloud_of = cloud_sorted;
    ta.cloud_root = d_croot;
    // variants 1-4 start every lane at one root and 6, 9-12 need the Morton
    // cells of one cloud: a batch runs them as 7 (and 13 with the start of 7)
    int t = 13, depth = 8;
    pick_shape(ctx, 1, 3, n, &t, &depth);
    const int variant = (t == 0 || t == 5 || t == 8 || t == 13) ? t : 7;
    ta.lds_depth = depth;
    S.traversal_lds_depth = variant == 13 ? depth : 0;
    if (int rc = run_rounds<3>(ctx, b, ta, n, nonempty, S.tree_height, variant, cloud_sorted, S, st)) return rc;
    if ((int64_t)ctx->h_ctrl->edge_count != eoff) return fail(ctx, EMST_EINTERNAL, "wrong edge count");
    if (prof) HIP_TRY(hipEventRecord(E[2], st));

    // ---- per-cloud canonical order (the full sort only after a long run of ties)
    const uint32_t* order = nullptr;
    for (int full = 0; full < 2; ++full) {
        if (int rc = sort_edges<3>(ctx, b, n, cloud_sorted, cloud_bits, full != 0, &order, st)) return rc;
        k_batch_edge_write<<<grid_for(n), 256, 0, st>>>(b.eud, order, cloud_sorted, d_cin, n, edges, weights, d2);
        HIP_TRY(hipGetLastError());
        if (prof) HIP_TRY(hipEventRecord(E[3], st));
        if (int rc = read_ctrl(ctx, b.ctrl, st)) return rc;
        if (!ctx->h_ctrl->long_ties) break;
    }
    finish_stats(ctx, S);
    return EMST_OK;
}

}  // namespace

extern "C" int emst_build(emst_ctx* ctx, const float* d_points, int64_t n, int dim, int32_t* d_edges,
                          float* d_weights, float* d_d2, void* d_workspace, size_t ws_bytes, void* stream) {
    if (!ctx) return EMST_EINVAL;
    ctx->err.clear();
    if (n < 0 || n > 0x7FFFFFFFll) return fail(ctx, EMST_EINVAL, "n out of range");
    if (dim != 2 && dim != 3) return fail(ctx, EMST_EINVAL, "dim must be 2 or 3");
    if (n < 2) {
        memset(&ctx->stats, 0, sizeof(ctx->stats));
        ctx->stats.n = n;
        ctx->stats.dim = dim;
        return EMST_OK;
    }
    if (!d_points || !d_edges || !d_weights || !d_workspace) return fail(ctx, EMST_EINVAL, "null pointer");
    if (((uintptr_t)d_workspace & 255u) != 0) return fail(ctx, EMST_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < emst_workspace_bytes(n, dim)) return fail(ctx, EMST_ENOMEM, "workspace too small");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, EMST_EHIP, "hipSetDevice failed");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (dim == 3) return build_impl<3>(ctx, d_points, n, d_edges, d_weights, d_d2, (char*)d_workspace, st);
    return build_impl<2>(ctx, d_points, n, d_edges, d_weights, d_d2, (char*)d_workspace, st);
}


extern "C" int emst_build_noalloc(emst_ctx* ctx, const float* d_points, int64_t n, int dim, int32_t* d_edges,
                                  float* d_weights, float* d_d2, void* stream) {
    if (!ctx) return EMST_EINVAL;
    ctx->err.clear();
    if (n < 0 || n > 0x7FFFFFFFll) return fail(ctx, EMST_EINVAL, "n out of range");
    if (dim != 2 && dim != 3) return fail(ctx, EMST_EINVAL, "dim must be 2 or 3");
    const size_t need = emst_workspace_bytes(n, dim);
    if (need > (size_t)EMST_NOALLOC_WORKSPACE_BYTES) {
        ctx->err = "emst_build_noalloc: " + std::to_string(n) + " points need " + std::to_string(need) +
                   " workspace bytes, more than the " + std::to_string((size_t)EMST_NOALLOC_WORKSPACE_BYTES) +
                   " of the static workspace";
        return EMST_ENOMEM;
    }
    if (n >= 2 && !ctx->scratch) {
        ctx->err = "emst_build_noalloc: static workspace unavailable (" + ctx->scratch_err + ")";
        return EMST_EHIP;
    }
    const int rc = emst_build(ctx, d_points, n, dim, d_edges, d_weights, d_d2, ctx->scratch,
                              (size_t)EMST_NOALLOC_WORKSPACE_BYTES, stream);
    return rc;
}

static int check_single(emst_ctx* ctx, const float* d_points, int64_t n, int dim, void* d_workspace,
                        size_t ws_bytes) {
    if (!d_points || !d_workspace) return fail(ctx, EMST_EINVAL, "null pointer");
    if (((uintptr_t)d_workspace & 255u) != 0) return fail(ctx, EMST_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < emst_workspace_bytes(n, dim)) return fail(ctx, EMST_ENOMEM, "workspace too small");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, EMST_EHIP, "hipSetDevice failed");
    return EMST_OK;
}

extern "C" int emst_core_distances(emst_ctx* ctx, const float* d_points, int64_t n, int dim, int32_t k_pts,
                                   float* d_core2, void* d_workspace, size_t ws_bytes, void* stream) {
    if (!ctx) return EMST_EINVAL;
    ctx->err.clear();
    if (n < 0 || n > 0x7FFFFFFFll) return fail(ctx, EMST_EINVAL, "n out of range");
    if (dim != 2 && dim != 3) return fail(ctx, EMST_EINVAL, "dim must be 2 or 3");
    if (k_pts < 1 || k_pts > 64 || k_pts > n) return fail(ctx, EMST_EINVAL, "k_pts must be in [1, min(n, 64)]");
    if (!d_core2) return fail(ctx, EMST_EINVAL, "null pointer");
    memset(&ctx->stats, 0, sizeof(ctx->stats));
    ctx->stats.n = n;
    ctx->stats.dim = dim;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (n == 1 || k_pts == 1) {  // the point itself: 0
        if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, EMST_EHIP, "hipSetDevice failed");
        k_fill_u32<<<grid_for(n), 256, 0, st>>>(reinterpret_cast<uint32_t*>(d_core2), n, 0u);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(st));
        return EMST_OK;
    }
    if (int rc = check_single(ctx, d_points, n, dim, d_workspace, ws_bytes)) return rc;
    if (dim == 3)
        return build_impl<3>(ctx, d_points, n, nullptr, nullptr, nullptr, (char*)d_workspace, st, k_pts, d_core2, true);
    return build_impl<2>(ctx, d_points, n, nullptr, nullptr, nullptr, (char*)d_workspace, st, k_pts, d_core2, true);
}

extern "C" int emst_build_mreach(emst_ctx* ctx, const float* d_points, int64_t n, int dim, int32_t k_pts,
                                 int32_t* d_edges, float* d_weights, float* d_d2, float* d_core2, void* d_workspace,
                                 size_t ws_bytes, void* stream) {
    if (!ctx) return EMST_EINVAL;
    ctx->err.clear();
    if (n < 0 || n > 0x7FFFFFFFll) return fail(ctx, EMST_EINVAL, "n out of range");
    if (dim != 2 && dim != 3) return fail(ctx, EMST_EINVAL, "dim must be 2 or 3");
    if (k_pts < 1 || k_pts > 64 || (n > 0 && k_pts > n)) return fail(ctx, EMST_EINVAL, "k_pts must be in [1, min(n, 64)]");
    if (n < 2) {
        memset(&ctx->stats, 0, sizeof(ctx->stats));
        ctx->stats.n = n;
        ctx->stats.dim = dim;
        if (n == 1 && d_core2) {
            if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, EMST_EHIP, "hipSetDevice failed");
            hipStream_t st = reinterpret_cast<hipStream_t>(stream);
            k_fill_u32<<<1, 64, 0, st>>>(reinterpret_cast<uint32_t*>(d_core2), 1, 0u);
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipStreamSynchronize(st));
        }
        return EMST_OK;
    }
    if (!d_edges || !d_weights) return fail(ctx, EMST_EINVAL, "null pointer");
    if (int rc = check_single(ctx, d_points, n, dim, d_workspace, ws_bytes)) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (dim == 3)
        return build_impl<3>(ctx, d_points, n, d_edges, d_weights, d_d2, (char*)d_workspace, st, k_pts, d_core2);
    return build_impl<2>(ctx, d_points, n, d_edges, d_weights, d_d2, (char*)d_workspace, st, k_pts, d_core2);
}

// ---------------------------------------------------------------------------
// Round-granular continuous batching.  A solver holds up to max_slots
// requests inside a caller-provided device budget.  The requests admitted
// between two steps start together as one cohort: a batch as
// emst_build_batched builds it (one tree in which every request is its own
// subtree, one round loop), run as a resumable sequence of phases -- boxes
// and Morton codes, tree, boxes and the first round, one Boruvka round per
// phase, edge order.  Each cohort has its own stream (default priority); a
// step starts a cohort, then moves every cohort whose queued phase has
// completed on to its next one, and returns once at least one has moved.
// As in emst_build, the round after the one in flight is queued before the
// host has read the first while the last shrink predicts that more rounds
// are needed (a round queued past the end returns at once), so a cohort's
// rounds do not wait for the host.  Cohorts progress at their own pace, the
// kernels of all requests of a cohort are launched once per phase, and at
// most kSolverCohorts run at once, so that requests arriving meanwhile
// gather into the next cohort.

constexpr int kSolverCohorts = 8;  // live cohorts at most (4 and 16 measured no better on a serving trace)

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// The device arrays of a batch, carved from its workspace.
struct BatchBufs {
    Bufs<3> b;
    float* pts3;
    uint32_t* cloud_of;
    uint32_t* cloud_sorted;
    CloudIn* cin;
    CloudBox* cbox;
    CloudMorton* cm;
    uint32_t* croot;
};

static BatchBufs batch_bufs(char* ws, int64_t n, int32_t B) {
    const BatchLayout BL = make_batch_layout(n, B);
    BatchBufs x;
    x.b = carve<3>(ws, BL.base);
    x.pts3 = reinterpret_cast<float*>(ws + BL.pts3);
    x.cloud_of = reinterpret_cast<uint32_t*>(ws + BL.cloud_of);
    x.cloud_sorted = reinterpret_cast<uint32_t*>(ws + BL.cloud_sorted);
    x.cin = reinterpret_cast<CloudIn*>(ws + BL.cin);
    x.cbox = reinterpret_cast<CloudBox*>(ws + BL.cbox);
    x.cm = reinterpret_cast<CloudMorton*>(ws + BL.cm);
    x.croot = reinterpret_cast<uint32_t*>(ws + BL.croot);
    return x;
}

enum BPhase { kBCodes, kBTree, kBFit, kBRound, kBFinal, kBDone };

// One batch as phases.  Every queued phase ends with a copy of the control
// block into one of two pinned mirrors (after the first phase also of the
// cloud boxes); bjob_advance reads it once the phase has completed.
struct BJob {
    int32_t B = 0;
    int64_t n = 0;               // points of all clouds (each has two or more)
    int64_t edges_total = 0;
    const float* pts = nullptr;  // the clouds' float offsets (CloudIn::foff) count from here
    char* ws = nullptr;          // emst_workspace_bytes_batched(n, B)
    int32_t* edges = nullptr;
    float* weights = nullptr;
    float* d2 = nullptr;
    char* h = nullptr;           // pinned host block (bjob_host_bytes(B))
    int phase = kBCodes;         // the next phase to queue
    bool wait = false;           // the phase in flight must be read before the next is queued
    bool rounds_done = false;    // a round left one component per cloud
    int next_round = 0;          // the next round to queue
    int round = 0;               // the next round to read
    int64_t ncomp = 0;           // components entering `round`
    int64_t prev = 0;            // components entering `round` - 1 (0: none)
    int variant = 13;
    int lds_depth = 8;
    int height = 0;
    uint32_t root = 0;
    int codes_in1 = 0;
    int full = 0;
    int cloud_bits = 0;
    int nshifts = 0;
    int shifts[8] = {};
    emst_stats S;
    Ctrl* ctrl(int k) const { return reinterpret_cast<Ctrl*>(h + (size_t)k * a256(sizeof(Ctrl))); }
    CloudIn* cin() const { return reinterpret_cast<CloudIn*>(h + 2 * a256(sizeof(Ctrl))); }
    CloudBox* cbox() const {
        return reinterpret_cast<CloudBox*>(reinterpret_cast<char*>(cin()) + a256(sizeof(CloudIn) * (size_t)B));
    }
};

static size_t bjob_host_bytes(int32_t B) {
    return 2 * a256(sizeof(Ctrl)) + a256(sizeof(CloudIn) * (size_t)B) + a256(sizeof(CloudBox) * (size_t)B);
}

// Whether the job's next phase may be queued while `inflight` (0-2) queued
// phases have not been read.
static bool bjob_can_queue(const BJob& j, int inflight) {
    if (j.phase == kBDone) return false;
    if (inflight == 0) return true;
    if (inflight >= 2 || j.wait) return false;
    if (j.phase == kBRound)  // one round in flight: queue the next if the last shrink predicts it is needed
        return j.next_round < 64 &&
               (j.prev == 0 || (double)j.ncomp * (double)j.ncomp >= 2.0 * (double)j.prev * (double)j.B);
    return j.phase == kBFinal;  // the round in flight was queued past the end
}

static TraverseArgs<3> bjob_args(const BJob& j, const BatchBufs& x) {
    TraverseArgs<3> ta = traverse_args<3>(x.b, j.n, j.root);
    ta.cloud_of = x.cloud_sorted;
    ta.cloud_root = x.croot;
    ta.lds_depth = j.lds_depth;
    return ta;
}

// Queue the job's next phase; its control block goes to `mirror`, and
// *kind receives the phase queued.
static int bjob_enqueue(emst_ctx* ctx, BJob& j, hipStream_t st, Ctrl* mirror, int* kind) {
    BatchBufs x = batch_bufs(j.ws, j.n, j.B);
    Bufs<3>& b = x.b;
    const int64_t n = j.n;
    *kind = j.phase;
    switch (j.phase) {
    case kBCodes: {  // per-cloud boxes and quantisation, codes with the cloud id on top
        HIP_TRY(hipMemcpyAsync(x.cin, j.cin(), sizeof(CloudIn) * j.B, hipMemcpyHostToDevice, st));
        k_init_ctrl<<<1, 64, 0, st>>>(b.ctrl);
        k_batch_box_init<<<grid_for(j.B), 256, 0, st>>>(x.cin, j.B, x.cbox);
        k_batch_unpack<<<unpack_grid(n), 256, 0, st>>>(j.pts, x.cin, j.B, n, x.pts3, x.cloud_of, x.cbox);
        j.cloud_bits = j.B > 1 ? 64 - __builtin_clzll((unsigned long long)(j.B - 1)) : 0;
        // a cloud that fails validation gets codes from its unusable box; the
        // batch is then started again without it
        k_batch_mparams<<<grid_for(j.B), 256, 0, st>>>(x.cbox, x.cin, j.B, 64 - j.cloud_bits, x.cm);
        const int nb = (int)std::min<unsigned>(grid_for(n), kPartBlocks);
        uint64_t* part = reinterpret_cast<uint64_t*>(b.bpart);
        k_batch_morton<<<nb, 256, 0, st>>>(x.pts3, x.cloud_of, x.cm, n, 64 - j.cloud_bits, b.k0, b.v0, part);
        k_or_and_final<<<1, 256, 0, st>>>(part, nb, b.ctrl);
        HIP_TRY(hipMemcpyAsync(j.cbox(), x.cbox, sizeof(CloudBox) * j.B, hipMemcpyDeviceToHost, st));
        j.wait = true;
        break;
    }
    case kBTree: {  // sort, gather, hierarchy
        HIP_TRY(radix_sort_pairs(st, b.k0, b.v0, b.k1, b.v1, b.hist, n, j.shifts, j.nshifts, &j.codes_in1));
        const uint64_t* codes = j.codes_in1 ? b.k1 : b.k0;
        const uint32_t* perm = j.codes_in1 ? b.v1 : b.v0;
        k_gather<3><<<grid_for(n), 256, 0, st>>>(x.pts3, perm, n, b.spts, b.orig, b.labels, b.exch);
        k_fill_u32<<<grid_for(4 * n), 256, 0, st>>>(reinterpret_cast<uint32_t*>(b.eud), 4 * n, kNone);
        k_batch_sorted_cloud<<<grid_for(n), 256, 0, st>>>(x.cloud_of, perm, n, x.cloud_sorted);
        if (int rc = build_hierarchy<3>(ctx, b, codes, n, st)) return rc;
        j.wait = true;
        break;
    }
    case kBFit: {  // boxes, every cloud's subtree root, the first round
        const uint64_t* codes = j.codes_in1 ? b.k1 : b.k0;
        if (int rc = fit_levels<3>(ctx, b, codes, n, (uint32_t)j.height, st)) return rc;
        k_fill_u32<<<grid_for(j.B), 256, 0, st>>>(x.croot, j.B, kNone);
        k_cloud_roots<<<grid_for(n - 1), 256, 0, st>>>(b.rlo, b.rhi, x.cloud_sorted, x.cin, n - 1, x.croot);
        HIP_TRY(hipGetLastError());
        TraverseArgs<3> ta = bjob_args(j, x);
        if (int rc = enqueue_round<3>(ctx, b, ta, n, 0, j.height, j.variant, x.cloud_sorted, j.B, false, st))
            return rc;
        j.next_round = 1;
        j.phase = kBRound;
        break;
    }
    case kBRound: {
        if (j.next_round >= 64) return fail(ctx, EMST_EINTERNAL, "too many rounds");
        TraverseArgs<3> ta = bjob_args(j, x);
        if (int rc = enqueue_round<3>(ctx, b, ta, n, j.next_round, j.height, j.variant, x.cloud_sorted, j.B, false,
                                      st))
            return rc;
        ++j.next_round;
        break;
    }
    case kBFinal: {  // per-cloud canonical order (the full sort only after a long run of ties)
        const uint32_t* order = nullptr;
        if (int rc = sort_edges<3>(ctx, b, n, x.cloud_sorted, j.cloud_bits, j.full != 0, &order, st)) return rc;
        k_batch_edge_write<<<grid_for(n), 256, 0, st>>>(b.eud, order, x.cloud_sorted, x.cin, n, j.edges, j.weights,
                                                        j.d2);
        j.wait = true;
        break;
    }
    default:
        return fail(ctx, EMST_EINTERNAL, "batch already finished");
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(mirror, b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    return EMST_OK;
}

// Once a queued phase of kind `kind` has completed: read its mirror `h` and
// pick the next phase.  After the first phase, clouds that fail validation
// are listed in *bad (cloud, status) and the job stays where it is; the
// caller drops them and starts the job again.  A round read after the last
// one (queued before the end was known) changes nothing.
static int bjob_advance(emst_ctx* ctx, BJob& j, int kind, const Ctrl* h, std::vector<std::pair<int, int>>* bad) {
    switch (kind) {
    case kBCodes: {
        j.wait = false;
        const CloudBox* cb = j.cbox();
        bad->clear();
        for (int32_t c = 0; c < j.B; ++c) {
            float l[3], u[3];
            for (int k = 0; k < 3; ++k) { l[k] = ord_dec(cb[c].mn[k]); u[k] = ord_dec(cb[c].mx[k]); }
            if (cb[c].bad) bad->push_back({c, EMST_ENONFINITE});
            else if (!extent_ok(l, u, 3)) bad->push_back({c, EMST_ERANGE});
        }
        if (!bad->empty()) return EMST_OK;
        const uint64_t vary = h->key_or ^ h->key_and;
        j.nshifts = 0;
        for (int s = 0; s < 64; s += 8)
            if ((vary >> s) & 0xFFull) j.shifts[j.nshifts++] = s;
        j.phase = kBTree;
        return EMST_OK;
    }
    case kBTree:
        j.wait = false;
        if (int rc = check_hierarchy(ctx, h, j.n)) return rc;
        j.height = (int)h->height;
        j.root = h->root;
        j.S.tree_height = (int32_t)h->height;
        j.ncomp = j.n;
        j.prev = 0;
        j.round = 0;
        j.next_round = 0;
        j.rounds_done = false;
        j.phase = kBFit;
        return EMST_OK;
    case kBFit:
    case kBRound: {
        if (j.rounds_done) return EMST_OK;  // queued past the end: it returned at once
        const int64_t entering = j.ncomp;
        j.S.components[j.round] = entering;
        if (int rc = finish_round(ctx, h, j.round, j.B, j.ncomp, j.S)) return rc;
        j.prev = entering;
        ++j.round;
        if (j.ncomp <= j.B) {
            if ((int64_t)h->edge_count != j.edges_total) return fail(ctx, EMST_EINTERNAL, "wrong edge count");
            j.S.rounds = j.round;
            j.S.traversal_launches = j.round;
            j.S.traversal_variant = j.variant;
            j.rounds_done = true;
            j.phase = kBFinal;
        }
        return EMST_OK;
    }
    case kBFinal:
        j.wait = false;
        if (h->long_ties && !j.full) j.full = 1;  // again, with the full sort
        else j.phase = kBDone;
        return EMST_OK;
    default:
        return fail(ctx, EMST_EINTERNAL, "batch already finished");
    }
}

struct SolverSlot {
    int state = 0;          // 0 free, 1 running, 2 done, < 0: failed with that status
    int64_t tag = 0;
    size_t off = 0, bytes = 0;   // the points, until the cohort has unpacked them (bytes = 0 after)
    size_t quota = 0;            // emst_solver_slot_bytes, held from admit to take
    int64_t n = 0;
    int dim = 3;
    int cohort = -1;        // -1: waiting for the next step
    int64_t eoff = 0;       // first edge in the cohort's outputs
    uint64_t order = 0;     // admission order
    std::string err;
};

struct Cohort {
    bool live = false;      // phases still to run
    bool held = false;      // owns its region (live: outputs and workspace; finished: the outputs
                            // until every member's result is taken and copied)
    bool fresh = false;     // not started: its first phase waits for the caller's stream
    bool releasing = false; // every result taken; the region is free once `rel` has completed
    std::vector<int> slots; // member slots, in cloud order
    size_t off = 0, bytes = 0;
    int remaining = 0;      // members whose results were not taken yet
    BJob job;
    char* host = nullptr;   // pinned block of the job
    size_t host_bytes = 0;
    hipStream_t st = nullptr;
    int nq = 0, head = 0;   // queued phases not yet read: a ring of two
    int kind[2] = {};
    hipEvent_t ev[2] = {};  // follows each queued phase
    hipEvent_t rel = nullptr;
};

struct emst_solver {
    emst_ctx* ctx = nullptr;
    char* base = nullptr;
    size_t budget = 0;
    size_t reserved = 0;    // sum of the shares of the admitted, not yet taken requests
    uint64_t next_order = 0;
    std::vector<SolverSlot> slots;
    std::vector<Cohort> cohorts;
    hipEvent_t fork = nullptr;  // orders a cohort's first phase after the caller's stream
};

// Budget a request holds from admit to take: its points while they wait,
// and the workspace and outputs of a cohort of that one request, so the
// requests admitted together always fit one cohort.
extern "C" size_t emst_solver_slot_bytes(int64_t n, int dim) {
    if (n < 0 || n > 0x7FFFFFFFll || (dim != 2 && dim != 3)) return 0;
    const size_t m = (size_t)(n > 1 ? n - 1 : 0);
    return a256((size_t)n * dim * 4) + a256(emst_workspace_bytes_batched(n > 1 ? n : 2, 1)) + a256(m * 8) +
           2 * a256(m * 4);
}

static size_t output_bytes(int64_t edges) { return a256((size_t)edges * 8) + 2 * a256((size_t)edges * 4); }

static size_t cohort_bytes(int64_t points, int32_t clouds, int64_t edges) {
    return output_bytes(edges) + a256(emst_workspace_bytes_batched(points, clouds));
}

// A free range of `need` bytes in the budget: the lowest one (cohorts) or
// the highest one (the points of waiting requests), so that the two kinds
// of region grow from opposite ends.
static bool sv_place(const emst_solver* sv, size_t need, bool high, size_t* at) {
    std::vector<std::pair<size_t, size_t>> used;
    for (const SolverSlot& q : sv->slots)
        if (q.state != 0 && q.bytes) used.push_back({q.off, q.off + q.bytes});
    for (const Cohort& c : sv->cohorts)
        if (c.held) used.push_back({c.off, c.off + c.bytes});
    std::sort(used.begin(), used.end());
    bool found = false;
    size_t prev = 0;  // end of the used range before the current gap
    for (size_t k = 0; k <= used.size(); ++k) {
        const size_t gap_end = k < used.size() ? used[k].first : sv->budget;
        if (gap_end >= prev && gap_end - prev >= need) {
            if (!high) {
                *at = prev;
                return true;
            }
            *at = (gap_end - need) & ~(size_t)255;
            found = *at >= prev;
        }
        if (k < used.size()) prev = std::max(prev, used[k].second);
    }
    return found;
}

// The largest free range of the budget.
static size_t sv_largest_gap(const emst_solver* sv) {
    std::vector<std::pair<size_t, size_t>> used;
    for (const SolverSlot& q : sv->slots)
        if (q.state != 0 && q.bytes) used.push_back({q.off, q.off + q.bytes});
    for (const Cohort& c : sv->cohorts)
        if (c.held) used.push_back({c.off, c.off + c.bytes});
    std::sort(used.begin(), used.end());
    size_t best = 0, prev = 0;
    for (size_t k = 0; k <= used.size(); ++k) {
        const size_t gap_end = k < used.size() ? used[k].first : sv->budget;
        if (gap_end > prev) best = std::max(best, gap_end - prev);
        if (k < used.size()) prev = std::max(prev, used[k].second);
    }
    return best;
}

extern "C" void emst_solver_destroy(emst_solver* sv);

extern "C" int emst_solver_create(emst_ctx* ctx, void* d_budget, size_t budget_bytes, int32_t max_slots,
                                  emst_solver** out) {
    if (!ctx || !out || max_slots < 1 || max_slots > 4096) return EMST_EINVAL;
    *out = nullptr;
    if (!d_budget || ((uintptr_t)d_budget & 255u)) return fail(ctx, EMST_EINVAL, "budget must be 256-byte aligned");
    emst_solver* sv = new (std::nothrow) emst_solver();
    if (!sv) return EMST_ENOMEM;
    sv->ctx = ctx;
    sv->base = (char*)d_budget;
    sv->budget = budget_bytes & ~(size_t)255;
    sv->slots.resize(max_slots);
    sv->cohorts.resize(max_slots);
    const bool ok = hipSetDevice(ctx->device) == hipSuccess &&
                    hipEventCreateWithFlags(&sv->fork, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        emst_solver_destroy(sv);
        return fail(ctx, EMST_EHIP, "solver set-up failed");
    }
    *out = sv;
    return EMST_OK;
}

extern "C" void emst_solver_destroy(emst_solver* sv) {
    if (!sv) return;
    for (Cohort& c : sv->cohorts) {
        if (c.st) {
            (void)hipStreamSynchronize(c.st);
            (void)hipStreamDestroy(c.st);
        }
        for (hipEvent_t e : c.ev)
            if (e) (void)hipEventDestroy(e);
        if (c.rel) (void)hipEventDestroy(c.rel);
        if (c.host) (void)hipHostFree(c.host);
    }
    if (sv->fork) (void)hipEventDestroy(sv->fork);
    delete sv;
}

// Regions of cohorts whose results have all been taken and copied are free.
static void reclaim(emst_solver* sv) {
    for (Cohort& c : sv->cohorts)
        if (c.releasing && hipEventQuery(c.rel) == hipSuccess) {
            c.releasing = false;
            c.held = false;
        }
}

extern "C" int emst_solver_admit(emst_solver* sv, const float* d_points, int64_t n, int32_t dim, int64_t tag,
                                 void* stream, int32_t* slot) {
    if (!sv || !slot) return EMST_EINVAL;
    emst_ctx* ctx = sv->ctx;
    ctx->err.clear();
    *slot = -1;
    if (n < 0 || n > 0x7FFFFFFFll) return fail(ctx, EMST_EINVAL, "n out of range");
    if (dim != 2 && dim != 3) return fail(ctx, EMST_EINVAL, "dim must be 2 or 3");
    if (n > 0 && !d_points) return fail(ctx, EMST_EINVAL, "null pointer");
    const size_t quota = emst_solver_slot_bytes(n, dim);
    if (quota > sv->budget) return fail(ctx, EMST_ENOMEM, "request larger than the whole budget");
    int free_slot = -1;
    for (int s = 0; s < (int)sv->slots.size() && free_slot < 0; ++s)
        if (sv->slots[s].state == 0) free_slot = s;
    if (free_slot < 0) return fail(ctx, EMST_EBUSY, "no free slot");
    if (sv->reserved + quota > sv->budget) return fail(ctx, EMST_EBUSY, "budget full");
    const size_t pts_bytes = n >= 2 ? a256((size_t)n * dim * 4) : 0;
    reclaim(sv);
    size_t at = 0;
    if (pts_bytes && !sv_place(sv, pts_bytes, true, &at)) return fail(ctx, EMST_EBUSY, "budget full");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, EMST_EHIP, "hipSetDevice failed");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (pts_bytes)
        HIP_TRY(hipMemcpyAsync(sv->base + at, d_points, (size_t)n * dim * 4, hipMemcpyDeviceToDevice, st));
    SolverSlot& q = sv->slots[free_slot];
    q.tag = tag;
    q.off = at;
    q.bytes = pts_bytes;
    q.quota = quota;
    q.n = n;
    q.dim = dim;
    q.cohort = -1;
    q.eoff = 0;
    q.order = sv->next_order++;
    q.err.clear();
    q.state = n < 2 ? 2 : 1;  // 0 or 1 point: nothing to do
    sv->reserved += quota;
    *slot = free_slot;
    return EMST_OK;
}

static void release_points(SolverSlot& q) { q.bytes = 0; }

// Fill the cloud table of cohort c from its member slots and restart its job.
static void cohort_tables(emst_solver* sv, Cohort& co) {
    BJob& j = co.job;
    j.B = (int32_t)co.slots.size();
    j.n = 0;
    j.edges_total = 0;
    CloudIn* cin = j.cin();
    for (int32_t c = 0; c < j.B; ++c) {
        SolverSlot& q = sv->slots[co.slots[c]];
        cin[c].off = j.n;
        cin[c].n = q.n;
        cin[c].foff = (int64_t)(q.off / 4);  // floats from the budget's base
        cin[c].eoff = j.edges_total;
        cin[c].dim = q.dim;
        cin[c].pad = 0;
        q.eoff = j.edges_total;
        j.n += q.n;
        j.edges_total += q.n - 1;
    }
    // the outputs first: a finished cohort keeps only them
    const size_t E = (size_t)j.edges_total;
    char* region = sv->base + co.off;
    j.edges = reinterpret_cast<int32_t*>(region);
    j.weights = reinterpret_cast<float*>(region + a256(E * 8));
    j.d2 = reinterpret_cast<float*>(region + a256(E * 8) + a256(E * 4));
    j.ws = region + output_bytes(j.edges_total);
    j.pts = reinterpret_cast<const float*>(sv->base);
    j.phase = kBCodes;
    j.wait = false;
    j.rounds_done = false;
    j.next_round = 0;
    j.round = 0;
    j.ncomp = 0;
    j.prev = 0;
    j.full = 0;
    memset(&j.S, 0, sizeof(j.S));
}

// Start a cohort from the requests waiting since the last step: as many, in
// admission order, as fit one free range of the budget together, unless
// kSolverCohorts cohorts run already.
static int form_cohort(emst_solver* sv, int* done) {
    emst_ctx* ctx = sv->ctx;
    int live = 0;
    for (const Cohort& c : sv->cohorts) live += c.live;
    if (live >= kSolverCohorts) return EMST_OK;
    reclaim(sv);
    std::vector<int> wait;
    for (int s = 0; s < (int)sv->slots.size(); ++s)
        if (sv->slots[s].state == 1 && sv->slots[s].cohort < 0) wait.push_back(s);
    if (wait.empty()) return EMST_OK;
    std::sort(wait.begin(), wait.end(), [&](int a, int b) { return sv->slots[a].order < sv->slots[b].order; });
    const size_t gap = sv_largest_gap(sv);
    int k = 0;
    size_t at = 0;
    int64_t pts = 0, edges = 0;
    for (int s : wait) {
        const int64_t n = sv->slots[s].n;
        if (cohort_bytes(pts + n, k + 1, edges + n - 1) > gap) break;
        pts += n;
        edges += n - 1;
        ++k;
    }
    if (k > 0 && !sv_place(sv, cohort_bytes(pts, k, edges), false, &at))
        return fail(ctx, EMST_EINTERNAL, "no range for a cohort that fits the largest gap");
    if (k == 0) {
        bool any_held = false;
        for (const Cohort& c : sv->cohorts) any_held |= c.held;
        if (!any_held) {
            // no cohort holds memory that a step or a take could free: the
            // first waiting request fails instead of waiting for ever
            SolverSlot& q = sv->slots[wait[0]];
            q.state = EMST_ENOMEM;
            q.err = "the budget has no free range for this request";
            release_points(q);
            ++*done;
        }
        return EMST_OK;
    }
    int ci = -1;
    for (int c = 0; c < (int)sv->cohorts.size() && ci < 0; ++c)
        if (!sv->cohorts[c].held) ci = c;
    if (ci < 0) return EMST_OK;  // (cannot happen: a held cohort has a member slot)
    Cohort& co = sv->cohorts[ci];
    if (!co.st && hipStreamCreateWithFlags(&co.st, hipStreamNonBlocking) != hipSuccess)
        return fail(ctx, EMST_EHIP, "hipStreamCreate failed");
    for (hipEvent_t* e : {&co.ev[0], &co.ev[1], &co.rel})
        if (!*e && hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess)
            return fail(ctx, EMST_EHIP, "hipEventCreate failed");
    if (!co.host) {  // sized once for the largest cohort (pinned allocations are slow)
        const size_t hb = bjob_host_bytes((int32_t)sv->slots.size());
        if (hipHostMalloc((void**)&co.host, hb, hipHostMallocDefault) != hipSuccess)
            return fail(ctx, EMST_EHIP, "hipHostMalloc failed");
        co.host_bytes = hb;
    }
    co.slots.assign(wait.begin(), wait.begin() + k);
    co.off = at;
    co.bytes = cohort_bytes(pts, k, edges);
    co.held = true;
    co.live = true;
    co.remaining = k;
    co.nq = 0;
    co.head = 0;
    co.fresh = true;
    co.releasing = false;
    co.job = BJob();
    co.job.h = co.host;
    int t = 13, depth = 8;
    pick_shape(ctx, 1, 3, pts, &t, &depth);
    co.job.variant = (t == 0 || t == 5 || t == 8 || t == 13) ? t : 7;
    co.job.lds_depth = depth;
    for (int s : co.slots) sv->slots[s].cohort = ci;
    cohort_tables(sv, co);
    return EMST_OK;
}

// A cohort's members fail together with `rc`.
static void cohort_fail(emst_solver* sv, Cohort& co, int rc, const std::string& msg, int* done) {
    (void)hipStreamSynchronize(co.st);  // nothing queued may outlive the region
    co.nq = 0;
    for (int s : co.slots) {
        SolverSlot& q = sv->slots[s];
        q.state = rc;
        q.err = msg;
        q.cohort = -1;
        release_points(q);
        ++*done;
    }
    co.slots.clear();
    co.live = false;
    co.held = false;
    co.remaining = 0;
}

// The host side of a completed phase (kind, mirror) of a cohort.
static void cohort_advance(emst_solver* sv, Cohort& co, int kind, const Ctrl* mirror, int* done) {
    emst_ctx* ctx = sv->ctx;
    std::vector<std::pair<int, int>> bad;
    const int rc = bjob_advance(ctx, co.job, kind, mirror, &bad);
    if (rc) {
        cohort_fail(sv, co, rc, ctx->err, done);
        return;
    }
    if (!bad.empty()) {
        // invalid requests fail alone; the others start again without them
        std::vector<int> keep;
        size_t b = 0;
        for (int32_t k = 0; k < (int32_t)co.slots.size(); ++k) {
            SolverSlot& q = sv->slots[co.slots[k]];
            if (b < bad.size() && bad[b].first == k) {
                q.state = bad[b].second;
                q.err = bad[b].second == EMST_ENONFINITE ? "non-finite coordinate"
                                                         : "squared extent of the cloud overflows float32";
                q.cohort = -1;
                release_points(q);
                ++*done;
                ++b;
            } else {
                keep.push_back(co.slots[k]);
            }
        }
        co.slots = keep;
        co.remaining = (int)keep.size();
        if (keep.empty()) {
            co.live = false;
            co.held = false;
        } else {
            cohort_tables(sv, co);  // the region, sized for more, still fits
        }
        return;
    }
    if (kind == kBCodes)  // the points are in the workspace now
        for (int s : co.slots) release_points(sv->slots[s]);
    if (co.job.phase == kBDone) {
        co.live = false;
        co.bytes = output_bytes(co.job.edges_total);  // the workspace is free again
        for (int s : co.slots) {
            sv->slots[s].state = 2;
            ++*done;
        }
    }
}

extern "C" int emst_solver_step(emst_solver* sv, void* stream, int32_t* n_finished) {
    if (!sv) return EMST_EINVAL;
    emst_ctx* ctx = sv->ctx;
    ctx->err.clear();
    if (n_finished) *n_finished = 0;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, EMST_EHIP, "hipSetDevice failed");
    int done = 0;
    if (int rc = form_cohort(sv, &done)) return rc;
    bool fresh = false;
    std::vector<Cohort*> act;  // the live cohorts (the table holds one entry per slot)
    for (Cohort& c : sv->cohorts)
        if (c.live) {
            act.push_back(&c);
            fresh |= c.fresh;
        }
    // a new cohort starts after what the caller's stream holds (admitted points)
    if (fresh) HIP_TRY(hipEventRecord(sv->fork, reinterpret_cast<hipStream_t>(stream)));
    for (;;) {
        bool moved = false, busy = false;
        for (Cohort* cp : act) {
            Cohort& co = *cp;
            if (!co.live) continue;
            while (co.nq > 0) {  // read the completed phases in order
                const hipError_t q = hipEventQuery(co.ev[co.head]);
                if (q == hipErrorNotReady) break;
                if (q != hipSuccess) return fail(ctx, EMST_EHIP, hipGetErrorString(q));
                const int k = co.head;
                co.head ^= 1;
                --co.nq;
                moved = true;
                cohort_advance(sv, co, co.kind[k], co.job.ctrl(k), &done);
                if (!co.live) break;
            }
            if (!co.live) continue;
            while (bjob_can_queue(co.job, co.nq)) {
                if (co.fresh) {
                    HIP_TRY(hipStreamWaitEvent(co.st, sv->fork, 0));
                    co.fresh = false;
                }
                const int k = co.head ^ co.nq;
                if (int rc = bjob_enqueue(ctx, co.job, co.st, co.job.ctrl(k), &co.kind[k])) {
                    cohort_fail(sv, co, rc, ctx->err, &done);
                    moved = true;
                    break;
                }
                HIP_TRY(hipEventRecord(co.ev[k], co.st));
                ++co.nq;
            }
            busy |= co.live && co.nq > 0;
        }
        if (moved || !busy) break;
        std::this_thread::yield();
    }
    if (n_finished) *n_finished = done;
    return EMST_OK;
}

extern "C" int emst_solver_poll(const emst_solver* sv, int32_t slot, int32_t* state, int64_t* tag) {
    if (!sv || slot < 0 || slot >= (int)sv->slots.size() || !state) return EMST_EINVAL;
    *state = sv->slots[slot].state;
    if (tag) *tag = sv->slots[slot].tag;
    return EMST_OK;
}

extern "C" int emst_solver_ready(const emst_solver* sv, int32_t* slots, int32_t cap, int32_t* count) {
    if (!sv || !count || cap < 0 || (cap > 0 && !slots)) return EMST_EINVAL;
    std::vector<std::pair<std::pair<int, int64_t>, int32_t>> r;
    for (int s = 0; s < (int)sv->slots.size(); ++s)
        if (sv->slots[s].state == 2 || sv->slots[s].state < 0) r.push_back({{sv->slots[s].cohort, sv->slots[s].eoff}, s});
    std::sort(r.begin(), r.end());
    int32_t k = 0;
    for (; k < cap && k < (int32_t)r.size(); ++k) slots[k] = r[k].second;
    *count = k;
    return EMST_OK;
}

extern "C" int emst_solver_take_many(emst_solver* sv, const int32_t* slots, int32_t count, int32_t* d_edges,
                                     float* d_weights, float* d_d2, int64_t* h_offsets, void* stream) {
    if (!sv || count < 0 || (count > 0 && (!slots || !h_offsets))) return EMST_EINVAL;
    emst_ctx* ctx = sv->ctx;
    ctx->err.clear();
    std::vector<char> seen(sv->slots.size(), 0);
    int64_t total = 0;
    for (int32_t i = 0; i < count; ++i) {
        const int32_t s = slots[i];
        if (s < 0 || s >= (int32_t)sv->slots.size() || seen[s]) return fail(ctx, EMST_EINVAL, "bad or repeated slot");
        seen[s] = 1;
        if (sv->slots[s].state != 2) return fail(ctx, EMST_EINVAL, "slot holds no finished result");
        h_offsets[i] = total;
        total += sv->slots[s].n > 1 ? sv->slots[s].n - 1 : 0;
    }
    if (count > 0) h_offsets[count] = total;
    if (total > 0 && (!d_edges || !d_weights)) return fail(ctx, EMST_EINVAL, "null pointer");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, EMST_EHIP, "hipSetDevice failed");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // one copy per array for every run of results that lie back to back in
    // one cohort's outputs
    for (int32_t i = 0; i < count;) {
        const SolverSlot& q = sv->slots[slots[i]];
        int64_t m = q.n > 1 ? q.n - 1 : 0;
        int32_t k = i + 1;
        if (q.cohort >= 0) {
            for (; k < count; ++k) {
                const SolverSlot& r = sv->slots[slots[k]];
                if (r.cohort != q.cohort || r.eoff != q.eoff + m) break;
                m += r.n - 1;
            }
            const BJob& j = sv->cohorts[q.cohort].job;
            const int64_t o = h_offsets[i];
            HIP_TRY(hipMemcpyAsync(d_edges + 2 * o, j.edges + 2 * q.eoff, (size_t)m * 8, hipMemcpyDeviceToDevice, st));
            HIP_TRY(hipMemcpyAsync(d_weights + o, j.weights + q.eoff, (size_t)m * 4, hipMemcpyDeviceToDevice, st));
            if (d_d2) HIP_TRY(hipMemcpyAsync(d_d2 + o, j.d2 + q.eoff, (size_t)m * 4, hipMemcpyDeviceToDevice, st));
        }
        i = k;
    }
    // each cohort touched passes the copies on its (idle) stream; the last
    // take of a cohort frees its region once they are done
    std::vector<int> taken(sv->cohorts.size(), 0);
    for (int32_t i = 0; i < count; ++i)
        if (sv->slots[slots[i]].cohort >= 0) ++taken[sv->slots[slots[i]].cohort];
    for (int c = 0; c < (int)sv->cohorts.size(); ++c) {
        if (!taken[c]) continue;
        Cohort& co = sv->cohorts[c];
        HIP_TRY(hipEventRecord(co.rel, st));
        HIP_TRY(hipStreamWaitEvent(co.st, co.rel, 0));
        co.remaining -= taken[c];
        if (co.remaining == 0) {
            HIP_TRY(hipEventRecord(co.rel, co.st));
            co.releasing = true;
        }
    }
    for (int32_t i = 0; i < count; ++i) {
        SolverSlot& q = sv->slots[slots[i]];
        sv->reserved -= q.quota;
        release_points(q);
        q.cohort = -1;
        q.state = 0;
    }
    return EMST_OK;
}

extern "C" int emst_solver_take(emst_solver* sv, int32_t slot, int32_t* d_edges, float* d_weights, float* d_d2,
                                void* stream) {
    if (!sv || slot < 0 || slot >= (int)sv->slots.size()) return EMST_EINVAL;
    emst_ctx* ctx = sv->ctx;
    SolverSlot& q = sv->slots[slot];
    if (q.state == 0) return fail(ctx, EMST_EINVAL, "slot is free");
    if (q.state == 1) return fail(ctx, EMST_EBUSY, "request still running");
    if (q.state < 0) {
        const int rc = q.state;
        ctx->err = q.err;
        sv->reserved -= q.quota;
        release_points(q);
        q.state = 0;
        return rc;
    }
    const size_t m = (size_t)(q.n > 1 ? q.n - 1 : 0);
    if (m) {
        if (!d_edges || !d_weights) return fail(ctx, EMST_EINVAL, "null pointer");
        if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, EMST_EHIP, "hipSetDevice failed");
        Cohort& co = sv->cohorts[q.cohort];
        const BJob& j = co.job;
        hipStream_t st = reinterpret_cast<hipStream_t>(stream);
        HIP_TRY(hipMemcpyAsync(d_edges, j.edges + 2 * q.eoff, m * 8, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_weights, j.weights + q.eoff, m * 4, hipMemcpyDeviceToDevice, st));
        if (d_d2) HIP_TRY(hipMemcpyAsync(d_d2, j.d2 + q.eoff, m * 4, hipMemcpyDeviceToDevice, st));
        // the cohort's (idle) stream passes these copies, so that its release
        // event follows the copies of every take, whatever their streams
        HIP_TRY(hipEventRecord(co.rel, st));
        HIP_TRY(hipStreamWaitEvent(co.st, co.rel, 0));
    }
    if (q.cohort >= 0) {
        Cohort& co = sv->cohorts[q.cohort];
        if (--co.remaining == 0) {
            HIP_TRY(hipEventRecord(co.rel, co.st));
            co.releasing = true;
        }
        q.cohort = -1;
    }
    sv->reserved -= q.quota;
    release_points(q);
    q.state = 0;
    return EMST_OK;
}

extern "C" size_t emst_workspace_bytes_batched(int64_t total_points, int32_t n_clouds) {
    if (total_points < 0 || total_points > 0x7FFFFFFFll || n_clouds < 1) return 0;
    return make_batch_layout(total_points, n_clouds).total;
}

extern "C" int emst_build_batched(emst_ctx* ctx, const float* d_points, const int64_t* h_offsets,
                                  const int32_t* h_dims, int32_t n_clouds, int32_t* d_edges, float* d_weights,
                                  float* d_d2, int64_t* h_edge_offsets, void* d_workspace, size_t ws_bytes,
                                  void* stream) {
    if (!ctx) return EMST_EINVAL;
    ctx->err.clear();
    if (n_clouds < 1 || !h_offsets || !h_dims) return fail(ctx, EMST_EINVAL, "bad batch description");
    if (h_offsets[0] != 0) return fail(ctx, EMST_EINVAL, "offsets must start at 0");
    for (int32_t c = 0; c < n_clouds; ++c) {
        if (h_offsets[c + 1] < h_offsets[c]) return fail(ctx, EMST_EINVAL, "offsets must not decrease");
        if (h_dims[c] != 2 && h_dims[c] != 3) return fail(ctx, EMST_EINVAL, "dim must be 2 or 3");
    }
    const int64_t n = h_offsets[n_clouds];
    if (n > 0x7FFFFFFFll) return fail(ctx, EMST_EINVAL, "too many points");
    if (n < 2) {
        if (h_edge_offsets)
            for (int32_t c = 0; c <= n_clouds; ++c) h_edge_offsets[c] = 0;
        memset(&ctx->stats, 0, sizeof(ctx->stats));
        ctx->stats.n = n;
        return EMST_OK;
    }
    int64_t m = 0;
    for (int32_t c = 0; c < n_clouds; ++c) m += std::max<int64_t>(h_offsets[c + 1] - h_offsets[c] - 1, 0);
    if (!d_points || !d_workspace || (m > 0 && (!d_edges || !d_weights)))
        return fail(ctx, EMST_EINVAL, "null pointer");
    if (((uintptr_t)d_workspace & 255u) != 0) return fail(ctx, EMST_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < emst_workspace_bytes_batched(n, n_clouds)) return fail(ctx, EMST_ENOMEM, "workspace too small");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, EMST_EHIP, "hipSetDevice failed");
    return batched_impl(ctx, d_points, h_offsets, h_dims, n_clouds, d_edges, d_weights, d_d2, h_edge_offsets,
                        (char*)d_workspace, reinterpret_cast<hipStream_t>(stream));
}

// ===========================================================================
// test entry points (include/emst_test.h)

namespace emst {

__global__ __launch_bounds__(256) void k_test_prep(const uint32_t* __restrict__ leaf_labels, int64_t n,
                                                   float* __restrict__ spts, uint32_t* __restrict__ orig,
                                                   uint32_t* __restrict__ labels, uint64_t* __restrict__ exch) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    spts[3 * i] = spts[3 * i + 1] = spts[3 * i + 2] = 0.f;
    orig[i] = (uint32_t)i;
    labels[i] = leaf_labels[i];
    if (i + 1 < n) exch[i] = ~0ull;
}

__global__ __launch_bounds__(256) void k_test_extract(const Rec<3>* __restrict__ recs, const uint2* __restrict__ lab2,
                                                      const uint32_t* __restrict__ node_parent, int64_t m,
                                                      int32_t* __restrict__ left, int32_t* __restrict__ right,
                                                      uint32_t* __restrict__ label) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    Child<3> c0, c1;
    unpack<3>(recs[k], c0, c1);
    left[k] = (c0.ref & kLeafFlag) ? -(int32_t)(c0.ref & ~kLeafFlag) - 1 : (int32_t)c0.ref;
    right[k] = (c1.ref & kLeafFlag) ? -(int32_t)(c1.ref & ~kLeafFlag) - 1 : (int32_t)c1.ref;
    const uint32_t link = node_parent[k];
    if (link == kNone) {
        const uint2 L = lab2[k];
        label[k] = (L.x == L.y) ? L.x : kInvalid;
    } else {
        const uint2 L = lab2[link >> 1];
        label[k] = (link & 1u) ? L.y : L.x;
    }
}

__global__ __launch_bounds__(256) void k_test_boxes(const Rec<3>* __restrict__ recs, int64_t m,
                                                    int32_t* __restrict__ left, int32_t* __restrict__ right,
                                                    float* __restrict__ lo, float* __restrict__ hi) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    Child<3> c0, c1;
    unpack<3>(recs[k], c0, c1);
    left[k] = (c0.ref & kLeafFlag) ? -(int32_t)(c0.ref & ~kLeafFlag) - 1 : (int32_t)c0.ref;
    right[k] = (c1.ref & kLeafFlag) ? -(int32_t)(c1.ref & ~kLeafFlag) - 1 : (int32_t)c1.ref;
    for (int d = 0; d < 3; ++d) {
        lo[3 * k + d] = fminf(c0.lo[d], c1.lo[d]);
        hi[3 * k + d] = fmaxf(c0.hi[d], c1.hi[d]);
    }
}

// emst_test_round: the smallest sorted position of every component
// (rep[c], initialised to kNone) ...
__global__ __launch_bounds__(256) void k_test_reps(const int32_t* __restrict__ comp,
                                                   const uint32_t* __restrict__ orig, int64_t n, uint32_t* rep) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) atomicMin(&rep[comp[orig[p]]], (uint32_t)p);
}

// ... becomes the label of its points, and every component starts the
// round as k_merge_parent leaves a root (no bound, no key, no edge).  Every
// point starts with itself as its last candidate (index and position),
// which lies in its own component, so no earlier result is reused.
__global__ __launch_bounds__(256) void k_test_labels(const int32_t* __restrict__ comp,
                                                     const uint32_t* __restrict__ orig,
                                                     const uint32_t* __restrict__ rep, int64_t n,
                                                     uint32_t* __restrict__ labels, uint32_t* __restrict__ ub,
                                                     uint64_t* __restrict__ compkey, uint32_t* __restrict__ compmax,
                                                     uint32_t* __restrict__ cand_d, uint32_t* __restrict__ cand_j,
                                                     uint32_t* __restrict__ cand_p) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t o = orig[p];
    const uint32_t l = rep[comp[o]];
    labels[p] = l;
    cand_j[p] = o;
    cand_d[p] = 0u;
    cand_p[p] = (uint32_t)p;
    if (l == (uint32_t)p) {
        ub[p] = kInfBits;
        compkey[p] = kKeyMax;
        compmax[p] = kNone;
    }
}

// The root list a round starts from: segment b holds, in ascending order,
// the roots among positions [b * cap, (b + 1) * cap).
__global__ __launch_bounds__(256) void k_test_root_list(const uint32_t* __restrict__ labels, int64_t n, RootList rl) {
    __shared__ uint32_t s_w[4];
    const int64_t lo = (int64_t)blockIdx.x * rl.cap;
    const int64_t hi = std::min<int64_t>(lo + rl.cap, n);
    uint32_t* seg = const_cast<uint32_t*>(rl.in) + rl.cap * blockIdx.x;
    uint32_t at = 0;
    const int lane = lane_id(), w = threadIdx.x >> 6;
    for (int64_t base = lo; base < hi; base += 256) {
        const int64_t p = base + threadIdx.x;
        const bool root = p < hi && labels[p] == (uint32_t)p;
        const uint64_t m = __ballot(root);
        if (lane == 0) s_w[w] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = at;
        for (int k = 0; k < w; ++k) before += s_w[k];
        if (root) seg[before + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = (uint32_t)p;
        at += s_w[0] + s_w[1] + s_w[2] + s_w[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) const_cast<uint32_t*>(rl.cnt_in)[blockIdx.x] = at;
}

// The component of every point after the round: the original index of its
// root point.
__global__ __launch_bounds__(256) void k_test_comp_out(const uint32_t* __restrict__ labels,
                                                       const uint32_t* __restrict__ orig, int64_t n,
                                                       int32_t* __restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) out[orig[p]] = (int32_t)orig[labels[p]];
}

template <int DIM>
int test_round(emst_ctx* ctx, const float* pts, int64_t n, const int32_t* comp, int round, int variant,
               const RoundCapture& cap, int32_t* comp_out, int64_t* ncomp_out, char* ws, hipStream_t st) {
    // the tree of emst_build (the phases up to the boxes, without round 0)
    Job j = make_job(ctx, pts, n, DIM, ws, nullptr, nullptr, nullptr, 0, nullptr, true, ctx->h_ctrl, false);
    j.variant = variant;
    if (int rc = job_run<DIM>(ctx, j, st)) return rc;
    const Layout L = make_layout(n, DIM);
    Bufs<DIM> b = carve<DIM>(ws, L);
    TraverseArgs<DIM> ta = job_args<DIM>(j, b);
    k_fill_u32<<<grid_for(n), 256, 0, st>>>(b.succ, n, kNone);
    k_test_reps<<<grid_for(n), 256, 0, st>>>(comp, b.orig, n, b.succ);
    k_test_labels<<<grid_for(n), 256, 0, st>>>(comp, b.orig, b.succ, n, b.labels, b.ub, b.compkey, b.compmax,
                                               b.cand_d, b.cand_j, b.cand_p);
    k_run_partials<<<run_tiles(n), 256, 0, st>>>(b.labels, n, b.run_part);
    RootList rl;
    uint32_t* lists[2] = {reinterpret_cast<uint32_t*>(b.k0), reinterpret_cast<uint32_t*>(b.k1)};
    uint32_t* counts = b.bpart + 4 * kPartBlocks;
    rl.in = lists[round & 1];
    rl.cnt_in = counts + kPartBlocks * (round & 1);
    rl.out = lists[(round + 1) & 1];
    rl.cnt_out = counts + kPartBlocks * ((round + 1) & 1);
    rl.cap = root_list_cap(n);
    k_test_root_list<<<root_list_blocks(n), 256, 0, st>>>(b.labels, n, rl);
    HIP_TRY(hipGetLastError());
    if (int rc = enqueue_round<DIM>(ctx, b, ta, n, round, j.height, variant, nullptr, 1, false, st, &cap)) return rc;
    k_test_comp_out<<<grid_for(n), 256, 0, st>>>(b.labels, b.orig, n, comp_out);
    HIP_TRY(hipGetLastError());
    if (int rc = read_ctrl(ctx, b.ctrl, st)) return rc;
    const Ctrl* h = ctx->h_ctrl;
    if (h->error & kErrStack) return fail(ctx, EMST_EINTERNAL, "traversal stack overflow");
    if (h->error & kErrJump) return fail(ctx, EMST_EINTERNAL, "component merge did not converge");
    if (h->error) return fail(ctx, EMST_EINTERNAL, "a component found no outgoing edge");
    *ncomp_out = (int64_t)h->ncomp_next;
    return EMST_OK;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_test_distances(const float* __restrict__ a, const float* __restrict__ b,
                                                        int64_t m, float* __restrict__ sq, float* __restrict__ box,
                                                        float* __restrict__ w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    float p[DIM], q[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        p[k] = a[i * DIM + k];
        q[k] = b[i * DIM + k];
    }
    const float d = sqdist<DIM>(p, q);
    sq[i] = d;
    box[i] = boxdist<DIM>(p, q, q);
    w[i] = edge_weight(d);
}

__global__ __launch_bounds__(256) void k_test_weights(uint32_t first, int64_t count, float* __restrict__ w) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) w[k] = edge_weight(bitsf(first + (uint32_t)k));
}

}  // namespace emst

extern "C" int emst_test_distances(emst_ctx* ctx, const float* d_a, const float* d_b, int64_t m, int dim,
                                   float* d_sq, float* d_box, float* d_w, void* stream) {
    if (!ctx) return EMST_EINVAL;
    ctx->err.clear();
    if (m < 0 || (dim != 2 && dim != 3)) return fail(ctx, EMST_EINVAL, "bad m or dim");
    if (m == 0) return EMST_OK;
    if (!d_a || !d_b || !d_sq || !d_box || !d_w) return fail(ctx, EMST_EINVAL, "null pointer");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const unsigned grid = (unsigned)((m + 255) / 256);
    if (dim == 3) k_test_distances<3><<<grid, 256, 0, st>>>(d_a, d_b, m, d_sq, d_box, d_w);
    else k_test_distances<2><<<grid, 256, 0, st>>>(d_a, d_b, m, d_sq, d_box, d_w);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    return EMST_OK;
}

extern "C" int emst_test_weights(emst_ctx* ctx, uint32_t first, int64_t count, float* d_w, void* stream) {
    if (!ctx) return EMST_EINVAL;
    ctx->err.clear();
    if (count < 0 || (uint64_t)first + (uint64_t)count > (1ull << 32)) return fail(ctx, EMST_EINVAL, "bad range");
    if (count == 0) return EMST_OK;
    if (!d_w) return fail(ctx, EMST_EINVAL, "null pointer");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    k_test_weights<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(first, count, d_w);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    return EMST_OK;
}

extern "C" int emst_test_round(emst_ctx* ctx, const float* d_points, int64_t n, int dim, const int32_t* d_comp,
                               int32_t round, int32_t variant, float* d_bound, float* d_cand_d, int32_t* d_cand_j,
                               float* d_comp_d2, int32_t* d_comp_u, int32_t* d_comp_v, int32_t* d_comp_out,
                               int64_t* ncomp_out, void* d_workspace, size_t ws_bytes, void* stream) {
    if (!ctx) return EMST_EINVAL;
    ctx->err.clear();
    if (n < 2 || n > 0x7FFFFFFFll || (dim != 2 && dim != 3)) return fail(ctx, EMST_EINVAL, "bad n or dim");
    if (round < 1 || round > 63) return fail(ctx, EMST_EINVAL, "round must be in [1, 63]");
    if (!variant_ok(variant)) return fail(ctx, EMST_EINVAL, "unknown traversal variant");
    if (!d_points || !d_comp || !d_bound || !d_cand_d || !d_cand_j || !d_comp_d2 || !d_comp_u || !d_comp_v ||
        !d_comp_out || !ncomp_out || !d_workspace)
        return fail(ctx, EMST_EINVAL, "null pointer");
    if (((uintptr_t)d_workspace & 255u) != 0) return fail(ctx, EMST_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < emst_workspace_bytes(n, dim)) return fail(ctx, EMST_ENOMEM, "workspace too small");
    HIP_TRY(hipSetDevice(ctx->device));
    const bool counting = ctx->counting;
    ctx->counting = false;
    RoundCapture cap{d_bound, d_cand_d, d_cand_j, d_comp_d2, d_comp_u, d_comp_v};
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int rc = dim == 3 ? test_round<3>(ctx, d_points, n, d_comp, round, variant, cap, d_comp_out, ncomp_out,
                                            (char*)d_workspace, st)
                            : test_round<2>(ctx, d_points, n, d_comp, round, variant, cap, d_comp_out, ncomp_out,
                                            (char*)d_workspace, st);
    ctx->counting = counting;
    return rc;
}

extern "C" int emst_test_tree_from_codes(emst_ctx* ctx, const uint64_t* d_codes, int64_t n,
                                         const uint32_t* d_leaf_labels, int32_t* d_left, int32_t* d_right,
                                         uint32_t* d_label, int32_t* root_out, void* d_workspace, size_t ws_bytes,
                                         void* stream) {
    if (!ctx) return EMST_EINVAL;
    ctx->err.clear();
    if (n < 2 || n > 0x7FFFFFFFll || !d_codes || !d_leaf_labels || !d_left || !d_right || !d_label || !root_out ||
        !d_workspace)
        return fail(ctx, EMST_EINVAL, "bad argument");
    if (((uintptr_t)d_workspace & 255u) != 0) return fail(ctx, EMST_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < emst_workspace_bytes(n, 3)) return fail(ctx, EMST_ENOMEM, "workspace too small");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char* ws = (char*)d_workspace;
    const Layout L = make_layout(n, 3);
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
    float* spts = reinterpret_cast<float*>(ws + L.spts);
    uint32_t* orig = reinterpret_cast<uint32_t*>(ws + L.orig);
    uint32_t* labels = reinterpret_cast<uint32_t*>(ws + L.labels);
    uint64_t* exch = reinterpret_cast<uint64_t*>(ws + L.exch);
    uint32_t* rlo = reinterpret_cast<uint32_t*>(ws + L.rlo);
    uint32_t* rhi = reinterpret_cast<uint32_t*>(ws + L.rhi);
    uint32_t* run_part = reinterpret_cast<uint32_t*>(ws + L.run_part);
    uint32_t* run_carry = reinterpret_cast<uint32_t*>(ws + L.run_carry);
    Rec<3>* recs = reinterpret_cast<Rec<3>*>(ws + L.recs);
    uint2* lab2 = reinterpret_cast<uint2*>(ws + L.lab2);
    uint32_t* node_parent = reinterpret_cast<uint32_t*>(ws + L.node_parent);
    uint32_t* leaf_parent = reinterpret_cast<uint32_t*>(ws + L.leaf_parent);
    k_init_ctrl<<<1, 64, 0, st>>>(ctrl);
    k_test_prep<<<grid_for(n), 256, 0, st>>>(d_leaf_labels, n, spts, orig, labels, exch);
    uint8_t* height = reinterpret_cast<uint8_t*>(ws + L.height);
    NodeInfo* info = reinterpret_cast<NodeInfo*>(ws + L.up);
    k_build<3, true><<<grid_for(n), 256, 0, st>>>(d_codes, orig, n, recs, leaf_parent, info, exch, ctrl);
    k_unpack_nodes<<<grid_for(n - 1), 256, 0, st>>>(info, n - 1, rlo, rhi, node_parent, height);
    HIP_TRY(propagate_labels(labels, run_part, run_carry, rlo, rhi, lab2, n, ctrl, st));
    k_test_extract<<<grid_for(n - 1), 256, 0, st>>>(recs, lab2, node_parent, n - 1, d_left, d_right, d_label);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(ctx->h_ctrl, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (ctx->h_ctrl->error || ctx->h_ctrl->root == kNone) return fail(ctx, EMST_EINTERNAL, "tree construction failed");
    *root_out = (int32_t)ctx->h_ctrl->root;
    return EMST_OK;
}

extern "C" int emst_test_radix_sort(emst_ctx* ctx, uint64_t* d_keys, uint32_t* d_vals, int64_t n, void* d_workspace,
                                    size_t ws_bytes, void* stream) {
    if (!ctx) return EMST_EINVAL;
    ctx->err.clear();
    if (n < 0 || n > 0x7FFFFFFFll || (n > 0 && (!d_keys || !d_vals || !d_workspace)))
        return fail(ctx, EMST_EINVAL, "bad argument");
    if (n < 2) return EMST_OK;
    if (((uintptr_t)d_workspace & 255u) != 0) return fail(ctx, EMST_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < emst_workspace_bytes(n, 3)) return fail(ctx, EMST_ENOMEM, "workspace too small");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char* ws = (char*)d_workspace;
    const Layout L = make_layout(n, 3);
    uint64_t* k1 = reinterpret_cast<uint64_t*>(ws + L.k1);
    uint32_t* v1 = reinterpret_cast<uint32_t*>(ws + L.v1);
    uint32_t* hist = reinterpret_cast<uint32_t*>(ws + L.hist);
    int shifts[8];
    for (int q = 0; q < 8; ++q) shifts[q] = 8 * q;
    int in1 = 0;
    HIP_TRY(radix_sort_pairs(st, d_keys, d_vals, k1, v1, hist, n, shifts, 8, &in1));
    if (in1) {
        HIP_TRY(hipMemcpyAsync(d_keys, k1, 8 * (size_t)n, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_vals, v1, 4 * (size_t)n, hipMemcpyDeviceToDevice, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    return EMST_OK;
}

extern "C" int emst_test_tree_boxes(emst_ctx* ctx, const float* d_points, int64_t n, int32_t* d_left,
                                    int32_t* d_right, float* d_lo, float* d_hi, int32_t* root_out, void* d_workspace,
                                    size_t ws_bytes, void* stream) {
    if (!ctx) return EMST_EINVAL;
    ctx->err.clear();
    if (n < 2 || n > 0x7FFFFFFFll || !d_points || !d_left || !d_right || !d_lo || !d_hi || !root_out ||
        !d_workspace)
        return fail(ctx, EMST_EINVAL, "bad argument");
    if (((uintptr_t)d_workspace & 255u) != 0) return fail(ctx, EMST_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < emst_workspace_bytes(n, 3)) return fail(ctx, EMST_ENOMEM, "workspace too small");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char* ws = (char*)d_workspace;
    const Layout L = make_layout(n, 3);
    Bufs<3> b = carve<3>(ws, L);
    k_init_ctrl<<<1, 64, 0, st>>>(b.ctrl);
    HIP_TRY(launch_bbox<3>(d_points, n, b.bpart, b.ctrl, st));
    HIP_TRY(hipGetLastError());
    if (int rc = read_ctrl(ctx, b.ctrl, st)) return rc;
    if (ctx->h_ctrl->nonfinite) return fail(ctx, EMST_ENONFINITE, "non-finite coordinate");
    float lo[3], hi[3];
    for (int k = 0; k < 3; ++k) { lo[k] = ord_dec(ctx->h_ctrl->bb_min[k]); hi[k] = ord_dec(ctx->h_ctrl->bb_max[k]); }
    const MortonParams mp = morton_params(lo, hi, 3, 21);
    k_morton<3><<<std::min<unsigned>(grid_for(n), 1024), 256, 0, st>>>(d_points, n, mp, nullptr, b.k0, b.v0);
    int shifts[8];
    for (int q = 0; q < 8; ++q) shifts[q] = 8 * q;
    int in1 = 0;
    HIP_TRY(radix_sort_pairs(st, b.k0, b.v0, b.k1, b.v1, b.hist, n, shifts, 8, &in1));
    const uint64_t* codes = in1 ? b.k1 : b.k0;
    const uint32_t* perm = in1 ? b.v1 : b.v0;
    k_gather<3><<<grid_for(n), 256, 0, st>>>(d_points, perm, n, b.spts, b.orig, b.labels, b.exch);
    if (int rc = build_tree<3>(ctx, b, codes, n, st)) return rc;
    k_test_boxes<<<grid_for(n - 1), 256, 0, st>>>(b.recs, n - 1, d_left, d_right, d_lo, d_hi);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    *root_out = (int32_t)ctx->h_ctrl->root;
    return EMST_OK;
}
