// Device-side building blocks shared by the EMST kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace emst {

constexpr uint32_t kLeafFlag = 0x80000000u;   // child ref: leaf (low 31 bits = original index)
constexpr uint32_t kInvalid = 0xFFFFFFFFu;    // label of a subtree that spans several components
constexpr uint32_t kNone = 0xFFFFFFFFu;       // "no candidate" / "no parent"
constexpr uint32_t kInfBits = 0x7F800000u;    // +inf as float32 bits
constexpr uint64_t kKeyMax = ~0ull;
constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Node record of the binary LBVH.  One record per internal node holds
// everything a traversal needs about BOTH children, so testing the two
// children of a node is one contiguous read: per child its bounding box and
// its reference (internal node index, or kLeafFlag | original point index).
// With one point per leaf a leaf child's box is the point itself.  The
// component labels of the children change every round and live in a
// separate 8-byte entry per record; the record's label slots stay unused.
//
//   3D, 64 B:  child c at [32c, 32c+32): float4(lo.x, lo.y, lo.z, unused)
//                                        float4(hi.x, hi.y, hi.z, ref)
//   2D, 48 B:  float4(lo0.x, lo0.y, hi0.x, hi0.y)
//              float4(lo1.x, lo1.y, hi1.x, hi1.y)
//              uint4 (unused, ref0, unused, ref1)
template <int DIM> struct Rec;

template <> struct alignas(64) Rec<3> {
    float4 a0, b0, a1, b1;
};
template <> struct alignas(16) Rec<2> {
    float4 box0, box1;
    uint4 meta;
};

static_assert(sizeof(Rec<3>) == 64, "3D record is 64 bytes");
static_assert(sizeof(Rec<2>) == 48, "2D record is 48 bytes");

// Upward-walk metadata of an internal node (32 B): the node's Morton cell
// shrunk by a safety margin (every point whose coordinates lie inside it is
// a leaf of the node; an empty cell, lo = +inf, for nodes that split equal
// codes by index), and the link to its parent ((parent << 1) | side, or
// kNone at the root).
struct alignas(16) Up {
    float4 a;  // cell lo x, y, z, parent link (bits)
    float4 b;  // cell hi x, y, z, unused
};

template <int DIM> struct Child {
    float lo[DIM], hi[DIM];
    uint32_t lab, ref;  // label (from the per-round entry), reference
};

__device__ __forceinline__ uint32_t fbits(float f) { return __float_as_uint(f); }
__device__ __forceinline__ float bitsf(uint32_t u) { return __uint_as_float(u); }

template <int DIM>
__device__ __forceinline__ void unpack(const Rec<DIM>& r, Child<DIM>& c0, Child<DIM>& c1);

template <>
__device__ __forceinline__ void unpack<3>(const Rec<3>& r, Child<3>& c0, Child<3>& c1) {
    c0.lo[0] = r.a0.x; c0.lo[1] = r.a0.y; c0.lo[2] = r.a0.z; c0.lab = kInvalid;
    c0.hi[0] = r.b0.x; c0.hi[1] = r.b0.y; c0.hi[2] = r.b0.z; c0.ref = fbits(r.b0.w);
    c1.lo[0] = r.a1.x; c1.lo[1] = r.a1.y; c1.lo[2] = r.a1.z; c1.lab = kInvalid;
    c1.hi[0] = r.b1.x; c1.hi[1] = r.b1.y; c1.hi[2] = r.b1.z; c1.ref = fbits(r.b1.w);
}

template <>
__device__ __forceinline__ void unpack<2>(const Rec<2>& r, Child<2>& c0, Child<2>& c1) {
    c0.lo[0] = r.box0.x; c0.lo[1] = r.box0.y; c0.hi[0] = r.box0.z; c0.hi[1] = r.box0.w;
    c1.lo[0] = r.box1.x; c1.lo[1] = r.box1.y; c1.hi[0] = r.box1.z; c1.hi[1] = r.box1.w;
    c0.lab = kInvalid; c0.ref = r.meta.y; c1.lab = kInvalid; c1.ref = r.meta.w;
}

// Write the reference of child `side` of record r.
template <int DIM>
__device__ __forceinline__ void set_child_ref(Rec<DIM>* r, int side, uint32_t ref) {
    if (DIM == 3) reinterpret_cast<uint32_t*>(r)[8 * side + 7] = ref;
    else reinterpret_cast<uint32_t*>(r)[8 + 2 * side + 1] = ref;
}

// Box and reference of child `side` in one go (3D: the whole 32-byte half
// of the record, two 16-byte stores).
template <int DIM>
__device__ __forceinline__ void set_child(Rec<DIM>* r, int side, const float* lo, const float* hi, uint32_t ref) {
    if constexpr (DIM == 3) {
        float4* f = reinterpret_cast<float4*>(r) + 2 * side;
        f[0] = make_float4(lo[0], lo[1], lo[2], 0.f);
        f[1] = make_float4(hi[0], hi[1], hi[2], __uint_as_float(ref));
    } else {
        reinterpret_cast<float4*>(r)[side] = make_float4(lo[0], lo[1], hi[0], hi[1]);
        reinterpret_cast<uint32_t*>(r)[8 + 2 * side + 1] = ref;
    }
}

// ---------------------------------------------------------------------------
// Distances.  The float32 squared distance D is evaluated in one fixed
// order -- d = a0 - b0; s = d*d; then s = s + (ak - bk)^2 for k = 1.. --
// with every step rounded separately (no contraction into FMA).  The box
// distance uses the same order on the per-coordinate gap
// g = max(lo - p, 0, p - hi); rounding is monotone, so it never exceeds D(p, q)
// for a q inside the box, and for a degenerate box (a leaf, lo = hi = q) it
// equals D(p, q) bit for bit because |fl(q - p)| = |fl(p - q)|.

#pragma clang fp contract(off)

template <int DIM>
__device__ __forceinline__ float sqdist(const float* a, const float* b) {
    float d = a[0] - b[0];
    float s = d * d;
#pragma unroll
    for (int k = 1; k < DIM; ++k) {
        d = a[k] - b[k];
        s = s + d * d;
    }
    return s;
}

template <int DIM>
__device__ __forceinline__ float boxdist(const float* p, const float* lo, const float* hi) {
    float g = fmaxf(fmaxf(lo[0] - p[0], p[0] - hi[0]), 0.0f);
    float s = g * g;
#pragma unroll
    for (int k = 1; k < DIM; ++k) {
        g = fmaxf(fmaxf(lo[k] - p[k], p[k] - hi[k]), 0.0f);
        s = s + g * g;
    }
    return s;
}

// The reported weight of an edge of squared length d2: its square root,
// correctly rounded (the library is built with correctly rounded float32
// square roots).
__device__ __forceinline__ float edge_weight(float d2) { return sqrtf(d2); }

// ---------------------------------------------------------------------------
// atomics with explicit scope / ordering

__device__ __forceinline__ uint32_t load_relaxed(const uint32_t* p) {
    return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t load_relaxed64(const uint64_t* p) {
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// gfx950 hands workgroups to its 8 XCDs round-robin (workgroup w runs on
// XCD w % 8), and every XCD has its own L2.  For a grid whose size is a
// multiple of 8 this maps the hardware workgroup id to a logical one so
// that each XCD sweeps one contiguous eighth of the logical range: queries
// that are neighbours in Morton order then share one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t hw, int64_t grid) {
    const int64_t per = grid / kXcds;
    return (hw % kXcds) * per + hw / kXcds;
}

// Segmented inclusive min-scan over the lanes of a wave, segments = runs of
// equal `lab` in lane order.  Lanes only ever combine values carrying the
// same label, and the last lane of a run ends up with the minimum of the
// whole run; *run_end tells whether this lane is that last lane.  Every lane
// of the wave must call it.
template <typename T>
__device__ __forceinline__ T wave_seg_min(uint32_t lab, T v, bool* run_end) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t ol = __shfl_up(lab, off);
        const T ov = __shfl_up(v, off);
        if (lane >= off && ol == lab && ov < v) v = ov;
    }
    const uint32_t next = __shfl_down(lab, 1);
    *run_end = (lane == 63) || (next != lab);
    return v;
}

}  // namespace emst
