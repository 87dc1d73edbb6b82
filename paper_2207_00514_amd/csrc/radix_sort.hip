// Stable LSD radix sort of (uint64 key, uint32 value) pairs, 8-bit digits,
// written for gfx950 wave64.
//
// One pass = three launches:
//   upsweep    every block counts the digits of its contiguous chunk of
//              tiles into an LDS histogram (one sub-histogram per wave);
//   rowscan    one block per digit scans that digit's counts across the
//              blocks (exclusive) and records the digit total;
//   downsweep  every block walks its chunk tile by tile; inside a tile the
//              stable rank of each item among equal digits comes from 8
//              wave ballots (lanes with the same digit), per-(slot, wave)
//              digit counts are staged in LDS and prefix-summed per digit,
//              and the tile is staged in LDS in digit order, so every run of
//              equal digits is written by consecutive threads to
//              consecutive addresses (every block first turns the 256
//              digit totals into digit start offsets itself).
// Items are loaded striped (item s of thread t is tile element s*256 + t),
// so the (slot, wave, lane) order equals the input order and the sort is
// stable.
//
// From kRadixOneMin keys on, a pass is instead one launch of rs_onesweep
// (decoupled look-back across tiles, after one count of every digit of
// every pass by rs_global_hist), described below.
#include "radix_sort.h"

namespace emst {

constexpr int kRsThreads = 256;
constexpr int kRsWaves = kRsThreads / 64;
// Items per thread of a tile: 8 for small sorts, 16 (longer runs of equal
// digits per tile, so longer write segments; fewer resident blocks) from
// kRsBigN keys on, where that measures faster.
constexpr int64_t kRsBigN = (int64_t)1 << 23;

template <int ITEMS>
__global__ __launch_bounds__(kRsThreads) void rs_upsweep(const uint64_t* __restrict__ keys, int64_t n,
                                                         int shift, int64_t tiles_per_block,
                                                         uint32_t* __restrict__ hist, int nb) {
    constexpr int kRsTile = kRsThreads * ITEMS;
    __shared__ uint32_t h[kRsWaves][256];
    const int t = threadIdx.x, w = t / 64;
    for (int k = t; k < kRsWaves * 256; k += kRsThreads) (&h[0][0])[k] = 0;
    __syncthreads();
    const int64_t begin = (int64_t)blockIdx.x * tiles_per_block * kRsTile;
    const int64_t end = min(n, begin + tiles_per_block * kRsTile);
    for (int64_t i = begin + t; i < end; i += kRsThreads) {
        uint32_t d = (uint32_t)(keys[i] >> shift) & 255u;
        atomicAdd(&h[w][d], 1u);
    }
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kRsWaves; ++k) s += h[k][t];
    hist[(int64_t)t * nb + blockIdx.x] = s;
}

// Exclusive scan of every digit's row of the count table across the blocks
// (one block per digit, one entry per thread); the row total goes to
// row_total[digit].  Rows have at most kRadixMaxBlocks = 1024 entries.
__global__ __launch_bounds__(1024) void rs_rowscan(uint32_t* __restrict__ hist, int nb,
                                                   uint32_t* __restrict__ row_total) {
    __shared__ uint32_t wsum[16];
    const int d = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
    const uint32_t v = (t < nb) ? hist[(int64_t)d * nb + t] : 0u;
    uint32_t x = v;  // inclusive scan inside the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (t < 16) {
        uint32_t s = wsum[t];
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const uint32_t y = __shfl_up(s, off);
            if (t >= off) s += y;
        }
        wsum[t] = s;
    }
    __syncthreads();
    const uint32_t incl = x + (w > 0 ? wsum[w - 1] : 0u);
    if (t < nb) hist[(int64_t)d * nb + t] = incl - v;
    if (t == 1023) row_total[d] = incl;
}

template <int ITEMS>
__global__ __launch_bounds__(kRsThreads) void rs_downsweep(const uint64_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ vin,
                                                           uint64_t* __restrict__ kout,
                                                           uint32_t* __restrict__ vout, int64_t n, int shift,
                                                           int64_t tiles_per_block,
                                                           const uint32_t* __restrict__ hist, int nb,
                                                           const uint32_t* __restrict__ row_total) {
    constexpr int kRsItems = ITEMS;
    constexpr int kRsTile = kRsThreads * ITEMS;
    __shared__ uint32_t gbase[256];   // running global start of every digit for this block
    __shared__ uint32_t lstart[256];  // tile-local start of every digit
    __shared__ uint32_t wsum[kRsWaves];
    // per-(slot, wave, digit) counts, then offsets; afterwards the same
    // storage stages the tile's keys and values in digit order
    __shared__ __attribute__((aligned(16))) uint32_t cnt[kRsItems][kRsWaves][256];
    static_assert(sizeof(cnt) >= kRsTile * (sizeof(uint64_t) + sizeof(uint32_t)), "staging fits");
    uint64_t* skey = reinterpret_cast<uint64_t*>(&cnt[0][0][0]);
    uint32_t* sval = reinterpret_cast<uint32_t*>(skey + kRsTile);
    const int t = threadIdx.x, w = t / 64, lane = t & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    {
        // global start of digit t = sum of the totals of the smaller digits
        const uint32_t v = row_total[t];
        uint32_t x = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        uint32_t before = 0;
        for (int k = 0; k < w; ++k) before += wsum[k];
        gbase[t] = (x - v) + before + hist[(int64_t)t * nb + blockIdx.x];
    }
    const int64_t first_tile = (int64_t)blockIdx.x * tiles_per_block;
    const int64_t num_tiles = (n + kRsTile - 1) / kRsTile;
    const int64_t last_tile = min(num_tiles, first_tile + tiles_per_block);
    // the next tile's items are loaded while the current one is ranked and
    // scattered
    uint64_t nkey[kRsItems];
    uint32_t nval[kRsItems];
    auto load_tile = [&](int64_t tile) {
        const int64_t tb = tile * kRsTile;
#pragma unroll
        for (int s = 0; s < kRsItems; ++s) {
            const int64_t idx = tb + (int64_t)s * kRsThreads + t;
            const bool in = tile < last_tile && idx < n;
            nkey[s] = in ? kin[idx] : 0ull;
            nval[s] = in ? vin[idx] : 0u;
        }
    };
    load_tile(first_tile);
    for (int64_t tile = first_tile; tile < last_tile; ++tile) {
        for (int k = t; k < kRsItems * kRsWaves * 256; k += kRsThreads) (&cnt[0][0][0])[k] = 0;
        __syncthreads();
        const int64_t tb = tile * kRsTile;
        const int valid = (int)min((int64_t)kRsTile, n - tb);
        uint64_t key[kRsItems];
        uint32_t val[kRsItems], dig[kRsItems], rank[kRsItems];
        bool ok[kRsItems];
#pragma unroll
        for (int s = 0; s < kRsItems; ++s) {
            const int64_t idx = tb + (int64_t)s * kRsThreads + t;
            ok[s] = idx < n;
            key[s] = nkey[s];
            val[s] = nval[s];
            dig[s] = (uint32_t)(key[s] >> shift) & 255u;
        }
        load_tile(tile + 1);
#pragma unroll
        for (int s = 0; s < kRsItems; ++s) {
            uint64_t peers = __ballot(ok[s]);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (dig[s] >> b) & 1u;
                const uint64_t m = __ballot(bit);
                peers &= bit ? m : ~m;
            }
            rank[s] = (uint32_t)__popcll(peers & lt_mask);
            if (ok[s] && rank[s] == 0) cnt[s][w][dig[s]] = (uint32_t)__popcll(peers);
        }
        __syncthreads();
        // per digit: offsets of every (slot, wave) group inside the digit,
        // and the digit's tile total
        uint32_t total;
        {
            uint32_t off = 0;
#pragma unroll
            for (int s = 0; s < kRsItems; ++s)
#pragma unroll
                for (int ww = 0; ww < kRsWaves; ++ww) {
                    const uint32_t c = cnt[s][ww][t];
                    cnt[s][ww][t] = off;
                    off += c;
                }
            total = off;
            // tile-local start of digit t: exclusive scan of the totals
            uint32_t x = total;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(x, o);
                if (lane >= o) x += y;
            }
            if (lane == 63) wsum[w] = x;
            __syncthreads();
            uint32_t before = 0;
            for (int k = 0; k < w; ++k) before += wsum[k];
            lstart[t] = x - total + before;
        }
        __syncthreads();
        uint32_t lpos[kRsItems];
#pragma unroll
        for (int s = 0; s < kRsItems; ++s)
            lpos[s] = ok[s] ? lstart[dig[s]] + cnt[s][w][dig[s]] + rank[s] : 0u;
        __syncthreads();  // cnt is reused for staging from here on
#pragma unroll
        for (int s = 0; s < kRsItems; ++s) {
            if (ok[s]) {
                skey[lpos[s]] = key[s];
                sval[lpos[s]] = val[s];
            }
        }
        __syncthreads();
        // consecutive threads write consecutive positions of each digit run
#pragma unroll
        for (int s = 0; s < kRsItems; ++s) {
            const int lp = s * kRsThreads + t;
            if (lp < valid) {
                const uint64_t k = skey[lp];
                const uint32_t d = (uint32_t)(k >> shift) & 255u;
                const uint32_t dst = gbase[d] + (uint32_t)lp - lstart[d];
                kout[dst] = k;
                vout[dst] = sval[lp];
            }
        }
        __syncthreads();
        gbase[t] += total;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// One-sweep passes (decoupled look-back, Merrill & Garland; its use for LSD
// radix sort by Adinets & Merrill): one global count of every digit of every
// pass first, then per pass a single launch in which each workgroup takes
// the next tile (in launch order, from a counter), ranks it, publishes its
// per-digit counts, and adds up the counts of the tiles before it -- each
// tile publishes its own count before it looks back, and the inclusive
// prefix once it knows it, so a look-back stops at the first inclusive
// prefix it meets and only ever waits on tiles that have started.
// A status word is (flag << 30) | count: flag 1 = the tile's own count,
// 2 = inclusive prefix (counts stay below 2^30: kRadixOneMin <= n < 2^30).
// The words go through device-coherent atomics; each one holds its datum.

constexpr uint32_t kOsAgg = 1u << 30, kOsIncl = 2u << 30, kOsMask = (1u << 30) - 1u;
// predecessor status words a look-back step loads at once
constexpr int kOsWindow = 8;

struct RsShifts {
    int s[8];
};

__global__ __launch_bounds__(kRsThreads) void rs_fill(uint32_t* __restrict__ p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ghist[q][d] += occurrences of digit d at shift q among the keys.
__global__ __launch_bounds__(kRsThreads) void rs_global_hist(const uint64_t* __restrict__ keys, int64_t n,
                                                             RsShifts sh, int np, uint32_t* __restrict__ ghist) {
    __shared__ uint32_t h[kRsWaves][8][256];
    const int t = threadIdx.x, w = t / 64;
    for (int k = t; k < kRsWaves * 8 * 256; k += kRsThreads) (&h[0][0][0])[k] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + t; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[i];
        for (int q = 0; q < np; ++q) atomicAdd(&h[w][q][(uint32_t)(k >> sh.s[q]) & 255u], 1u);
    }
    __syncthreads();
    for (int k = t; k < np * 256; k += kRsThreads) {
        uint32_t c = 0;
#pragma unroll
        for (int v = 0; v < kRsWaves; ++v) c += (&h[v][0][0])[k];
        if (c) atomicAdd(&ghist[k], c);
    }
}

// gstart[q][d] = digits below d at shift q (one workgroup per shift).
__global__ __launch_bounds__(kRsThreads) void rs_global_scan(const uint32_t* __restrict__ ghist,
                                                             uint32_t* __restrict__ gstart) {
    __shared__ uint32_t wsum[kRsWaves];
    const int t = threadIdx.x, w = t / 64, lane = t & 63;
    const uint32_t v = ghist[blockIdx.x * 256 + t];
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < w; ++k) before += wsum[k];
    gstart[blockIdx.x * 256 + t] = x - v + before;
}

__device__ __forceinline__ uint32_t os_load(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void os_store(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Each wave owns a contiguous chunk of 64 x ITEMS keys of the tile (item s
// of lane l is key s * 64 + l of the chunk), so the tile's order is (wave,
// item, lane) and one running count per wave and digit ranks it stably: the
// lanes of an item read their digit's count, and the first lane of each
// digit adds the item's peers (a wave's LDS operations complete in order).
// The first 256 threads then own one digit each for the scans and the
// look-back.  Keys, then values, go through LDS in the sorted order so that
// the stores of a digit's run are contiguous.  At most 80 registers keep
// six waves per SIMD (three 512-thread workgroups per compute unit, which
// their 35 KB of LDS allows too).
template <int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(6))) void rs_onesweep(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ vout, int64_t n, int shift, const uint32_t* __restrict__ gstart, uint32_t* status,
    uint32_t* status_next, uint32_t* counter, uint32_t* err) {
    constexpr int kWaves = THREADS / 64;
    constexpr int kTile = THREADS * ITEMS;
    static_assert(THREADS >= 256 && THREADS % 64 == 0, "one digit per thread of the first 256");
    __shared__ uint32_t s_tile;
    __shared__ uint32_t gbase[256];   // global start of every digit for this tile
    __shared__ uint32_t lstart[256];  // tile-local start of every digit
    __shared__ uint32_t wsum[4];
    __shared__ __attribute__((aligned(16))) uint64_t stage[kTile];
    static_assert(sizeof(stage) >= kWaves * 256 * sizeof(uint32_t), "the wave counts fit");
    uint32_t* cnt = reinterpret_cast<uint32_t*>(stage);  // [wave][digit] until the staging
    uint32_t* sval = cnt;
    const int t = threadIdx.x, w = t / 64, lane = t & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (t == 0) s_tile = atomicAdd(counter, 1u);
    for (int k = t; k < kWaves * 256; k += THREADS) cnt[k] = 0;
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t tb = tile * kTile;
    const int valid = (int)min((int64_t)kTile, n - tb);
    uint64_t key[ITEMS];
    uint32_t val[ITEMS], rank[ITEMS];
    bool ok[ITEMS];
    // (a key's digit is recomputed where needed: fewer live registers)
    auto digit = [&](uint64_t k) { return (uint32_t)(k >> shift) & 255u; };
#pragma unroll
    for (int s = 0; s < ITEMS; ++s) {
        const int64_t idx = tb + (int64_t)(w * ITEMS + s) * 64 + lane;
        ok[s] = idx < n;
        key[s] = ok[s] ? kin[idx] : 0ull;
        val[s] = ok[s] ? vin[idx] : 0u;
    }
    uint32_t* wcnt = cnt + w * 256;
#pragma unroll
    for (int s = 0; s < ITEMS; ++s) {
        const uint32_t dg = digit(key[s]);
        uint64_t peers = __ballot(ok[s]);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dg >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t r = (uint32_t)__popcll(peers & lt_mask);
        const uint32_t before = ok[s] ? wcnt[dg] : 0u;
        rank[s] = before + r;
        if (ok[s] && r == 0) wcnt[dg] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    uint32_t total = 0, x = 0;
    if (t < 256) {
        uint32_t off = 0;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) {
            const uint32_t c = cnt[ww * 256 + t];
            cnt[ww * 256 + t] = off;
            off += c;
        }
        total = off;
        x = total;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[w] = x;
    }
    __syncthreads();
    if (t < 256) {
        uint32_t before = 0;
        for (int k = 0; k < w; ++k) before += wsum[k];
        lstart[t] = x - total + before;
        // digit t: publish this tile's count, add up the tiles before it
        uint32_t excl = 0;
        if (tile == 0) {
            os_store(&status[t], kOsIncl | total);
        } else {
            os_store(&status[tile * 256 + t], kOsAgg | total);
            // the status words of kOsWindow tiles before are loaded at once,
            // then added up nearest first until an inclusive one
            bool found = false;
            for (int64_t p = tile - 1; !found; p -= kOsWindow) {
                uint32_t v[kOsWindow];
#pragma unroll
                for (int j = 0; j < kOsWindow; ++j) v[j] = p - j >= 0 ? os_load(&status[(p - j) * 256 + t]) : kOsIncl;
#pragma unroll
                for (int j = 0; j < kOsWindow; ++j) {
                    if (found) break;
                    for (uint32_t spin = 0; (v[j] >> 30) == 0u; ++spin) {
                        if (spin > (1u << 22)) {  // (bounded: a missing tile is a bug, not a wait)
                            atomicOr(err, 1u);
                            v[j] = kOsIncl;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                        v[j] = os_load(&status[(p - j) * 256 + t]);
                    }
                    excl += v[j] & kOsMask;
                    found = (v[j] >> 30) == 2u;
                }
            }
            os_store(&status[tile * 256 + t], kOsIncl | (excl + total));
        }
        gbase[t] = gstart[t] + excl;
        os_store(&status_next[tile * 256 + t], 0u);  // the next pass's status starts empty
    }
    __syncthreads();
    uint32_t lpos[ITEMS];
#pragma unroll
    for (int s = 0; s < ITEMS; ++s) {
        const uint32_t dg = digit(key[s]);
        lpos[s] = ok[s] ? lstart[dg] + wcnt[dg] + rank[s] : 0u;
    }
    __syncthreads();  // the counts are overwritten by the staging from here on
#pragma unroll
    for (int s = 0; s < ITEMS; ++s)
        if (ok[s]) stage[lpos[s]] = key[s];
    __syncthreads();
    uint32_t dst[ITEMS];
#pragma unroll
    for (int s = 0; s < ITEMS; ++s) {
        const int lp = s * THREADS + t;
        dst[s] = 0u;
        if (lp < valid) {
            const uint64_t k = stage[lp];
            const uint32_t d = digit(k);
            dst[s] = gbase[d] + (uint32_t)lp - lstart[d];
            kout[dst[s]] = k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < ITEMS; ++s)
        if (ok[s]) sval[lpos[s]] = val[s];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < ITEMS; ++s) {
        const int lp = s * THREADS + t;
        if (lp < valid) vout[dst[s]] = sval[lp];
    }
}

// Threads and items per thread of a one-sweep tile (kRadixOneTile keys).
constexpr int kOsThreads = 512;
constexpr int kOsItems = kRadixOneTile / kOsThreads;

static int rs_items(int64_t n) { return n >= kRsBigN ? 16 : 8; }

RadixPlan radix_plan(int64_t n) {
    RadixPlan p;
    const int64_t tile = (int64_t)kRsThreads * rs_items(n);
    const int64_t tiles = (n + tile - 1) / tile;
    p.blocks = (int)std::min<int64_t>(std::max<int64_t>(tiles, 1), kRadixMaxBlocks);
    p.tiles_per_block = (tiles + p.blocks - 1) / p.blocks;
    if (p.tiles_per_block < 1) p.tiles_per_block = 1;
    return p;
}

template <int ITEMS>
static void rs_pass(hipStream_t stream, const RadixPlan& p, const uint64_t* ka, const uint32_t* va, uint64_t* kb,
                    uint32_t* vb, uint32_t* hist, int64_t n, int shift) {
    rs_upsweep<ITEMS><<<p.blocks, kRsThreads, 0, stream>>>(ka, n, shift, p.tiles_per_block, hist, p.blocks);
    rs_rowscan<<<256, 1024, 0, stream>>>(hist, p.blocks, hist + 256 * kRadixMaxBlocks);
    rs_downsweep<ITEMS><<<p.blocks, kRsThreads, 0, stream>>>(ka, va, kb, vb, n, shift, p.tiles_per_block, hist,
                                                             p.blocks, hist + 256 * kRadixMaxBlocks);
}

hipError_t radix_sort_pairs(hipStream_t stream, uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1,
                            uint32_t* hist, int64_t n, const int* shifts, int nshifts, int* result_in_1) {
    *result_in_1 = 0;
    if (n <= 1 || nshifts == 0) return hipSuccess;
    uint64_t *ka = k0, *kb = k1;
    uint32_t *va = v0, *vb = v1;
    if (n >= kRadixOneMin && n < ((int64_t)1 << 30) && nshifts <= 8) {
        // scratch after the count table: global counts, global starts, the
        // pass counters and an error word, two status arrays
        const int64_t tiles = (n + kRadixOneTile - 1) / kRadixOneTile;
        uint32_t* base = hist + radix_hist_elems();
        uint32_t* ghist = base;
        uint32_t* gstart = base + 8 * 256;
        uint32_t* counters = base + 3 * 8 * 256;  // [8] pass counters, [9] error
        uint32_t* status[2] = {counters + 64, counters + 64 + tiles * 256};
        RsShifts sh;
        for (int q = 0; q < 8; ++q) sh.s[q] = q < nshifts ? shifts[q] : 0;
        rs_fill<<<1, kRsThreads, 0, stream>>>(ghist, 8 * 256);
        rs_fill<<<1, kRsThreads, 0, stream>>>(counters, 64);
        rs_fill<<<(unsigned)std::min<int64_t>((tiles * 256 + kRsThreads - 1) / kRsThreads, 1024), kRsThreads, 0,
                  stream>>>(status[0], tiles * 256);
        rs_global_hist<<<(unsigned)std::min<int64_t>(tiles, 1024), kRsThreads, 0, stream>>>(ka, n, sh, nshifts,
                                                                                             ghist);
        rs_global_scan<<<nshifts, kRsThreads, 0, stream>>>(ghist, gstart);
        for (int q = 0; q < nshifts; ++q) {
            rs_onesweep<kOsThreads, kOsItems><<<(unsigned)tiles, kOsThreads, 0, stream>>>(
                ka, va, kb, vb, n, shifts[q], gstart + q * 256, status[q & 1], status[(q + 1) & 1], counters + q,
                counters + 8);
            std::swap(ka, kb);
            std::swap(va, vb);
        }
        *result_in_1 = (nshifts & 1);
        return hipGetLastError();
    }
    const RadixPlan p = radix_plan(n);
    for (int q = 0; q < nshifts; ++q) {
        if (rs_items(n) == 16) rs_pass<16>(stream, p, ka, va, kb, vb, hist, n, shifts[q]);
        else rs_pass<8>(stream, p, ka, va, kb, vb, hist, n, shifts[q]);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    *result_in_1 = (nshifts & 1);
    return hipGetLastError();
}

}  // namespace emst
