/*
 * CPU oracle for the Euclidean minimum spanning tree (EMST).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code with the HIP implementation.
 *
 * What it computes (Section 2, "EMST computation" and "MST computation";
 * tie-breaking rule of Section 2, "Boruvka's algorithm"):
 *
 *   The EMST is the MST of the complete distance graph of the points.  The
 *   weight of a pair (u, v), u != v, is ordered by the key
 *
 *       K(u, v) = ( bits(D(u, v)), min(u, v), max(u, v) )
 *
 *   compared lexicographically, where D is the float32 squared distance
 *   evaluated in one fixed order (dx = a0 - b0; s = dx*dx; then for every
 *   further coordinate dk = ak - bk; s = s + dk*dk), IEEE round-to-nearest,
 *   no fused multiply-add, denormals kept.  For non-negative finite floats
 *   the unsigned bit pattern orders like the value, and D >= +0 always.  K is
 *   a strict total order, so the MST under K is unique; Prim, Kruskal and
 *   Boruvka all reach it.  The paper orders equal-weight edges by
 *   (min index, max index); K applies that rule to the float32 squared
 *   distance, and sqrtf is monotone, so it also orders the reported
 *   weights sqrtf(D).
 *
 * Functions:
 *   oracle_sqdist       D for one pair (oracle_sqdist_pairs: for many)
 *   oracle_weights      the reported weight sqrtf(D), correctly rounded
 *   oracle_prim         dense O(n^2) Prim (Section 2, Prim's algorithm)
 *   oracle_kdboruvka    Boruvka (Algorithm 1) over a kd-tree nearest
 *                       other-component search, with subtree skipping
 *                       (Section 3, Optimization 1) and a per-component
 *                       bound shared by all points of a component (the
 *                       "extreme case" of Section 3, Optimization 2)
 *   oracle_canonicalize sort edges by K, weights = sqrtf(D)
 *
 * Mutual reachability (Section 4, "Mutual reachability distance"; Section 3,
 * "Non-Euclidean metrics"): the core distance of u is the distance to its
 * k_pts-th nearest neighbour counting u itself, and the mutual reachability
 * of u and v is the largest of core(u), core(v) and |u - v|.  Squaring is
 * monotone on non-negative values, so in squared terms
 *
 *       M(u, v) = max(core2(u), core2(v), D(u, v)),   core2 = squared core,
 *
 * and the tree is the MST under (bits(M), min, max).  With k_pts = 1 every
 * core distance is 0 (the point itself) and M = D.
 *   oracle_core_brute   core2 by sorting all n values D(u, .) per point
 *   oracle_core_kd      core2 by a kd-tree k-nearest search
 *   oracle_prim_mreach, oracle_kdboruvka_mreach
 *                       the two MST routines above under M (core2 given);
 *                       the kd-tree search still prunes by the Euclidean
 *                       box distance, a lower bound of M
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -fPIC -shared
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <xmmintrin.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* floating-point environment: keep denormals (clear FTZ bit 15, DAZ bit 6)  */

static unsigned int fp_enter(void) {
    unsigned int old = _mm_getcsr();
    _mm_setcsr(old & ~((1u << 15) | (1u << 6)));
    return old;
}
static void fp_leave(unsigned int old) { _mm_setcsr(old); }

static inline uint32_t fbits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static inline float bitsf(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

/* D: squared distance in the fixed order. */
static float sqdist(const float *a, const float *b, int dim) {
    float d = a[0] - b[0];
    float s = d * d;
    for (int k = 1; k < dim; ++k) {
        d = a[k] - b[k];
        s = s + d * d;
    }
    return s;
}

float oracle_sqdist(const float *a, const float *b, int dim) {
    unsigned int csr = fp_enter();
    float s = sqdist(a, b, dim);
    fp_leave(csr);
    return s;
}

/* D of m pairs: out[i] = D(a + i*dim, b + i*dim). */
void oracle_sqdist_pairs(const float *a, const float *b, int64_t m, int dim, float *out) {
    unsigned int csr = fp_enter();
    for (int64_t i = 0; i < m; ++i) out[i] = sqdist(a + i * dim, b + i * dim, dim);
    fp_leave(csr);
}

/* The reported weight of an edge: w[i] = sqrtf(d2[i]), IEEE correctly
 * rounded. */
void oracle_weights(const float *d2, int64_t m, float *w) {
    unsigned int csr = fp_enter();
    for (int64_t i = 0; i < m; ++i) w[i] = sqrtf(d2[i]);
    fp_leave(csr);
}

/* ------------------------------------------------------------------------ */
/* the key K                                                                 */

typedef struct { uint32_t w, u, v; } okey;   /* w = bits of D, u < v */

static const okey KEY_INF = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};

static inline int key_lt(okey a, okey b) {
    if (a.w != b.w) return a.w < b.w;
    if (a.u != b.u) return a.u < b.u;
    return a.v < b.v;
}

/* core2 == NULL: the key of D; else the key of M (all values are
 * non-negative, so comparing them as floats is comparing their bits). */
static inline okey make_key(const float *pts, int dim, const float *core2, int64_t i, int64_t j) {
    okey k;
    float w = sqdist(pts + i * dim, pts + j * dim, dim);
    if (core2) {
        if (core2[i] > w) w = core2[i];
        if (core2[j] > w) w = core2[j];
    }
    k.w = fbits(w);
    k.u = (uint32_t)(i < j ? i : j);
    k.v = (uint32_t)(i < j ? j : i);
    return k;
}

/* ------------------------------------------------------------------------ */
/* dense Prim: the tree grows from vertex 0; every step adds the outside
 * vertex whose cheapest connection to the tree is smallest under K.        */

static int prim_impl(const float *pts, int64_t n, int dim, const float *core2, int32_t *edges, float *d2) {
    if (n < 2) return 0;
    if (dim < 1) return -1;
    unsigned int csr = fp_enter();
    okey *best = (okey *)malloc((size_t)n * sizeof(okey));
    unsigned char *in_tree = (unsigned char *)calloc((size_t)n, 1);
    if (!best || !in_tree) { free(best); free(in_tree); fp_leave(csr); return -4; }
    in_tree[0] = 1;
    for (int64_t v = 1; v < n; ++v) best[v] = make_key(pts, dim, core2, 0, v);
    for (int64_t step = 0; step + 1 < n; ++step) {
        int64_t pick = -1;
        for (int64_t v = 0; v < n; ++v)
            if (!in_tree[v] && (pick < 0 || key_lt(best[v], best[pick]))) pick = v;
        okey e = best[pick];
        edges[2 * step] = (int32_t)e.u;
        edges[2 * step + 1] = (int32_t)e.v;
        d2[step] = bitsf(e.w);
        in_tree[pick] = 1;
        for (int64_t w = 0; w < n; ++w) {
            if (in_tree[w]) continue;
            okey k = make_key(pts, dim, core2, pick, w);
            if (key_lt(k, best[w])) best[w] = k;
        }
    }
    free(best);
    free(in_tree);
    fp_leave(csr);
    return 0;
}

int oracle_prim(const float *pts, int64_t n, int dim, int32_t *edges, float *d2) {
    return prim_impl(pts, n, dim, NULL, edges, d2);
}

int oracle_prim_mreach(const float *pts, int64_t n, int dim, const float *core2, int32_t *edges, float *d2) {
    return prim_impl(pts, n, dim, core2, edges, d2);
}

/* ------------------------------------------------------------------------ */
/* kd-tree                                                                   */

#define KD_LEAF 16
#define MIXED 0xFFFFFFFFu
#define KD_STACK 256

typedef struct {
    float lo[3], hi[3];
    int64_t begin, end;      /* range in idx[] */
    int32_t left, right;     /* child node ids, -1 for a leaf */
} kdnode;

typedef struct {
    const float *pts;
    int dim;
    int32_t *idx;
    kdnode *nodes;
    int64_t n_nodes, cap;
} kdtree;

static float coord(const kdtree *t, int32_t i, int ax) { return t->pts[(int64_t)i * t->dim + ax]; }

/* Put the k-th smallest (by coordinate ax) of idx[lo, hi) at position k,
 * smaller-or-equal ones before it and greater-or-equal ones after it
 * (quickselect with three-way partitioning, so duplicates cost nothing). */
static void select_kth(kdtree *t, int64_t lo, int64_t hi, int64_t k, int ax) {
    int32_t *a = t->idx;
    while (hi - lo > 1) {
        float x0 = coord(t, a[lo], ax), x1 = coord(t, a[lo + (hi - lo) / 2], ax), x2 = coord(t, a[hi - 1], ax);
        float piv = (x0 < x1) ? ((x1 < x2) ? x1 : (x0 < x2 ? x2 : x0)) : ((x0 < x2) ? x0 : (x1 < x2 ? x2 : x1));
        int64_t lt = lo, i = lo, gt = hi;   /* [lo,lt) < piv, [lt,i) == piv, [gt,hi) > piv */
        while (i < gt) {
            float x = coord(t, a[i], ax);
            if (x < piv) { int32_t tmp = a[lt]; a[lt] = a[i]; a[i] = tmp; ++lt; ++i; }
            else if (x > piv) { --gt; int32_t tmp = a[gt]; a[gt] = a[i]; a[i] = tmp; }
            else ++i;
        }
        if (k < lt) hi = lt;
        else if (k >= gt) lo = gt;
        else return;
    }
}

static int32_t kd_new_node(kdtree *t) {
    if (t->n_nodes == t->cap) {
        int64_t nc = t->cap ? 2 * t->cap : 1024;
        kdnode *nn = (kdnode *)realloc(t->nodes, (size_t)nc * sizeof(kdnode));
        if (!nn) return -1;
        t->nodes = nn;
        t->cap = nc;
    }
    return (int32_t)t->n_nodes++;
}

static int kd_build(kdtree *t, int64_t n) {
    /* explicit work stack of node ids; each node's box is the exact min/max
     * of its points, its split is the median along the widest box side */
    int32_t root = kd_new_node(t);
    if (root < 0) return -4;
    t->nodes[root].begin = 0;
    t->nodes[root].end = n;
    int64_t sp = 0, scap = 256;
    int32_t *stack = (int32_t *)malloc((size_t)scap * sizeof(int32_t));
    if (!stack) return -4;
    stack[sp++] = root;
    while (sp > 0) {
        int32_t id = stack[--sp];
        kdnode nd = t->nodes[id];
        for (int k = 0; k < 3; ++k) { nd.lo[k] = 0.0f; nd.hi[k] = 0.0f; }
        for (int k = 0; k < t->dim; ++k) { nd.lo[k] = INFINITY; nd.hi[k] = -INFINITY; }
        for (int64_t q = nd.begin; q < nd.end; ++q)
            for (int k = 0; k < t->dim; ++k) {
                float x = coord(t, t->idx[q], k);
                if (x < nd.lo[k]) nd.lo[k] = x;
                if (x > nd.hi[k]) nd.hi[k] = x;
            }
        nd.left = nd.right = -1;
        int64_t cnt = nd.end - nd.begin;
        if (cnt > KD_LEAF) {
            int ax = 0;
            for (int k = 1; k < t->dim; ++k)
                if (nd.hi[k] - nd.lo[k] > nd.hi[ax] - nd.lo[ax]) ax = k;
            int64_t mid = nd.begin + cnt / 2;
            select_kth(t, nd.begin, nd.end, mid, ax);
            int32_t l = kd_new_node(t), r = kd_new_node(t);
            if (l < 0 || r < 0) { free(stack); return -4; }
            t->nodes[l].begin = nd.begin; t->nodes[l].end = mid;
            t->nodes[r].begin = mid;      t->nodes[r].end = nd.end;
            nd.left = l; nd.right = r;
            if (sp + 2 > scap) {
                scap *= 2;
                int32_t *ns = (int32_t *)realloc(stack, (size_t)scap * sizeof(int32_t));
                if (!ns) { free(stack); return -4; }
                stack = ns;
            }
            stack[sp++] = l;
            stack[sp++] = r;
        }
        t->nodes[id] = nd;
    }
    free(stack);
    return 0;
}

/* Lower bound of D(p, q) over q in the box: per-coordinate gap
 * t = lo - p below the box, p - hi above it, 0 inside; then the same
 * square-and-sum order as D.  Rounding is monotone, so this never exceeds
 * D(p, q) for any q in the box. */
static float boxdist(const float *p, const kdnode *nd, int dim) {
    float s = 0.0f;
    for (int k = 0; k < dim; ++k) {
        float g;
        if (p[k] < nd->lo[k]) g = nd->lo[k] - p[k];
        else if (p[k] > nd->hi[k]) g = p[k] - nd->hi[k];
        else g = 0.0f;
        if (k == 0) s = g * g;
        else s = s + g * g;
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* union-find (path halving)                                                 */

static int64_t uf_find(int64_t *par, int64_t x) {
    while (par[x] != x) { par[x] = par[par[x]]; x = par[x]; }
    return x;
}

/* ------------------------------------------------------------------------ */
/* nearest other-component search for one point, sharing the component's
 * running best key (Algorithm 2 with the bound updated at every leaf).     */

static void query_point(const kdtree *t, const float *core2, const uint32_t *lab, const uint32_t *node_comp,
                        int64_t i, okey *best, int32_t *stack) {
    const int dim = t->dim;
    const float *p = t->pts + i * dim;
    const uint32_t c = lab[i];
    int64_t sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        int32_t id = stack[--sp];
        const kdnode *nd = &t->nodes[id];
        if (node_comp[id] == c) continue;                   /* subtree skipping */
        if (best->w != 0xFFFFFFFFu && boxdist(p, nd, dim) > bitsf(best->w)) continue;
        if (nd->left < 0) {
            for (int64_t q = nd->begin; q < nd->end; ++q) {
                int32_t j = t->idx[q];
                if (lab[j] == c) continue;
                okey k = make_key(t->pts, dim, core2, i, j);
                if (key_lt(k, *best)) *best = k;
            }
        } else {
            /* visit the nearer child first (order does not change the result) */
            float dl = boxdist(p, &t->nodes[nd->left], dim);
            float dr = boxdist(p, &t->nodes[nd->right], dim);
            if (dl <= dr) { stack[sp++] = nd->right; stack[sp++] = nd->left; }
            else { stack[sp++] = nd->left; stack[sp++] = nd->right; }
        }
    }
}

/* Boruvka over the kd-tree.  rounds_out (nullable) gets the number of
 * rounds; comps_out (nullable, capacity >= 64) gets the component count at
 * the start of every round.  nthreads <= 0 uses the OpenMP default. */
static int kdboruvka_impl(const float *pts, int64_t n, int dim, const float *core2, int32_t *edges, float *d2,
                          int nthreads, int64_t *rounds_out, int64_t *comps_out) {
    if (rounds_out) *rounds_out = 0;
    if (n < 2) return 0;
    if (dim < 1 || dim > 3) return -1;
    unsigned int csr = fp_enter();
    int rc = 0;
    kdtree t;
    memset(&t, 0, sizeof(t));
    t.pts = pts;
    t.dim = dim;
    t.idx = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int64_t *par = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    uint32_t *lab = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    okey *best = (okey *)malloc((size_t)n * sizeof(okey));
    int64_t *cstart = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t *members = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int64_t *fill = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    uint32_t *node_comp = NULL;
    if (!t.idx || !par || !lab || !best || !cstart || !members || !fill) { rc = -4; goto done; }
    for (int64_t i = 0; i < n; ++i) { t.idx[i] = (int32_t)i; par[i] = i; }
    rc = kd_build(&t, n);
    if (rc) goto done;
    node_comp = (uint32_t *)malloc((size_t)t.n_nodes * sizeof(uint32_t));
    if (!node_comp) { rc = -4; goto done; }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    /* ORACLE_PROGRESS set: one line per round on stderr (long runs) */
    const int progress = getenv("ORACLE_PROGRESS") != NULL;
    int64_t n_edges = 0, n_comp = n, round = 0;
    while (n_comp > 1) {
        if (comps_out && round < 64) comps_out[round] = n_comp;
        if (progress) {
            fprintf(stderr, "oracle: kd-Boruvka round %lld, %lld components\n", (long long)round, (long long)n_comp);
            fflush(stderr);
        }
        /* (i) component of every point, fixed for the round */
        for (int64_t i = 0; i < n; ++i) lab[i] = (uint32_t)uf_find(par, i);
        /* (ii) component of every node: children were created after their
         * parent, so a reverse sweep over node ids is a bottom-up order */
        for (int64_t id = t.n_nodes - 1; id >= 0; --id) {
            const kdnode *nd = &t.nodes[id];
            uint32_t c;
            if (nd->left < 0) {
                c = lab[t.idx[nd->begin]];
                for (int64_t q = nd->begin + 1; q < nd->end && c != MIXED; ++q)
                    if (lab[t.idx[q]] != c) c = MIXED;
            } else {
                uint32_t a = node_comp[nd->left], b = node_comp[nd->right];
                c = (a == b) ? a : MIXED;
            }
            node_comp[id] = c;
        }
        /* (iii) group points by component, best[c] = +inf */
        for (int64_t c = 0; c <= n; ++c) cstart[c] = 0;
        for (int64_t i = 0; i < n; ++i) cstart[lab[i] + 1]++;
        for (int64_t c = 0; c < n; ++c) cstart[c + 1] += cstart[c];
        for (int64_t c = 0; c < n; ++c) fill[c] = cstart[c];
        for (int64_t i = 0; i < n; ++i) members[fill[lab[i]]++] = (int32_t)i;
        for (int64_t c = 0; c < n; ++c) best[c] = KEY_INF;
        /* (iv) every point of every component searches; components are
         * independent, so they run in parallel and best[c] has one writer */
#pragma omp parallel
        {
            fp_enter();
            /* median splits keep the depth <= 64 for any n < 2^63, and the
             * search stack holds at most one entry more than the depth */
            int32_t stk[KD_STACK];
#pragma omp for schedule(dynamic, 64)
            for (int64_t c = 0; c < n; ++c) {
                for (int64_t q = cstart[c]; q < cstart[c + 1]; ++q)
                    query_point(&t, core2, lab, node_comp, members[q], &best[c], stk);
            }
        }
        /* (v) add every component's shortest outgoing edge; a mutual pair
         * selects the same edge twice and adds it once */
        for (int64_t c = 0; c < n; ++c) {
            if (cstart[c + 1] == cstart[c]) continue;
            okey e = best[c];
            if (e.w == 0xFFFFFFFFu) { rc = -7; goto done; }
            int64_t a = uf_find(par, e.u), b = uf_find(par, e.v);
            if (a == b) continue;
            par[a < b ? b : a] = a < b ? a : b;
            edges[2 * n_edges] = (int32_t)e.u;
            edges[2 * n_edges + 1] = (int32_t)e.v;
            d2[n_edges] = bitsf(e.w);
            ++n_edges;
            --n_comp;
        }
        ++round;
    }
    if (rounds_out) *rounds_out = round;
    if (n_edges != n - 1) rc = -7;
done:
    free(t.idx); free(t.nodes); free(par); free(lab); free(best);
    free(cstart); free(members); free(fill); free(node_comp);
    fp_leave(csr);
    return rc;
}

int oracle_kdboruvka(const float *pts, int64_t n, int dim, int32_t *edges, float *d2,
                     int nthreads, int64_t *rounds_out, int64_t *comps_out) {
    return kdboruvka_impl(pts, n, dim, NULL, edges, d2, nthreads, rounds_out, comps_out);
}

int oracle_kdboruvka_mreach(const float *pts, int64_t n, int dim, const float *core2, int32_t *edges, float *d2,
                            int nthreads, int64_t *rounds_out, int64_t *comps_out) {
    return kdboruvka_impl(pts, n, dim, core2, edges, d2, nthreads, rounds_out, comps_out);
}

/* ------------------------------------------------------------------------ */
/* core distances (Section 4, "Mutual reachability distance")               */

static int cmp_float(const void *a, const void *b) {
    float x = *(const float *)a, y = *(const float *)b;
    return (x < y) ? -1 : (x > y) ? 1 : 0;
}

/* core2[u] = the k-th smallest of the n values D(u, v), v = 0..n-1 (v = u
 * gives 0: the point itself counts).  1 <= k <= n. */
int oracle_core_brute(const float *pts, int64_t n, int dim, int k, float *core2, int nthreads) {
    if (n < 1) return 0;
    if (dim < 1 || k < 1 || k > n) return -1;
    unsigned int csr = fp_enter();
    int rc = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        fp_enter();
        float *row = (float *)malloc((size_t)n * sizeof(float));
#pragma omp for schedule(dynamic, 16)
        for (int64_t u = 0; u < n; ++u) {
            if (!row) { rc = -4; continue; }
            for (int64_t v = 0; v < n; ++v) row[v] = sqdist(pts + u * dim, pts + v * dim, dim);
            qsort(row, (size_t)n, sizeof(float), cmp_float);
            core2[u] = row[k - 1];
        }
        free(row);
    }
    fp_leave(csr);
    return rc;
}

/* The same by a k-nearest search over the kd-tree: a max-heap keeps the k
 * smallest values seen (the point itself is among the candidates); a box is
 * skipped when the heap is full and its box distance exceeds the heap top. */
static void heap_push(float *h, int *len, int k, float x) {
    if (*len < k) {
        int i = (*len)++;
        h[i] = x;
        while (i > 0 && h[(i - 1) / 2] < h[i]) {
            float tmp = h[i]; h[i] = h[(i - 1) / 2]; h[(i - 1) / 2] = tmp;
            i = (i - 1) / 2;
        }
    } else if (x < h[0]) {
        h[0] = x;
        int i = 0;
        for (;;) {
            int l = 2 * i + 1, r = l + 1, m = i;
            if (l < k && h[l] > h[m]) m = l;
            if (r < k && h[r] > h[m]) m = r;
            if (m == i) break;
            float tmp = h[i]; h[i] = h[m]; h[m] = tmp;
            i = m;
        }
    }
}

int oracle_core_kd(const float *pts, int64_t n, int dim, int k, float *core2, int nthreads) {
    if (n < 1) return 0;
    if (dim < 1 || dim > 3 || k < 1 || k > n) return -1;
    unsigned int csr = fp_enter();
    int rc = 0;
    kdtree t;
    memset(&t, 0, sizeof(t));
    t.pts = pts;
    t.dim = dim;
    t.idx = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!t.idx) { fp_leave(csr); return -4; }
    for (int64_t i = 0; i < n; ++i) t.idx[i] = (int32_t)i;
    rc = kd_build(&t, n);
    if (rc) { free(t.idx); free(t.nodes); fp_leave(csr); return rc; }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        fp_enter();
        float *heap = (float *)malloc((size_t)k * sizeof(float));
        int32_t stk[KD_STACK];
#pragma omp for schedule(dynamic, 256)
        for (int64_t u = 0; u < n; ++u) {
            if (!heap) { rc = -4; continue; }
            const float *p = pts + u * dim;
            int len = 0;
            int64_t sp = 0;
            stk[sp++] = 0;
            while (sp > 0) {
                const kdnode *nd = &t.nodes[stk[--sp]];
                if (len == k && boxdist(p, nd, dim) > heap[0]) continue;
                if (nd->left < 0) {
                    for (int64_t q = nd->begin; q < nd->end; ++q)
                        heap_push(heap, &len, k, sqdist(p, pts + (int64_t)t.idx[q] * dim, dim));
                } else {
                    float dl = boxdist(p, &t.nodes[nd->left], dim);
                    float dr = boxdist(p, &t.nodes[nd->right], dim);
                    if (dl <= dr) { stk[sp++] = nd->right; stk[sp++] = nd->left; }
                    else { stk[sp++] = nd->left; stk[sp++] = nd->right; }
                }
            }
            core2[u] = heap[0];
        }
        free(heap);
    }
    free(t.idx);
    free(t.nodes);
    fp_leave(csr);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* canonical output: edges sorted by K, weights = sqrtf(D)                   */

typedef struct { okey k; } sortrec;

static int cmp_key(const void *a, const void *b) {
    okey x = ((const sortrec *)a)->k, y = ((const sortrec *)b)->k;
    if (key_lt(x, y)) return -1;
    if (key_lt(y, x)) return 1;
    return 0;
}

int oracle_canonicalize(int64_t m, int32_t *edges, float *d2, float *w) {
    unsigned int csr = fp_enter();
    sortrec *r = (sortrec *)malloc((size_t)(m > 0 ? m : 1) * sizeof(sortrec));
    if (!r) { fp_leave(csr); return -4; }
    for (int64_t e = 0; e < m; ++e) {
        int32_t a = edges[2 * e], b = edges[2 * e + 1];
        r[e].k.w = fbits(d2[e]);
        r[e].k.u = (uint32_t)(a < b ? a : b);
        r[e].k.v = (uint32_t)(a < b ? b : a);
    }
    qsort(r, (size_t)m, sizeof(sortrec), cmp_key);
    for (int64_t e = 0; e < m; ++e) {
        edges[2 * e] = (int32_t)r[e].k.u;
        edges[2 * e + 1] = (int32_t)r[e].k.v;
        d2[e] = bitsf(r[e].k.w);
        if (w) w[e] = sqrtf(d2[e]);
    }
    free(r);
    fp_leave(csr);
    return 0;
}

/* FP64 left-to-right sum of the weights in the given order. */
double oracle_total_weight(int64_t m, const float *w) {
    double s = 0.0;
    for (int64_t e = 0; e < m; ++e) s += (double)w[e];
    return s;
}
