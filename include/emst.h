/*
 * emst.h -- single-tree Boruvka Euclidean minimum spanning tree on one
 * MI355X (gfx950), C ABI.
 *
 * The problem (Section 2, "EMST computation"): given n points in d
 * dimensions, return the minimum spanning tree of their complete distance
 * graph.  Equal weights are ordered by the vertex indices (Section 2, the
 * tie-breaking rule in "Boruvka's algorithm"), applied here to the float32
 * squared distance:
 *
 *     K(u, v) = ( bits(D(u, v)), min(u, v), max(u, v) )
 *
 * where D(a, b) = ((a0-b0)^2 + (a1-b1)^2) [+ (a2-b2)^2], each step rounded
 * to float32 (round to nearest even), evaluated left to right with no fused
 * multiply-add and with denormals kept.  K is a strict total order, so the
 * tree is unique, and it is the tree every entry point below returns.
 *
 * Method (Section 3, Figure 3): a linear BVH over the points (Morton codes,
 * radix sort, binary radix hierarchy, bottom-up bounding boxes), then
 * Boruvka rounds, each of which (1) propagates component labels to the
 * internal nodes (Optimization 1), (2) bounds every component's shortest
 * outgoing edge from Morton-adjacent pairs (Optimization 2), (3) runs one
 * nearest-other-component traversal per point (Algorithm 2) and keeps each
 * component's minimum edge, and (4) merges the components along the chains
 * of chosen edges ("Merging components together").
 *
 * Conventions for every entry point:
 *  - Every pointer named d_* is DEVICE memory on the context's HIP device;
 *    every pointer named h_* is HOST memory.  The caller owns all of them.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    All device work is ordered on it.
 *  - The library allocates no device memory in these calls: scratch space is
 *    the caller's workspace of at least emst_workspace_bytes(n, dim) bytes,
 *    256-byte aligned.
 *  - Functions return EMST_OK (0) or a negative EMST_E* code; the context
 *    keeps a message for the last error (emst_last_error).  No C++ exception
 *    crosses this interface.
 *  - A context is not thread-safe: one host thread at a time.
 */
#ifndef EMST_H
#define EMST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EMST_OK 0
#define EMST_EINVAL (-1)      /* bad argument: null pointer, n < 0, dim not 2 or 3, n > 2^31-1 */
#define EMST_ENONFINITE (-2)  /* a coordinate is NaN or +-inf */
#define EMST_ERANGE (-3)      /* the squared extent of the cloud overflows float32 */
#define EMST_ENOMEM (-4)      /* workspace smaller than emst_workspace_bytes() */
#define EMST_EHIP (-5)        /* a HIP runtime call failed; see emst_last_error */
#define EMST_EBUSY (-6)       /* reserved */
#define EMST_EINTERNAL (-7)   /* an internal consistency check failed */

typedef struct emst_ctx emst_ctx;

/* Create a context bound to HIP device `hip_device` (it becomes current on
 * the calling thread).  *out receives the handle.  autotune_json (nullable)
 * is a traversal-shape table as emst_set_autotune takes it; a malformed
 * table gives EMST_EINVAL and no context. */
int emst_create(emst_ctx **out, int hip_device, const char *autotune_json);

/* Destroy a context (NULL is allowed).  Waits for nothing: the caller
 * synchronises its streams first. */
void emst_destroy(emst_ctx *ctx);

/* Message of the last failing call on this context ("" if none). */
const char *emst_last_error(const emst_ctx *ctx);

/* Exact number of workspace bytes emst_build, emst_core_distances and
 * emst_build_mreach need for n points of dimension dim (0 for invalid
 * arguments).  Grows linearly in n, 238 bytes per point in 3D. */
size_t emst_workspace_bytes(int64_t n, int dim);

/*
 * emst_build -- EMST of one point cloud.
 *
 *  d_points   [n][dim] float32, row-major (point i at d_points[i*dim]).
 *  n, dim     0 <= n <= 2^31-1, dim in {2, 3}.
 *  d_edges    [n-1][2] int32 out: edge e joins d_edges[2e] < d_edges[2e+1],
 *             original point indices; edges sorted by K ascending.
 *  d_weights  [n-1] float32 out: sqrtf(D) of each edge, correctly rounded.
 *  d_d2       [n-1] float32 out, or NULL: D of each edge.
 *  d_workspace, ws_bytes   caller scratch, >= emst_workspace_bytes(n, dim).
 *
 * n = 0 or 1 writes nothing and returns EMST_OK.  Errors: EMST_EINVAL,
 * EMST_ENONFINITE, EMST_ERANGE (then nothing is written to the outputs),
 * EMST_ENOMEM, EMST_EHIP, EMST_EINTERNAL.  The call returns when the
 * result is complete on `stream` (the round loop reads the component
 * count back once per round, as in Figure 3).
 */
int emst_build(emst_ctx *ctx, const float *d_points, int64_t n, int dim,
               int32_t *d_edges, float *d_weights, float *d_d2,
               void *d_workspace, size_t ws_bytes, void *stream);

/*
 * emst_build_noalloc -- emst_build for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  It takes no workspace: its scratch space is a
 * static device array of EMST_NOALLOC_WORKSPACE_BYTES that every device the
 * library runs on holds until the process ends; the call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine).
 *
 *  d_points, n, dim, d_edges, d_weights, d_d2, stream   as for emst_build;
 *  the result is bit-identical to emst_build's.
 *
 * Limit: emst_workspace_bytes(n, dim) <= EMST_NOALLOC_WORKSPACE_BYTES
 * (about 280,000 points in 3D, 300,000 in 2D); larger n gives EMST_ENOMEM
 * with a message naming the sizes, and nothing is written.  Every call on
 * one device shares that device's array and leaves its contents behind
 * (the kernels initialise everything they read), so calls that overlap on
 * one device -- from two host threads, or on two streams without an order
 * between them -- race and must not be issued.  Other errors as for
 * emst_build; EMST_EHIP also if the array's device address could not be
 * obtained when the context was created.
 */
#define EMST_NOALLOC_WORKSPACE_BYTES (64u << 20)
int emst_build_noalloc(emst_ctx *ctx, const float *d_points, int64_t n, int dim,
                       int32_t *d_edges, float *d_weights, float *d_d2, void *stream);

/* Exact workspace bytes emst_build_batched needs for `total_points` points
 * in `n_clouds` clouds (0 for invalid arguments). */
size_t emst_workspace_bytes_batched(int64_t total_points, int32_t n_clouds);

/*
 * emst_build_batched -- EMSTs of many independent clouds in one pass.
 *
 * The clouds are built as one tree in which every cloud is its own
 * subtree; one round loop serves all of them and a query only searches its
 * own cloud.  The result of every cloud is exactly what emst_build returns
 * for that cloud alone.
 *
 *  d_points       float32, the clouds one after the other; cloud c holds
 *                 n_c = h_offsets[c+1] - h_offsets[c] points of h_dims[c]
 *                 coordinates each (row-major), starting at float index
 *                 sum_{c' < c} n_c' * h_dims[c'].
 *  h_offsets      [n_clouds + 1] host, h_offsets[0] = 0, non-decreasing;
 *                 h_offsets[n_clouds] <= 2^31 - 1 points in total.
 *  h_dims         [n_clouds] host, each 2 or 3 (mixed dims are fine).
 *  d_edges        [sum max(n_c - 1, 0)][2] int32 out: cloud c's edges start
 *                 at edge h_edge_offsets[c], with cloud-local indices
 *                 (0 .. n_c - 1), u < v, sorted by K within the cloud.
 *  d_weights, d_d2  as in emst_build, same edge order (d_d2 nullable).
 *  h_edge_offsets [n_clouds + 1] host out (nullable): first edge of every
 *                 cloud; h_edge_offsets[n_clouds] = total edges.
 *
 * Errors as emst_build, for any cloud (the message names the cloud).
 */
int emst_build_batched(emst_ctx *ctx, const float *d_points, const int64_t *h_offsets,
                       const int32_t *h_dims, int32_t n_clouds, int32_t *d_edges,
                       float *d_weights, float *d_d2, int64_t *h_edge_offsets,
                       void *d_workspace, size_t ws_bytes, void *stream);

/*
 * emst_core_distances -- squared core distances of the mutual reachability
 * metric (Section 4, "Mutual reachability distance"): the core distance of
 * point i is its distance to the k_pts-th nearest point, i itself counted
 * (so k_pts = 1 gives 0).
 *
 *  d_points, n, dim   as for emst_build.
 *  k_pts      1 <= k_pts <= min(n, 64).
 *  d_core2    [n] float32 out, input order: the k_pts-th smallest D(i, j)
 *             over all j (float32 D as for emst_build, so bit-exact).
 *  d_workspace, ws_bytes   >= emst_workspace_bytes(n, dim).
 *
 * Errors: EMST_EINVAL (also for k_pts out of range), EMST_ENONFINITE,
 * EMST_ERANGE, EMST_ENOMEM, EMST_EHIP, EMST_EINTERNAL.  Returns when the
 * result is complete on `stream`.
 */
int emst_core_distances(emst_ctx *ctx, const float *d_points, int64_t n, int dim, int32_t k_pts,
                        float *d_core2, void *d_workspace, size_t ws_bytes, void *stream);

/*
 * emst_build_mreach -- minimum spanning tree under the mutual reachability
 * of HDBSCAN* (Section 4, "Mutual reachability distance"; Section 3,
 * "Non-Euclidean metrics"):
 *
 *   M(u, v) = max(core2(u), core2(v), D(u, v))      (squared terms)
 *
 * with core2 as emst_core_distances computes it; the tree is the unique
 * MST under (bits(M), min(u, v), max(u, v)).  k_pts = 1 gives the EMST.
 *
 *  d_points, n, dim, d_edges   as for emst_build (edges sorted by that key).
 *  k_pts      1 <= k_pts <= min(n, 64).
 *  d_weights  [n-1] float32 out: sqrtf(M) of each edge.
 *  d_d2       [n-1] float32 out, or NULL: M of each edge.
 *  d_core2    [n] float32 out, or NULL: the squared core distances.
 *  d_workspace, ws_bytes   >= emst_workspace_bytes(n, dim).
 *
 * n = 0 or 1 writes no edges and returns EMST_OK.  Errors as for
 * emst_core_distances.
 */
int emst_build_mreach(emst_ctx *ctx, const float *d_points, int64_t n, int dim, int32_t k_pts,
                      int32_t *d_edges, float *d_weights, float *d_d2, float *d_core2,
                      void *d_workspace, size_t ws_bytes, void *stream);

/*
 * Round-granular continuous batching (serving).  A solver keeps up to
 * max_slots requests inside a caller-provided device budget.  The requests
 * admitted between two steps start together at the next emst_solver_step
 * as one cohort: a batch as emst_build_batched builds it (one tree, one
 * round loop for all of them).  Each step advances every live cohort by one
 * phase -- per-cloud boxes, Morton codes, tree, boxes and the first round,
 * then one Boruvka round per step, then the edge order -- and waits once
 * for all of them, so a request admitted while others run starts at the
 * next step.  Every result is exactly emst_build of that request alone.
 * All calls on one solver must come from one thread; the budget must stay
 * allocated until emst_solver_destroy.
 */
typedef struct emst_solver emst_solver;

/* Budget bytes one request of n points of dimension dim holds from admit to
 * take (its points while it waits, the workspace and outputs of a cohort of
 * that request alone); 0 for invalid arguments.  The requests admitted
 * together share one cohort region of at most the sum of their shares; a
 * finished cohort keeps only its outputs until its last result is taken. */
size_t emst_solver_slot_bytes(int64_t n, int dim);

/* d_budget: device memory of budget_bytes, 256-byte aligned, owned by the
 * caller.  1 <= max_slots <= 4096.  The solver uses the context's traversal
 * choice and autotune table; the context must outlive it. */
int emst_solver_create(emst_ctx *ctx, void *d_budget, size_t budget_bytes, int32_t max_slots,
                       emst_solver **out);
void emst_solver_destroy(emst_solver *solver);

/* Admit a request: copies d_points [n][dim] into the budget (on `stream`)
 * and returns its slot.  EMST_EBUSY if no slot is free, or the shares of
 * the requests not yet taken leave less than this one's, or its points find
 * no contiguous range (retry after emst_solver_take); EMST_ENOMEM if the
 * request does not fit even an empty budget; EMST_EINVAL for bad
 * arguments.  A request of 0 or 1 point is finished at once.  Input
 * problems of the points (non-finite, overflowing extent) surface as the
 * slot's status; the other requests of its cohort go on without it. */
int emst_solver_admit(emst_solver *solver, const float *d_points, int64_t n, int32_t dim, int64_t tag,
                      void *stream, int32_t *slot);

/* Start a cohort of the requests admitted since the last step (as many, in
 * admission order, as fit one contiguous free range, unless 8 cohorts run
 * already; the others wait for a later step), then move every cohort whose
 * queued phase has completed on to its next phase; returns once at least
 * one cohort has moved (at once if none runs).  Each cohort runs on its own
 * stream of the solver (default priority), after the work queued on
 * `stream` before its first step.  A request that finds no range while no
 * cohort holds memory fails with EMST_ENOMEM.  *n_finished (nullable) =
 * requests that finished or failed in this step. */
int emst_solver_step(emst_solver *solver, void *stream, int32_t *n_finished);

/* *state: 0 free, 1 running, 2 finished, < 0 failed with that status;
 * *tag (nullable) the admit tag. */
int emst_solver_poll(const emst_solver *solver, int32_t slot, int32_t *state, int64_t *tag);

/* The slots whose request has finished or failed and is not taken yet: up
 * to `cap` of them into slots[], their number in *count.  They come ordered
 * by cohort and by position in the cohort's outputs, the order in which
 * emst_solver_take_many copies them in the fewest pieces. */
int emst_solver_ready(const emst_solver *solver, int32_t *slots, int32_t cap, int32_t *count);

/* emst_solver_take for `count` finished requests at once (every slot must
 * hold a finished result, state 2; else EMST_EINVAL and nothing is taken).
 * Their results go one after another into d_edges [total][2], d_weights
 * [total] and d_d2 [total] (nullable): request i owns rows
 * h_offsets[i] .. h_offsets[i+1]-1 (h_offsets: count + 1 entries, host).
 * Results that lie back to back in one cohort's outputs are copied in one
 * piece; copies are queued on `stream`, and the slots are free. */
int emst_solver_take_many(emst_solver *solver, const int32_t *slots, int32_t count, int32_t *d_edges,
                          float *d_weights, float *d_d2, int64_t *h_offsets, void *stream);

/* Queue on `stream` the copies of a finished request's n-1 edges, weights
 * and (nullable) d2, as emst_build writes them, and free its slot (the
 * outputs are complete once `stream` reaches that point; the solver reuses
 * the memory they come from only after the copies).  A failed request
 * returns its status (message in emst_last_error) and frees its slot; a
 * running one gives EMST_EBUSY. */
int emst_solver_take(emst_solver *solver, int32_t slot, int32_t *d_edges, float *d_weights, float *d_d2,
                     void *stream);

/* Per-call statistics of the last successful emst_build or
 * emst_build_batched on this context.
 * Timings are measured with HIP events on the call's stream when profiling
 * is on (emst_set_profiling), else they are 0. */
typedef struct emst_stats {
    int64_t n;
    int32_t dim;
    int32_t rounds;                 /* Boruvka rounds */
    int64_t components[64];         /* components at the start of each round */
    int32_t tree_height;            /* edges on the longest root-leaf path */
    int32_t traversal_launches;     /* = rounds */
    double traversal_ms;            /* sum over rounds, traversal kernel only */
    double traversal_ms_round[64];  /* per round */
    double tree_ms;                 /* Morton codes .. bounding boxes */
    double rounds_ms;               /* all rounds, every kernel */
    double finalize_ms;             /* canonical edge sort and weights */
    double total_ms;                /* whole call on the stream */
    /* filled only when counting is on (emst_set_counting): children
     * examined by the traversal, internal nodes and leaves separately,
     * summed over all points of all rounds, and per round */
    int64_t child_tests;
    int64_t leaf_tests;
    int64_t child_tests_round[64];
    int64_t leaf_tests_round[64];
    int64_t dist_evals;             /* leaf children outside the query's
                                       component: point distances computed */
    int32_t traversal_variant;      /* the traversal variant that ran */
    int32_t rank_codes;             /* 1 if the tree was built on rank-space
                                       codes (many points shared a Morton
                                       code), else 0 */
    int64_t queries_round[64];      /* points the traversal searched in each
                                       round: n, or the length of the round's
                                       query list (variant 13, third round on) */
    int64_t records_touched_round[64];  /* counting only: distinct node
                                       records the traversal loaded in each
                                       round */
    int32_t traversal_lds_depth;    /* LDS stack ring entries per lane of
                                       variant 13 (0 for other variants) */
    int32_t pad_;
} emst_stats;

/* Time every phase with HIP events (adds synchronisation; off by default). */
int emst_set_profiling(emst_ctx *ctx, int on);

/* Batches (emst_build_batched): run the rounds from the third on as replays
 * of a captured graph of two rounds, with one control-block read-back per
 * replay instead of one per round (off by default; profiling and counting
 * runs never use it).  The context keeps the last few instantiated graphs,
 * keyed by workspace, sizes and traversal shape.  Same results either way. */
int emst_set_graphs(emst_ctx *ctx, int on);

/* Use the instrumented traversal that counts child-box tests and leaf
 * distance evaluations (same result, slower; off by default). */
int emst_set_counting(emst_ctx *ctx, int on);

/* Traversal launch shape.  All compute the same result:
 *   0  one lane per query, top-down from the root, stack in private memory
 *   5  as 0 with a branch-free inner loop and a 16-deep LDS stack
 *   7  as 5 with an 8-deep LDS stack
 *   8  as 5 with a 4-deep LDS stack
 *  10  as 7, but each wave of 64 queries starts below the root, at the
 *      lowest ancestor of its leaves whose Morton cell holds every lane's
 *      search ball
 *  11  as 10 with the component bound shared while the round runs (every
 *      improved candidate lowers it with an atomicMin, every node visit
 *      re-reads it)
 *  13  as 10, and a point keeps last round's result where it still holds:
 *      its candidate if that is still outside its component, or "nothing"
 *      if it found nothing within a radius at least the new one (default)
 * -1 (the default) takes the variant from the context's autotune table
 * (emst_set_autotune) for the call's mode, dimension and size, else 13.
 * Batches (emst_build_batched) run 0, 5, 8 or 13 (with the start of 7) as
 * chosen and 7 for 10 and 11.
 * Returns EMST_EINVAL for any other value. */
int emst_set_traversal(emst_ctx *ctx, int variant);

/* LDS stack ring of variant 13: entries per lane kept in LDS (4, 8 or 16;
 * deeper entries spill to private memory).  Deeper rings spill less but
 * hold fewer waves per CU.  0 (the default) takes the depth from the
 * autotune table entry of the call, else 8.  EMST_EINVAL for any other
 * value.  Every depth gives the same result. */
int emst_set_lds_depth(emst_ctx *ctx, int depth);

/* Traversal-shape table (the autotuner's output), a JSON document
 *
 *   {"entries": [{"mode": "single" | "batched", "dim": 2 | 3,
 *                 "n_min": <points>, "variant": <0, 5, 7, 8, 10, 11 or 13>,
 *                 "lds_depth": <4, 8 or 16; optional, default 8>}, ...]}
 *
 * (other keys are ignored).  A call in auto mode (emst_set_traversal -1,
 * emst_set_lds_depth 0) with n points uses the entry of its mode and
 * dimension with the largest n_min <= n.  NULL clears the table.  EMST_EINVAL on a malformed table,
 * which then stays as it was.  Every variant gives the same result. */
int emst_set_autotune(emst_ctx *ctx, const char *json);

/* The table as JSON into buf (capacity cap bytes, NUL-terminated); *len
 * (nullable) receives the bytes needed.  buf = NULL only queries the
 * length; EMST_ENOMEM if cap is too small. */
int emst_get_autotune(const emst_ctx *ctx, char *buf, size_t cap, size_t *len);

int emst_get_stats(const emst_ctx *ctx, emst_stats *out);

#ifdef __cplusplus
}
#endif

#endif /* EMST_H */
