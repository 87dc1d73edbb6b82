/*
 * emst_test.h -- test entry points into single stages of the EMST pipeline.
 *
 * They run the same kernels emst_build runs, on inputs the caller chooses,
 * so the stages can be compared one by one with plain CPU definitions.
 * Same conventions as emst.h: d_* = device memory owned by the caller,
 * `stream` is a hipStream_t as void*, workspace of at least
 * emst_workspace_bytes(n, 3) bytes, 256-byte aligned; return EMST_OK or a
 * negative EMST_E* code.
 */
#ifndef EMST_TEST_H
#define EMST_TEST_H

#include "emst.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Hierarchy + label propagation on given codes (Section 3, Optimization 1
 * and Figure 4).  d_codes [n] sorted ascending (equal codes allowed);
 * d_leaf_labels [n] the component label of each leaf (values < 2^31).
 * Builds the binary radix tree of the augmented keys (code, leaf index)
 * bottom-up, propagates the labels once, and writes for every internal node
 * k in [0, n-2] (node k splits between leaves k and k+1):
 *   d_left[k], d_right[k]   child: internal node index >= 0, or -(p+1) for
 *                           leaf p
 *   d_label[k]              common label of its leaves, 0xFFFFFFFF if they
 *                           span several labels
 * *root_out (host) receives the root node index.  2 <= n <= 2^31-1.
 */
int emst_test_tree_from_codes(emst_ctx *ctx, const uint64_t *d_codes, int64_t n,
                              const uint32_t *d_leaf_labels, int32_t *d_left, int32_t *d_right,
                              uint32_t *d_label, int32_t *root_out, void *d_workspace,
                              size_t ws_bytes, void *stream);

/*
 * The tree construction of emst_build on given 3D points (Morton codes,
 * sort, hierarchy, box fit).  For every internal node k in [0, n-2]:
 *   d_left[k], d_right[k]   child: internal node index >= 0, or -(j+1) for
 *                           the leaf of ORIGINAL point index j
 *   d_lo[3k..3k+2], d_hi[3k..3k+2]   the node's bounding box
 * (the union of its two child boxes as the traversal sees them).
 * *root_out (host) receives the root.  2 <= n <= 2^31-1, d_points [n][3].
 */
int emst_test_tree_boxes(emst_ctx *ctx, const float *d_points, int64_t n, int32_t *d_left,
                         int32_t *d_right, float *d_lo, float *d_hi, int32_t *root_out,
                         void *d_workspace, size_t ws_bytes, void *stream);

/*
 * The radix sort of the tree construction: sorts the n pairs
 * (d_keys[i], d_vals[i]) in place, stably, by key bits [0, 64).
 */
int emst_test_radix_sort(emst_ctx *ctx, uint64_t *d_keys, uint32_t *d_vals, int64_t n,
                         void *d_workspace, size_t ws_bytes, void *stream);

/*
 * One Boruvka round of emst_build from a given partition (Section 3,
 * Figure 3): label propagation and component bounds (Optimizations 1 and
 * 2), the nearest-other-component traversal with stage A (Algorithm 2),
 * stage B of the tie-break, and the merge ("Merging components together"),
 * on the tree emst_build builds for d_points [n][dim].
 *
 *  d_comp     [n] int32: the component of every point (input order), values
 *             in [0, n), at least two distinct ones.
 *  round      which round's kernels run, 1 .. 63 (1: the second round; from
 *             2 on, variant 13 searches from a query list at 3 * 2^18 points
 *             and more).  No earlier result is reused: every point searches.
 *  variant    traversal variant, as emst_set_traversal takes it (not -1).
 * Outputs per point, input order (device memory, [n] each):
 *  d_bound    the bound of the point's component after the bound pass
 *  d_cand_d, d_cand_j   the point's candidate: the (D, j)-nearest point
 *             outside its component within the bound, or (+inf, -1)
 *  d_comp_d2, d_comp_u, d_comp_v   its component's edge after stages A and
 *             B: the minimum under (D, min, max), u < v original indices
 *  d_comp_out the component after the merge: the original index of one
 *             point of it, the same for all of its points
 * *ncomp_out (host) receives the number of components after the round.
 */
int emst_test_round(emst_ctx *ctx, const float *d_points, int64_t n, int dim, const int32_t *d_comp,
                    int32_t round, int32_t variant, float *d_bound, float *d_cand_d, int32_t *d_cand_j,
                    float *d_comp_d2, int32_t *d_comp_u, int32_t *d_comp_v, int32_t *d_comp_out,
                    int64_t *ncomp_out, void *d_workspace, size_t ws_bytes, void *stream);

/*
 * The distance and weight functions of the kernels on m pairs of points
 * (a_i, b_i), d_a and d_b [m][dim] float32 (dim 2 or 3):
 *   d_sq[i]   D(a_i, b_i) as the bound pass evaluates it
 *   d_box[i]  the box distance from a_i to the one-point box [b_i, b_i],
 *             as the traversal evaluates D at a leaf
 *   d_w[i]    the reported weight of an edge of squared length d_sq[i]
 */
int emst_test_distances(emst_ctx *ctx, const float *d_a, const float *d_b, int64_t m, int dim, float *d_sq,
                        float *d_box, float *d_w, void *stream);

/*
 * The weight function on float32 bit patterns: d_w[k] = weight of the
 * squared length whose bits are first + k, for k in [0, count);
 * first + count <= 2^32.
 */
int emst_test_weights(emst_ctx *ctx, uint32_t first, int64_t count, float *d_w, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* EMST_TEST_H */
