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

#ifdef __cplusplus
}
#endif

#endif /* EMST_TEST_H */
