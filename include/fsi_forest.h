/*
 * fsi_forest.h - the value function of a tree ensemble, generated on the
 * GPU, as the input of the FSI operator (include/fsi.h).
 *
 * FSI scores a value function v over all 2^d coalitions (Sec. 2.1: v(S) is
 * the model's output when only the features in S come from the explained
 * point). For tree models the paper obtains v by one model prediction per
 * coalition before the FSI computation, and its bottleneck analysis in the
 * appendix shows that step taking a large share of the total at d = 20. Here
 * it is a GPU kernel; the interventional form averages over background
 * points:
 *
 *   v(S) = (1/B) sum_{b=1..B} sum_{k=1..K} f_k(z_b(S)),
 *   z_b(S)_i = x_i if i in S, else bg_b,i        (bit i of S <=> feature i)
 *
 * Tree format (host arrays over n_nodes nodes, copied by fsi_forest_create):
 *  - node i is a leaf if feature[i] < 0; its output is value[i];
 *  - otherwise it sends z to right[i] if z[feature[i]] >= threshold[i] and
 *    to left[i] otherwise (a tie goes right);
 *  - roots[k] is the root of tree k. Nodes may be shared between trees.
 *
 * Conventions: as in fsi.h (status codes, fsi_last_error(), caller-owned
 * 16-byte aligned device memory, asynchronous calls on a HIP stream).
 */
#ifndef FSI_FOREST_MI355X_H
#define FSI_FOREST_MI355X_H

#include "fsi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsi_forest_s* fsi_forest_t;

/* Validate and upload a forest for d features and up to max_bg background
 * points per call.
 *  d in [1, 30]; n_trees >= 1; n_nodes >= 1; 1 <= max_bg <= 4096;
 *  roots[k], left[i], right[i] (internal nodes) in [0, n_nodes);
 *  feature[i] < d; thresholds finite; no cycle, and at most 64 internal
 *  nodes on any root-to-leaf path.
 * Violations return FSI_ERR_INVALID_ARG before any device work; no gfx950
 * device gives FSI_ERR_UNSUPPORTED. The forest owns device copies of the
 * arrays and a workspace of ceil(max_bg / 32) * n_nodes * 16 bytes.
 * *out receives the handle (NULL on failure). */
fsi_status fsi_forest_create(int d, int n_trees, const int32_t* roots, int n_nodes,
                             const int32_t* feature, const double* threshold,
                             const int32_t* left, const int32_t* right,
                             const double* value, int max_bg, fsi_forest_t* out);

/* Free a forest; NULL is a no-op. */
fsi_status fsi_forest_destroy(fsi_forest_t forest);

/* v(S) for all 2^d coalitions (formula above).
 *  x_dev:  d FP64 values, the explained point (device);
 *  bg_dev: n_bg x d FP64 values, row-major background points (device),
 *          1 <= n_bg <= max_bg;
 *  dtype:  FSI_DTYPE_F64 or FSI_DTYPE_F32, the element type of v_dev;
 *  v_dev:  2^d elements of dtype (device, caller-owned), index = coalition.
 * The sum runs in FP64, backgrounds outer and trees inner, each in
 * ascending order, then divides by n_bg and rounds once to dtype. Calls on
 * one forest share its workspace: concurrent calls on different streams
 * race; use one forest per stream. */
fsi_status fsi_forest_values(fsi_forest_t forest, const double* x_dev, int n_bg,
                             const double* bg_dev, int dtype, void* v_dev,
                             hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* FSI_FOREST_MI355X_H */
