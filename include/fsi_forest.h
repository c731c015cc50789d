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

/* The Moebius transform of v (the coefficients a the FSI operator starts
 * from, Sec. 2.2), without forming v: a leaf of a tree is reached at z_b(S)
 * iff every test on its root path passes, so its indicator is a product over
 * the path's features f of (beta_f + [f in S] (alpha_f - beta_f)), with
 * alpha_f (beta_f) = 1 if x (bg_b) passes every test on f of that path. Its
 * Moebius coefficients are +-value on the sets I u Q, I = {f: beta_f = 0},
 * Q a subset of {f: beta_f = 1, alpha_f = 0}, sign (-1)^|Q| (none if some f
 * in I has alpha_f = 0). One GPU thread per (background, root-to-leaf path)
 * adds value / n_bg at each of them.
 *  a_dev: 2^d FP64 (device, caller-owned); zeroed by the call, then summed
 *         with FP64 atomics, so the result is not bitwise repeatable (equal
 *         to rounding).
 * Arguments otherwise as fsi_forest_values. FSI_ERR_UNSUPPORTED if the
 * forest has more than 2^26 root-to-leaf paths, or paths of more than 24
 * splits while d > 24 (a path with k free features adds 2^k terms). */
fsi_status fsi_forest_mobius(fsi_forest_t forest, const double* x_dev, int n_bg,
                             const double* bg_dev, double* a_dev, hipStream_t stream);

/* v through the Moebius route: fsi_forest_mobius into work_dev, then the
 * subset-sum (zeta) butterfly v(S) = sum_{R subset of S} a(R) in FP64 passes
 * (the low 10 index bits in LDS, then 5 bits per pass in registers), the last
 * pass writing v_dev in dtype.
 *  work_dev: 2^d FP64 (device, caller-owned); may equal v_dev when dtype is
 *            FSI_DTYPE_F64, must differ from it for FSI_DTYPE_F32.
 * Equal to fsi_forest_values up to FP64 rounding (the sums run in another
 * order); much faster for shallow trees (work per path is 2^(free
 * features), not 2^d walks). */
fsi_status fsi_forest_values_mobius(fsi_forest_t forest, const double* x_dev, int n_bg,
                                    const double* bg_dev, double* work_dev, int dtype,
                                    void* v_dev, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* FSI_FOREST_MI355X_H */
