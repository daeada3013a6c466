/*
 * gkb_rsgd.h -- Riemannian mini-batch gradient descent on the manifold of
 * rank-r matrices for similarity learning (Section 4, Algorithm 4), with the
 * retraction computed by the partial SVD of this library.
 *
 * Model: f_W(x, v) = x^T W v, W in R^{d1 x d2} of rank r, kept in factored
 * form W = U diag(s) Vf^T (U d1 x r, Vf d2 x r column-major float32 with
 * orthonormal columns, s r doubles, descending).  One step on the batch
 * (x_i, v_i, y_i), i < b:
 *   M = (1/b) sum_i y_i x_i v_i^T,   G = -M + lambda W   (Euclidean gradient)
 *   Z = P_W(G) = G Vf Vf^T + U U^T G - U U^T G Vf Vf^T   (projection onto the
 *       tangent space at W; the factors are W's)
 *   Y = W - eta Z = (1 - eta lambda) W + eta P_W(M)      (rank <= 2r)
 *   (U, s, Vf) <- first r singular triplets of Y          (the retraction,
 *       closed form of the best rank-r approximation)
 * The retraction runs the batched solver of gkb_batched.h on Y with Krylov
 * dimension k and no restart (Algorithm 2 with k inner iterations), in one
 * persistent launch; the whole step (projection products, Y, retraction) is
 * captured into one hipGraph by the plan and replayed by gkb_rsgd_plan_step.
 *
 * The plan reads the batch from fixed device buffers X (b x d1 row-major),
 * V (b x d2 row-major), y (b floats, +1 or -1) that the caller refills
 * before each step, and updates the state buffers U, s, Vf in place.  All
 * pointers are device pointers owned by the caller.  Sizes: 1 <= r <= k <=
 * min(d1, d2), k <= 64, 1 <= b <= 4096.
 */
#ifndef GKB_RSGD_H
#define GKB_RSGD_H

#include "gkb.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gkb_rsgd_plan_s* gkb_rsgd_plan;

/* Workspace bytes of a plan (0 if the sizes are invalid). */
size_t gkb_rsgd_workspace_size(int d1, int d2, int r, int k, int b);

/* Validate, lay out the workspace and capture one step into a hipGraph. */
gkb_status gkb_rsgd_plan_create(int d1, int d2, int r, int k, int b, double eta, double lambda, const float* X,
                                const float* V, const float* y, float* U, double* s, float* Vf, void* workspace,
                                size_t ws_bytes, void* stream, gkb_rsgd_plan* plan);

/* One step (asynchronous on `stream`). */
gkb_status gkb_rsgd_plan_step(gkb_rsgd_plan plan, void* stream);

/* Status, nconv, restarts, matvecs of the last retraction (synchronises `stream`). */
gkb_status gkb_rsgd_plan_info(gkb_rsgd_plan plan, int* info4, void* stream);

void gkb_rsgd_plan_destroy(gkb_rsgd_plan plan);

/* W = U diag(s) Vf^T as a d1 x d2 row-major float32 device matrix. */
gkb_status gkb_rsgd_weights(int d1, int d2, int r, const float* U, const double* s, const float* Vf, float* W,
                            void* stream);

const char* gkb_rsgd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
