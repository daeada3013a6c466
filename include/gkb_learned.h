/*
 * gkb_learned.h -- a learned start vector for the Golub-Kahan recurrence on
 * sequences of slowly changing matrices A_1, A_2, ...
 *
 * The paper starts Algorithm 1 from a random q ~ N(2,1); any nonzero q is
 * allowed (Algorithm 2: "q is arbitrary").  Here a two-layer network proposes
 * q from the sketch S = A_t Omega (gkb_gemm_rowmajor) and the previous solve's
 * left Ritz vectors, row by row:
 *   x_i = [ S_i / c_S , sqrt(m) s_j U_prev[i, j] ] (c_S = RMS of S; s_j signs
 *         each previous vector so its largest-magnitude entry is positive),
 *   z_i = w2 . relu(W1 x_i + b1) + b2,   q = z (normalised by the solver).
 * Training minimises L = 1 - ||U_t^T z||^2 / ||z||^2, the energy of the start
 * vector outside the target left subspace U_t, on pairs produced by the solver
 * itself; the convergence test still decides when a solve is done, and a random start is the
 * fallback (the caller re-solves with q ~ N(2,1) if the learned start fails).
 *
 * Layouts (device, float32 unless stated):
 *   params  [W1 (hidden x in, row-major) | b1 (hidden) | w2 (hidden) | b2]
 *   X       m rows of gkb_mlp_feature_stride() floats: in features, a 1, zeros
 *   Ut      r x m, each target vector contiguous (the U output of gkb.h)
 * Constraints: in + 1 <= gkb_mlp_feature_stride() (64), 1 <= hidden <= 1024.
 */
#ifndef GKB_LEARNED_H
#define GKB_LEARNED_H

#include "gkb.h"

#ifdef __cplusplus
extern "C" {
#endif

int64_t gkb_mlp_param_count(int in, int hidden);
int gkb_mlp_feature_stride(void);
size_t gkb_mlp_workspace_size(int64_t m, int in, int hidden, int r);

/* Features from the sketch S (m x ws, column-major, leading dimension
   lds >= m: the C output of gkb_gemm_rowmajor) and the previous left vectors
   Ut_prev (r x m); in = ws + r.  workspace: 8-byte aligned, >= 64 doubles
   (partial sums of squares of S) + r + 1 floats. */
gkb_status gkb_mlp_features(const float* S, int64_t lds, int64_t m, int ws, const float* Ut_prev, int r, float* X,
                            void* workspace, size_t ws_bytes, void* stream);

/* z (m floats) = network(X). */
gkb_status gkb_mlp_forward(const float* params, int in, int hidden, const float* X, int64_t m, float* z,
                           void* stream);

/* Loss (device double) and its gradient with respect to params (device
   floats, gkb_mlp_param_count entries) for the target left vectors Ut (r x m).
   Forward, loss statistics, per-row backward, then the parameter gradients as
   sums over rows on the MFMA. */
gkb_status gkb_mlp_loss_grad(const float* params, int in, int hidden, const float* X, int64_t m, const float* Ut,
                             int r, float* grad, double* loss, void* workspace, size_t ws_bytes, void* stream);

/* The same with a choice of loss (kind 0 is the one above).  kind 1: the mean
   over the target vectors u_j of log tan^2 of the angle between z and u_j,
   L = (1/r) sum_j log(((1 + d) ||z||^2 - (u_j.z)^2) / ((u_j.z)^2 + d ||z||^2)),
   d = 1e-6: it rewards a start with a sizeable component along every target
   vector, which is what the convergence of the Krylov subspace to each of
   them depends on, rather than the energy inside the subspace as a whole.
   Same arguments and workspace; GKB_ERR_INVALID for another kind. */
gkb_status gkb_mlp_loss_grad_kind(const float* params, int in, int hidden, const float* X, int64_t m,
                                  const float* Ut, int r, int kind, float* grad, double* loss, void* workspace,
                                  size_t ws_bytes, void* stream);

/* Adam (Kingma and Ba 2015) with bias correction for step >= 1. */
gkb_status gkb_adam_step(float* params, const float* grad, float* m1, float* m2, int64_t count, double lr,
                         double beta1, double beta2, double eps, int step, void* stream);

/* q1 (m doubles) = network(X), ready to pass as gkb_options.q1. */
gkb_status gkb_mlp_start_vector(const float* params, int in, int hidden, const float* X, int64_t m, double* q1,
                                void* workspace, size_t ws_bytes, void* stream);

const char* gkb_learned_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GKB_LEARNED_H */
