// One sweep of A for both products of a Golub-Kahan step, and the small
// kernels of the one-pass step (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gkb {

constexpr int64_t FUSED_NMAX = 24576;    // longest row of the single-workgroup sweep (768 threads x 8 groups of 4 floats)
constexpr int64_t FUSED_TEAM_NMAX = 262144;   // longest float32 or bfloat16 row of the team sweep (32 x 8192 columns)
constexpr int64_t FUSED_TEAM_NMAX_F64 = 131072;   // the same for float64 rows (32 members x 4096 columns)
// a recovered A^T q column is recomputed directly once its error bound
// exceeds this fraction of the largest coefficient seen
constexpr double ONEPASS_TAU = 1e-10;

// true if A (m x n, lda; dtype 0 = float64, 1 = float32, 2 = bfloat16) can
// take the fused sweep: n and lda multiples of the 16-byte group (2, 4 or 8
// elements), A 16-byte aligned, and either float32 or bfloat16 rows of at
// most FUSED_NMAX (one workgroup per row range) or a team shape (rows longer
// than that, or float64 rows: n <= FUSED_TEAM_NMAX, FUSED_TEAM_NMAX_F64 for
// float64, and at most one member per compute unit)
bool fused_ok(int64_t m, int64_t n, int64_t lda, const void* A, int dtype);
// whether the sweep of this row length and type is the team form
inline bool team_form(int64_t n, int dtype) { return dtype == 0 || n > FUSED_NMAX; }
// number of partial-sum rows the sweep writes (workgroups, or teams)
int fused_blocks(int64_t m, int64_t n, int dtype);

// The team sweep: C members per team, each owning a near-equal slice of at
// most 8192 columns (4096 for float64, 16384 for bfloat16: 32 KB of a row in
// each case); teams of
// rpt rows (the last may be shorter, none empty), nsteps steps of rows per
// team; C = 0 if the shape has no team form.
struct TeamShape {
  int C, nteams, rpt, nsteps;
};
TeamShape team_shape(int64_t m, int64_t n, int dtype);
// device bytes of the team sweep's mailbox and counters (0 if no team form);
// the sweep's `team` argument points to this many bytes, 256-byte aligned,
// zeroed by launch_team_reset before the first sweep and then left to the
// sweeps (each launch leaves it ready for the next)
size_t team_bytes(int64_t m, int64_t n, int dtype);
hipError_t launch_team_reset(void* team, int64_t m, int64_t n, int dtype, hipStream_t st);

// A float32 (dtype 1), bfloat16 (dtype 2, widened exactly to float32) or
// float64 (dtype 0, team sweep only).  With win == nullptr: w = A p (float64,
// m) and the partials of y = A^T w; for float32 and bfloat16 A, p is read as
// float32 (a float64 p is rounded to float32 once, so w and y are the exact
// products with that float32 vector); for float64 A, p is read as it is.  With win != nullptr: the
// partials of y = A^T win (p, w unused).  All sums in float64; ypart holds
// fused_blocks(m, n, dtype) x ldy doubles (ldy >= n); y (n doubles) gets their sum in
// a fixed order unless y is null.  Skipped when flag[0] != 0, or when run_if
// is given and run_if[0] == 0.  With qprev given, w = A p - coef[0] qprev
// (the recurrence term of eq. (2.2)) while y stays A^T (A p).  The team form
// (team_form) needs `team` (team_bytes(m, n, dtype) bytes, see
// launch_team_reset) and may set flag[0] = 4 when a member waited
// too long for the others (its results are then NaN); flag must be writable
// device memory or null.
template <typename TP>
hipError_t launch_gemv_fused(const void* A, int dtype, int64_t lda, int64_t m, int64_t n, const TP* p,
                             const double* win, double* w, double* y, double* ypart, int64_t ldy, const int* flag,
                             hipStream_t st, const int* run_if = nullptr, const double* qprev = nullptr,
                             const double* coef = nullptr, void* team = nullptr);
template <typename TP>
hipError_t launch_gemv_fused_team(const void* A, int dtype, int64_t lda, int64_t m, int64_t n, const TP* p,
                                  const double* win, double* w, double* ypart, int64_t ldy, const int* flag,
                                  hipStream_t st, const int* run_if, const double* qprev, const double* coef,
                                  void* team);

// The recovery of A^T q_tq after w = A p - Q[:, 0..t) c_tot has been
// normalised to beta q_tq, with c_tot[j] = c[j] plus xc[j - x0] for
// x0 <= j < x0 + nx (the recurrence term: alpha on one column, or rho on the
// first l after a restart):
//   g = (y - G[:, 0..t) c_tot) / beta[0], G[:, tq] = g, z = g - beta[0] pprev,
// y summed from the sweep's partials.  Its guard (one thread):
//   e = (sum_j |c_tot[j]| err[j] + eps0 (s^2 + s sum_j |c_tot[j]|)) / beta[0],
//   s = sig[0]; if e > tau s: refresh[0] = 1, refresh[1] += 1,
//   err[tq] = eps0 s (the column is then recomputed by a direct sweep); else
//   refresh[0] = 0, err[tq] = e.
// With `norm` given, the same launch first normalises the left vector: beta =
// the norm of norm->x from its partial sums of squares (breakdown and
// non-finite tests as the normalisation kernel, flag set on either, and then
// nothing is recovered), norm->out = norm->x / beta, norm->coef_out = beta,
// norm->sig_out = max(sig_in, beta); beta and s then come from there (beta
// and sig are not read).
struct NormArgs {
  const double* x = nullptr;        // the orthogonalised vector (len)
  int64_t len = 0;
  const double* normpart = nullptr;  // its partial sums of squares
  int nparts = 0;
  double* out = nullptr;             // the new basis column
  double* coef_out = nullptr;        // beta
  const double* sig_in = nullptr;    // running largest coefficient, before
  double* sig_out = nullptr;         // and after this vector
  double eps = 0.0;                  // breakdown threshold
  int relative = 1;
  int code = 1;                      // flag[0] on breakdown
  int index = 0;                     // flag[1] on breakdown
};
hipError_t launch_onepass_recover(const double* ypart, int nb, int64_t ldy, double* G, int64_t ldg, int t,
                                  const double* c, const double* xc, int x0, int nx, const double* beta, int tq,
                                  const double* pprev, double* z, int64_t n, double* err, const double* sig,
                                  double eps0, double tau, int* refresh, int* flag, hipStream_t st,
                                  const NormArgs* norm = nullptr);
// err[idx] = eps0 * sig[0]
hipError_t launch_err_set(double* err, int idx, const double* sig, double eps0, const int* flag, hipStream_t st);
// dst[0..l) = sqrt(nq) * max(src[0..nq)) (columns of G X after a restart)
hipError_t launch_err_restart(const double* src, int nq, double* dst, int l, hipStream_t st);
// if refresh[0]: G[:, tq] = y (summed from the partials), z = y - beta[0] pprev
hipError_t launch_onepass_fix(const double* ypart, int nb, int64_t ldy, double* G, int64_t ldg, int tq,
                              const double* beta, const double* pprev, double* z, int64_t n, const int* flag,
                              const int* refresh, hipStream_t st);
// dst[i] = (float) src[i], i < len
hipError_t launch_narrow(const double* src, int64_t len, float* dst, hipStream_t st);

}  // namespace gkb
