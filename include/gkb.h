/*
 * gkb.h -- Golub-Kahan bidiagonalization partial SVD and numerical rank for
 * AMD Instinct MI355X (gfx950).  Plain C ABI: host or device pointers and sizes,
 * no framework types.
 *
 * Method (Godaz, Monsefi, Toutounian, Hosseini, "Accurate and fast matrix
 * factorization for low-rank learning", arXiv:2104.10785):
 *   - Bidiag 1 recurrences, eq. (2.1)-(2.2):
 *       beta_1 q_1 = q,  alpha_1 p_1 = A^T q_1,
 *       beta_{i+1} q_{i+1} = A p_i - alpha_i q_i,
 *       alpha_{i+1} p_{i+1} = A^T q_{i+1} - beta_{i+1} p_i,
 *     with every new vector re-orthogonalised against all previous ones
 *     (Algorithm 1; two classical Gram-Schmidt passes here).
 *   - A P_k = Q_{k+1} B_{k+1,k}, B lower bidiagonal, eq. (2.3)-(2.4).
 *   - Ritz triplets from the SVD of the small projected matrix (eq. (2.13) and
 *     Algorithm 2), left vectors U = Q X, which equals A V / sigma by eq. (2.4).
 *   - Numerical rank: count of singular values of B above a threshold
 *     (Section 3.2, Algorithm 3).
 *   Not in the paper and added here: a convergence tolerance with thick
 *   restart (keep l Ritz pairs and continue the recurrence), relative
 *   breakdown thresholds, a bfloat16 storage mode with a final float32
 *   Rayleigh-Ritz refinement (eq. (5)).
 *
 * Conventions for every entry point
 *   - A is dense, row-major, m x n, leading dimension lda >= n (elements),
 *     in device memory, owned by the caller and never written.
 *   - All device work is enqueued on `stream` (a hipStream_t; NULL = the null
 *     stream).  Calls return after the host part is done: host outputs are
 *     valid on return, device outputs are complete when the stream is.
 *   - The caller owns the workspace (device memory of at least the size the
 *     matching *_workspace_size call returns, 256-byte aligned).  The library
 *     allocates no device memory on these paths.
 *   - Arguments are validated before any device work is enqueued; a negative
 *     status means no output was written.  Positive statuses are warnings
 *     whose outputs are valid (see each status).
 *   - Not thread-safe for concurrent calls that share a workspace.
 */
#ifndef GKB_H
#define GKB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GKB_OK = 0,                /* all requested triplets converged              */
  GKB_NOT_CONVERGED = 1,     /* restarts exhausted; stats.nconv converged,    */
                             /* the rest are the best Ritz approximations     */
  GKB_RANK_DEFICIENT = 2,    /* A has fewer than r singular values above the  */
                             /* breakdown threshold; only those are returned  */
                             /* (later sigma entries and U, V columns are 0)  */
  GKB_ERR_INVALID = -1,      /* bad argument (see gkb_last_error)             */
  GKB_ERR_HIP = -2,          /* a HIP runtime call failed                     */
  GKB_ERR_NUMERIC = -3,      /* NaN or Inf appeared in a norm                 */
  GKB_ERR_WORKSPACE = -4,    /* workspace missing, too small or misaligned    */
  GKB_ERR_TIMEOUT = -5       /* a team of workgroups waited too long for one  */
                             /* of its members (batched form; one-sweep step */
                             /* on rows longer than 24576), which happens    */
                             /* only if the device is not free for the grid. */
                             /* For tests of this path only, the environment */
                             /* variable GKB_TEAM_STALL_POLLS = P > 0 (read  */
                             /* at every team-sweep launch) makes each wait  */
                             /* give up after P polls: leave it unset.       */
} gkb_status;

typedef enum {
  GKB_F64 = 0,   /* A double; bases double; all arithmetic double            */
  GKB_F32 = 1,   /* A float; bases float; products accumulate in float;      */
                 /* Gram-Schmidt coefficients, norms and B in double         */
  GKB_BF16 = 2   /* A bfloat16 (raw 16-bit, round-to-nearest-even of the     */
                 /* float32 matrix); otherwise as GKB_F32                    */
} gkb_dtype;

typedef struct {
  int64_t m, n;              /* rows, columns (>= 1)                          */
  int64_t lda;               /* row stride in elements (>= n)                 */
  gkb_dtype dtype;
  const void* data;          /* device, row-major                             */
  /* GKB_BF16 only: device float32 matrix (same m, n) used for the final
     Rayleigh-Ritz refinement, or NULL for no refinement.                     */
  const float* refine_f32;
  int64_t lda_refine;        /* row stride of refine_f32 (>= n)               */
} gkb_matrix;

typedef struct {
  int keep;            /* restart size l, r <= l < k; 0 = r + (k - r) / 2      */
  int eps_relative;    /* 1: breakdown threshold relative to the largest       */
                       /*    alpha/beta/Ritz value seen so far (default);      */
                       /* 0: absolute (the paper's user-chosen epsilon)        */
  double eps_break;    /* breakdown threshold; 0 = 1e-12 (F64) or 1e-6         */
  const double* q1;    /* device, m doubles: start vector (any nonzero         */
                       /* vector; normalised inside); NULL = q ~ N(2,1)^m      */
                       /* drawn on the device from `seed` (Philox4x32-10)      */
  uint64_t seed;
  int refine_dim;      /* GKB_BF16 with refine_f32: subspace size of the       */
                       /* refinement; 0 = min(k, 2 r)                           */
  int check_every;     /* > 0: also test convergence inside a cycle, after     */
                       /* every check_every right vectors once there are >= r  */
                       /* of them, and stop the cycle when the r largest Ritz  */
                       /* triplets pass (one host synchronisation per test);   */
                       /* 0 = test only at the end of a cycle (fixed k, as the */
                       /* paper's Algorithm 2)                                 */
  int one_pass;        /* 1: read A once per step instead of twice (GKB_F32   */
                       /* or GKB_BF16 with n, lda multiples of 4 or 8,         */
                       /* n <= 262144, or GKB_F64 with n, lda even,            */
                       /* n <= 131072; A 16-byte aligned; float64 rows and     */
                       /* rows longer than 24576 are split over teams of       */
                       /* workgroups that must all be resident, see            */
                       /* GKB_ERR_TIMEOUT; for any other                       */
                       /* A, including sparse A, the two-product step runs and */
                       /* stats.one_pass_used is 0).  One sweep forms          */
                       /* A p and A^T A p in float64; A^T q_{i+1} then follows */
                       /* from eq. (2.2) as (A^T A p - (A^T Q) c) / beta, with */
                       /* c the recurrence and Gram-Schmidt coefficients and   */
                       /* A^T Q kept in float64 (n x (k + 1) more workspace).  */
                       /* Bases are float64 so that A^T Q matches Q exactly;   */
                       /* U, V keep A's class (float32, or float64 for         */
                       /* GKB_F64).  A recovered A^T q column is recomputed    */
                       /* directly once its error bound passes 1e-10 sigma_1,  */
                       /* so with GKB_F64 the results carry errors up to about */
                       /* sqrt(k) 1e-10 sigma_1 (the two-product step: the     */
                       /* float64 rounding level).  Same statuses and stats    */
                       /* (matvecs counts products, two per sweep).            */
                       /* gkb_partial_svd and gkb_numerical_rank.              */
  int phase_timing;    /* 1: time the device phases with HIP events recorded   */
                       /* on `stream` at every phase boundary (a few events    */
                       /* per Golub-Kahan step, read at each host              */
                       /* synchronisation) and fill the ms_matvec ...          */
                       /* ms_other fields of gkb_stats; 0 (default): no events */
                       /* (those fields are then 0)                            */
} gkb_options;

typedef struct {
  int nconv;           /* converged triplets among the returned ones           */
  int restarts;        /* restarts performed                                   */
  int breakdown;       /* 0 none, 1 beta (q side), 2 alpha (p side)            */
  int returned;        /* triplets written (r unless rank deficient)           */
  int64_t matvecs;     /* products with A or A^T (start included)              */
  double max_res_est;  /* max over returned triplets of alpha_res |X[last,i]|  */
  double sigma1_est;   /* largest Ritz value                                   */
  double ms_total;     /* wall time of the call                                */
  double ms_host;      /* of which host small SVDs                             */
  int checks;          /* in-cycle convergence tests performed                 */
  int krylov_dim;      /* right basis vectors in the final projected matrix    */
  int refined;         /* bfloat16 refinement: 1 done, 0 not requested,        */
                       /* -1 skipped (subspace numerically rank deficient)     */
  double ms_refine;    /* wall time of the refinement                          */
  int refreshes;       /* one_pass: A^T q columns recomputed by a direct sweep */
                       /* because their error bound grew too large (counted    */
                       /* in matvecs as well)                                  */
  /* Device time per phase (opt.phase_timing = 1), from consecutive events on  */
  /* the stream, so the five add up to the span from the start vector to the  */
  /* last Ritz vector (ms_total less the host's launch time before the first  */
  /* and after the last event).                                               */
  double ms_matvec;    /* products with A and A^T (the one-sweep pair, the     */
                       /* recovery of A^T q and any direct recomputation)      */
  double ms_reorth;    /* Gram-Schmidt passes, norms, normalisation            */
  double ms_sync;      /* coefficient read-back and the device idle while the  */
                       /* host runs the small SVDs and uploads X, Y            */
  double ms_ritz;      /* restart and Ritz-vector GEMMs (and the bfloat16      */
                       /* refinement)                                          */
  double ms_other;     /* start vector and cycle set-up                        */
  double bytes_A;      /* algorithmic bytes of A streamed: passes over A (two  */
                       /* per step, one per sweep with one_pass, plus          */
                       /* recomputed columns and the start) x the bytes of A   */
                       /* (nonzero values and column indices for sparse A)     */
  int one_pass_used;   /* 1 if the one-sweep step ran (opt.one_pass and an A   */
                       /* it supports), 0 for the two-product step             */
} gkb_stats;

/* Fill *opt with the defaults above. */
void gkb_default_options(gkb_options* opt);

/* Workspace bytes needed by gkb_partial_svd for this problem (0 if the
   arguments are invalid). */
size_t gkb_workspace_size(const gkb_matrix* A, int r, int k, const gkb_options* opt);

/*
 * Top-r singular triplets of A (Algorithm 2 of the paper, with restart).
 *   r, k     1 <= r <= k <= min(m, n); k is the Krylov dimension (number of
 *            right basis vectors per cycle, Algorithm 1's k).
 *   tol      triplet i is converged when ||A^T u_i - sigma_i v_i||, as given
 *            by alpha_res |X[last, i]| from eq. (2.4), is <= tol * sigma_1.
 *   max_restarts  0 reproduces the paper's one-shot Algorithm 2.
 *   sigma    host, r doubles, descending.
 *   U        device, column-major m x r (u_i contiguous at U + i*m);
 *            double for GKB_F64, float otherwise.
 *   V        device, column-major n x r, same element type.
 *   stats    host, optional (NULL).
 * Singular vectors are determined up to a common sign of (u_i, v_i).
 * GKB_BF16 with A->refine_f32: the Golub-Kahan cycles run on the bfloat16
 * matrix; the top d = refine_dim (default 2r, at most the Krylov dimension)
 * Ritz vectors then span a Rayleigh-Ritz projection with the float32 matrix
 * (eq. (5)): W = A32 V_d (MFMA), W^T W = R^T R (float64 Cholesky), R = X S Y^T,
 * sigma = S, V = V_d Y, U = W R^-1 X.  Convergence status refers to the
 * bfloat16 solve.
 */
gkb_status gkb_partial_svd(const gkb_matrix* A, int r, int k, double tol, int max_restarts,
                           const gkb_options* opt, void* workspace, size_t ws_bytes,
                           double* sigma, void* U, void* V, gkb_stats* stats, void* stream);

/*
 * gkb_partial_svd without a workspace argument, for callers that cannot
 * allocate device memory (code that must not call hipMalloc: tight serving
 * loops, harnesses that forbid allocation, work prepared for later capture).
 * The workspace is a fixed device array inside the library,
 * GKB_NOALLOC_SCRATCH_BYTES (32 MiB) per GPU, held from the first call on a
 * GPU until the process ends; the call uses the array of the current device
 * (the stream must belong to it).  Problems whose gkb_workspace_size exceeds
 * it are rejected with GKB_ERR_WORKSPACE before any device work.  Arguments,
 * results, statuses and stats are those of gkb_partial_svd with the same
 * options, and the kernels are the same (every solve initialises the scratch
 * contents it reads).  All calls on one GPU share the array: calls that
 * overlap on one GPU (two host threads, or two streams whose work overlaps)
 * race and give undefined results; serialise them.  The call allocates no
 * device or pinned memory; opt->phase_timing (which creates HIP events) is
 * rejected with GKB_ERR_INVALID.
 */
#define GKB_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
gkb_status gkb_partial_svd_noalloc(const gkb_matrix* A, int r, int k, double tol, int max_restarts,
                                   const gkb_options* opt, double* sigma, void* U, void* V, gkb_stats* stats,
                                   void* stream);

/*
 * Plans: repeated solves of one matrix buffer (the same A pointer, shape and
 * type, the same workspace and options; the contents of A may change between
 * solves, as in a sequence of slowly changing matrices).  The device work
 * between two host synchronisations of a solve -- the Golub-Kahan steps of a
 * cycle up to the next convergence test (Algorithm 1 inside Algorithm 2) --
 * is captured as a HIP graph the first time a solve reaches it and replayed by
 * later solves, so a solve launches one graph per stretch instead of a dozen
 * kernels per step; host decisions (tests, restarts) are as in
 * gkb_partial_svd, whose results a plan reproduces bitwise.
 *   gkb_svd_plan_create  checks the arguments as gkb_partial_svd does (the
 *                        workspace stays the caller's and must outlive the
 *                        plan); opt->phase_timing is not available
 *                        (GKB_ERR_INVALID).  Creates one HIP stream (for the
 *                        captures).
 *   gkb_svd_plan_run     one solve: q1 (device, m doubles) replaces the
 *                        start vector of the options when non-NULL; sigma,
 *                        U, V, stats and statuses as gkb_partial_svd.  The
 *                        graphs launch on `stream`.  Not thread-safe for one
 *                        plan.
 *   gkb_svd_plan_destroy releases the graphs and the stream (NULL allowed).
 */
typedef struct gkb_svd_plan_s* gkb_svd_plan;
gkb_status gkb_svd_plan_create(const gkb_matrix* A, int r, int k, double tol, int max_restarts,
                               const gkb_options* opt, void* workspace, size_t ws_bytes, gkb_svd_plan* plan);
gkb_status gkb_svd_plan_run(gkb_svd_plan plan, const double* q1, double* sigma, void* U, void* V,
                            gkb_stats* stats, void* stream);
void gkb_svd_plan_destroy(gkb_svd_plan plan);

/* Workspace bytes needed by gkb_numerical_rank. */
size_t gkb_rank_workspace_size(const gkb_matrix* A, int k_max, const gkb_options* opt);

/*
 * Numerical rank #{ sigma_i > tau } (Section 3.2 and Algorithm 3).
 *   tau          threshold on singular values (> 0); Algorithm 3's epsilon
 *                is on eigenvalues of B^T B, i.e. epsilon = tau^2.
 *   tau_relative 1: tau is relative to sigma_1 of B; 0: absolute.
 *   k_max        maximum Bidiag 1 steps, 1..min(m, n); 0 = min(m, n).
 *                The recurrence stops early at a breakdown.
 *   rank         host: count of singular values of B above the threshold.
 *   rank_sturm   host, optional: the same count by Sylvester inertia of the
 *                Golub-Kahan tridiagonal (an independent check).
 *   sigma_out    host, optional, k_max doubles: singular values of B.
 *   nsigma       host, optional: number written to sigma_out (steps done).
 *   opt          eps_break / eps_relative (breakdown), q1 / seed (start
 *                vector), one_pass (one sweep of A per step, as for
 *                gkb_partial_svd); the other fields are not used.
 */
gkb_status gkb_numerical_rank(const gkb_matrix* A, double tau, int tau_relative, int k_max,
                              const gkb_options* opt, void* workspace, size_t ws_bytes,
                              int64_t* rank, int64_t* rank_sturm, double* sigma_out,
                              int* nsigma, gkb_stats* stats, void* stream);

/* Human-readable name of a status. */
const char* gkb_status_string(gkb_status s);

/* Message for the last negative status returned on this thread ("" if none). */
const char* gkb_last_error(void);

/* ------------------------------------------------------------------------
 * Host utility (no device work): the dense float64 SVD the library runs on
 * the projected matrix each cycle, exposed so it can be checked on its own.
 * H is nq x np row-major; kk = min(nq, np).  Writes s (kk, descending),
 * X (nq x kk row-major) and Y (np x kk row-major) with H = X diag(s) Y^T.
 * Householder reduction to bidiagonal form followed by implicit-shift QR
 * sweeps (Golub and Kahan 1965; Golub and Reinsch 1970).
 * Returns GKB_OK, GKB_ERR_INVALID, or GKB_ERR_NUMERIC (no convergence or
 * non-finite input).
 * ------------------------------------------------------------------------ */
gkb_status gkb_host_dense_svd(int nq, int np, const double* H, double* s, double* X, double* Y);

/* Host utility: number of singular values above tau (> 0) of the lower
   bidiagonal with diagonal alpha[0..np) and subdiagonal beta[0..nq-1),
   nq in {np, np+1}, by Sylvester inertia of its Golub-Kahan tridiagonal. */
int64_t gkb_host_bidiag_count_above(int nq, int np, const double* alpha, const double* beta,
                                    double tau);

/* Host utility (no device work): the screening step of the in-cycle
 * convergence test.  For the (np + 1) x np lower bidiagonal B of a first
 * Golub-Kahan cycle (diagonal alpha[0..np) = the alphas, subdiagonal
 * beta[0..np) = the betas of eq. (2.3)), writes its singular values s (np,
 * descending) and last[i] = the last entry of the i-th left singular vector
 * (its sign is that of the pair (u_i, v_i)), which with eq. (2.4) gives the
 * residual estimate alpha_res |last[i]| without the singular vectors:
 * rows rotated to upper bidiagonal form, then implicit-shift QR sweeps that
 * carry that one row, O(np^2).  Returns GKB_OK, GKB_ERR_INVALID (np < 1 or a
 * NULL pointer) or GKB_ERR_NUMERIC (no convergence or non-finite input).
 */
gkb_status gkb_host_bidiag_lastrow(int np, const double* alpha, const double* beta, double* s, double* last);

#ifdef __cplusplus
}
#endif
#endif /* GKB_H */
