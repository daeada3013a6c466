/*
 * gkb_batched.h -- many small, uneven partial SVDs in one persistent launch.
 *
 * Each problem is the restarted partial SVD of gkb.h (Golub-Kahan
 * bidiagonalization, eq. (2.1)-(2.4) of the paper, Ritz triplets as in
 * Algorithm 2, thick restart and the same convergence rule), but the whole
 * solve of a problem runs inside one workgroup -- or, for a problem whose
 * cost m * n * k exceeds half of the average per-workgroup share of the batch,
 * inside a team of up to max_team workgroups that split its rows and columns
 * and meet at bounded team barriers: products, two Gram-Schmidt passes, the
 * small SVD of the projected matrix (one-sided Jacobi in LDS, float64),
 * restarts and Ritz vectors.  A persistent grid takes (problem, member)
 * tickets from an atomic queue, largest per-member cost first.  Matrices
 * whose rows are not 16-byte aligned or whose n is not a multiple of 4 are
 * first copied into zero-padded rows inside the workspace.  The queue reset,
 * the copy and the solver are captured once into a hipGraph per plan and
 * replayed by gkb_batched_plan_run.  A team barrier that waits too long
 * (about 10 s) ends that problem with info status GKB_ERR_TIMEOUT.  For tests
 * of that path only, the environment variable GKB_BATCH_STALL_POLLS = P > 0,
 * read when a plan is created, gives that plan's team barriers a target no
 * team meets and a limit of P polls: leave it unset.
 *
 * Problems: GKB_F32, row-major, device pointers, 1 <= r <= k <= min(m, n),
 * k <= 64.  Outputs are packed in problem order:
 *   sigma  device doubles, r_0 + r_1 + ...
 *   U      device floats, problem i at offset sum_{j<i} m_j r_j, column-major m_i x r_i
 *   V      device floats, problem i at offset sum_{j<i} n_j r_j, column-major n_i x r_i
 *   info   host ints, 4 per problem: status (gkb_status), nconv, restarts, matvecs
 * Start vectors: opt->q1_packed (device doubles, problem i at offset
 * sum_{j<i} m_j), or N(2,1) from Philox4x32-10 with key seed + i.
 * Same ownership and validation rules as gkb.h.
 */
#ifndef GKB_BATCHED_H
#define GKB_BATCHED_H

#include "gkb.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int check_every;          /* in-cycle convergence test period (0 = cycle end only) */
  int eps_relative;         /* as gkb_options (default 1)                          */
  double eps_break;         /* 0 = 1e-6                                            */
  uint64_t seed;            /* Philox key base when q1_packed is NULL               */
  const double* q1_packed;  /* device start vectors or NULL                         */
  int workgroups;           /* persistent grid size; 0 = one per compute unit      */
  int no_graph;             /* 1: gkb_batched_plan_run launches directly instead of */
                            /*    replaying the captured graph                      */
  int threads;              /* workgroup size, 512 or 1024; 0 = 1024               */
  int max_team;             /* largest team of workgroups on one problem (1..8);   */
                            /*    0 = 8, 1 = every problem on one workgroup         */
  int form;                 /* compiled form of the products and Gram-Schmidt     */
                            /*    kernels: 0 = by size (out of line when the      */
                            /*    problems average >= 2 MB of A), 1 = inline,      */
                            /*    2 = out of line.  Same results either way.       */
  const double* cost_estimate; /* host, batch doubles or NULL: expected cost of     */
                            /*    each problem on one workgroup (any unit, e.g.    */
                            /*    gkb_batched_plan_work of a run of this batch).   */
                            /*    NULL: m n k.  The schedule splits the costliest  */
                            /*    problems over teams of workgroups and starts the */
                            /*    largest per-member cost first.  Team sizes change */
                            /*    how a problem's sums are split, so results can   */
                            /*    differ from another schedule's by rounding.      */
                            /*    Read during plan creation only.                  */
} gkb_batch_options;

typedef struct gkb_batch_plan_s* gkb_batch_plan;

void gkb_batch_default_options(gkb_batch_options* opt);

/* Workspace bytes for a batch (0 if the problems are invalid). */
size_t gkb_batched_workspace_size(int batch, const gkb_matrix* As, const int* r, const int* k);

/* Validate, upload the problem table into the workspace, capture the launch
   into a hipGraph.  The plan keeps the workspace and output pointers.  The
   persistent kernel comes in two compiled forms, chosen here from the
   batch: the row products and Gram-Schmidt kernels out of line (their own
   registers, more loads in flight) when the problems average at least 2 MB
   of A, inline otherwise; results are the same either way. */
gkb_status gkb_batched_plan_create(int batch, const gkb_matrix* As, const int* r, const int* k, double tol,
                                   int max_restarts, const gkb_batch_options* opt, void* workspace,
                                   size_t ws_bytes, double* sigma, float* U, float* V, void* stream,
                                   gkb_batch_plan* plan);

/* Replay the captured launch on `stream` (asynchronous). */
gkb_status gkb_batched_plan_run(gkb_batch_plan plan, void* stream);

/* Copy the per-problem info of the last completed run to the host (synchronises `stream`). */
gkb_status gkb_batched_plan_info(gkb_batch_plan plan, int* info, void* stream);

/* Per problem, the wall-clock time (ms, from the device clock) that its first
   workgroup spent on it in the last completed run, times its team size: an
   estimate of its cost on one workgroup, for gkb_batch_options.cost_estimate
   of a later plan of the same batch.  work_ms: host, batch doubles
   (synchronises `stream`). */
gkb_status gkb_batched_plan_work(gkb_batch_plan plan, double* work_ms, void* stream);

/* Persistent grid size chosen for the plan. */
int gkb_batched_plan_grid(gkb_batch_plan plan);

void gkb_batched_plan_destroy(gkb_batch_plan plan);

/*
 * Project autotuner for the batched launch: times every candidate on this
 * batch with hipEvents on `stream`, after one untimed run each, and returns
 * the fastest.  Candidates: launch shape (workgroup size 1024 with one
 * workgroup per compute unit, 512 with one, 512 with two, where the LDS
 * allows) x compiled form (inline, out of line; only opt->form if it is
 * non-zero) x team limit (8, 4; only opt->max_team if it is non-zero).
 * The fastest goes to *best_threads, *best_workgroups, *best_form and
 * *best_max_team (the last two may be NULL).  times_ms (optional, room for 12)
 * receives every candidate's time, -1 for a shape the LDS does not allow, in
 * the order shape, then form, then team limit; *ncand their count.  The
 * outputs are written by the runs.  Callers cache the choice (the Python
 * binding keeps a JSON cache keyed by device and batch shape).
 */
gkb_status gkb_batched_autotune(int batch, const gkb_matrix* As, const int* r, const int* k, double tol,
                                int max_restarts, const gkb_batch_options* opt, void* workspace,
                                size_t ws_bytes, double* sigma, float* U, float* V, void* stream,
                                int* best_threads, int* best_workgroups, int* best_form, int* best_max_team,
                                double* times_ms, int* ncand);

/* One call: plan, run, info (host, 4 * batch ints, may be NULL), destroy. */
gkb_status gkb_partial_svd_batched(int batch, const gkb_matrix* As, const int* r, const int* k, double tol,
                                   int max_restarts, const gkb_batch_options* opt, void* workspace,
                                   size_t ws_bytes, double* sigma, float* U, float* V, int* info,
                                   void* stream);

/* Message for the last negative status of a batched call on this thread. */
const char* gkb_batched_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GKB_BATCHED_H */
