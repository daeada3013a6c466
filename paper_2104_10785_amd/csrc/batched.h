// Batched persistent solver: device-side problem table and launch (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gkb {

constexpr int BATCH_KMAX = 64;  // largest Krylov dimension of a batched problem
constexpr int BATCH_TEAM_NMAX = 4096;  // largest n of a problem solved by a team of workgroups

struct BatchProblem {
  const float* A;     // row-major m x n, float32 (the caller's, or its staged copy)
  int64_t lda;
  int m, n, r, k, l;  // rows, columns, wanted triplets, Krylov dimension, restart size
  int index;          // position in the caller's arrays
  int ldq, ldp;       // column strides of the Q and P bases (multiples of 4)
  int padded;         // 1: A is a staged copy whose rows are zero-padded to a multiple of 4
  int team;           // workgroups solving this problem together (1 = alone)
  int team_id;        // index of its barrier counter (teams of more than one)
  int64_t offTeam;    // double offset of its team buffers: T x n partial products, 2 x T x (KMAX + 4) dots
  int64_t offQ, offP; // float offsets of the two Q and two P buffers in the pool
  int64_t offW;       // double offset of w (m) and z (n) in the work area
  int64_t offU, offV; // float offsets of U (m x r) and V (n x r) in the outputs
  int64_t offS;       // double offset of sigma (r)
  int64_t offQ1;      // double offset of this problem's start vector in q1 (if given)
};

// One matrix to stage: rows [row_start, row_start + m) of the flattened row
// range; src (lds) -> dst (ldd = 4 ceil(n / 4), zero padding).
struct StageCopy {
  const float* src;
  float* dst;
  int64_t lds, ldd, row_start;
  int m, n;
};

struct BatchParams {
  const BatchProblem* problems;
  const int* order;   // ticket -> problem (largest per-member cost first, a team's tickets adjacent)
  const int* member;  // ticket -> member index within the problem's team
  int* counter;       // work-queue head
  int batch;
  int ntickets;
  float* pool;
  double* work;
  float* U;
  float* V;
  double* sigma;
  int* info;          // 4 ints per problem: status, nconv, restarts, matvecs
  unsigned long long* ticks;  // per problem: device wall-clock ticks its first member spent on it
  const double* q1;   // packed start vectors or null (Philox with seed + index)
  uint64_t seed;
  double eps_break;
  double tol;
  int max_restarts;
  int check_every;
  int relative;
  const StageCopy* stage;  // matrices copied to aligned rows before the solves
  int nstage;
  int64_t stage_rows;
  int* team_cnt;           // barrier counters, one per team (zeroed before each run)
  int nteams;
  double* team_buf;        // team reduction buffers
  int outline;             // 1: products and Gram-Schmidt kernels out of line (long rows)
  long spin_limit;         // polls of a team barrier before it gives up (BATCH_TEAM_SPIN_LIMIT)
  int barrier_skew;        // 0; 1 only in tests of the timeout path (no barrier can be met)
};

// Bound on the polls of a team barrier (each poll sleeps ~100 cycles and
// reads one counter: about 10 s in all).  The environment variable
// GKB_BATCH_STALL_POLLS = P > 0, read when a plan is made, sets the bound to
// P and the barrier skew to 1, so every team barrier times out (for tests of
// that path; every kernel still runs to its end).
constexpr long BATCH_TEAM_SPIN_LIMIT = 1L << 23;

// threads per workgroup: 512 or 1024
size_t batched_lds_bytes(int threads);
hipError_t batched_setup();
hipError_t launch_batched(const BatchParams& prm, int grid, int threads, hipStream_t st);

}  // namespace gkb
