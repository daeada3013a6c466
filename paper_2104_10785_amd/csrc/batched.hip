// Batched partial SVD: many small, uneven problems in one persistent launch.
//
// A problem is solved end to end -- the Golub-Kahan recurrences of
// eq. (2.1)-(2.2) with CGS2 reorthogonalisation, the small SVD of the
// projected matrix (one-sided Jacobi in LDS, float64), the convergence test,
// thick restarts and the Ritz vectors V = P Y, U = Q X (Algorithm 2) -- by a
// team of T workgroups (T = 1 for most problems).  Member j of a team owns
// rows [j m / T, (j + 1) m / T) of A, Q, w and U and entries
// [j n / T, (j + 1) n / T) of P, z and V; the partial sums of the products
// and of the Gram-Schmidt dots meet in a per-team buffer and are added in
// member order after a team barrier, so every member holds the same
// coefficients and takes the same decisions (and runs the same small SVD).
// Workgroups take (problem, member) tickets from an atomic queue ordered by
// per-member cost, largest first.  Every wait is bounded; every wave of the
// grid reaches the queue's end, so the grid drains; all reductions have a
// fixed order, so a result does not depend on which workgroups solved it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "../../include/gkb.h"
#include "batched.h"

namespace gkb {

namespace {

constexpr int KMAX = BATCH_KMAX;   // max Krylov dimension
constexpr int HLD = KMAX + 2;      // LDS leading dimension of H columns
constexpr int SLD = KMAX + 4;      // per-member stride of the small team reduction buffers

// Pointers taken from the problem table are generic; the hot loops cast them
// to the global (or LDS) address space so that the compiler emits global
// loads with a scalar base instead of flat loads.
#define GMEM __attribute__((address_space(1)))
#define LMEM __attribute__((address_space(3)))
typedef float f4 __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ const GMEM T* gc(const T* p) {
  return (const GMEM T*)p;
}
template <typename T>
__device__ __forceinline__ GMEM T* gw(T* p) {
  return (GMEM T*)p;
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// BT = threads per workgroup (512 or 1024), NW = waves per workgroup.
template <int BT>
struct Lds {
  static constexpr int NW = BT / 64;
  double red[NW];
  double h[KMAX + 2];          // Gram-Schmidt coefficients / rho
  double qc[KMAX + 2];         // beta of Q column j
  double pc[KMAX + 2];         // alpha of P column j
  double sres[KMAX + 2];       // Ritz values kept at a restart
  double rho[KMAX + 2];
  double Hs[KMAX * HLD];       // projected matrix, column-major (col j at Hs + j*HLD)
  double Vs[KMAX * KMAX];      // right rotations (col j at Vs + j*KMAX)
  double sv[KMAX];             // column norms after Jacobi (sorted via perm)
  double scal;                 // team-reduced scalar
  float tpart[4 * BT];         // gemv_t row-group partial sums
  float pvec[BATCH_TEAM_NMAX]; // a team's current p (read from the coherence point)
  int perm[KMAX];
  int rotated;
  int problem;
  int member;
  int flag;                    // breakdown: 0 none, 1 beta, 2 alpha, 3 numeric
  int flag_idx;
  int team_fail;               // a team barrier timed out
};

// Block-wide sum in a fixed order (all threads get the result).
template <int BT>
__device__ double block_sum(double v, Lds<BT>& L) {
  v = wsum(v);
  constexpr int NW = BT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) L.red[wave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) t += L.red[w];
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------- teams
struct Team {
  int T, member;
  int* cnt;        // arrivals at this team's barriers (zeroed before the launch)
  double* zpart;   // T x n partial sums of A^T q
  double* small;   // 2 x T x SLD partial dots / norms (alternating regions)
  int nbar;        // barriers this member has passed
  int parity;
  long spin_limit; // polls before a barrier gives up (BatchParams)
  int skew;        // added to a barrier's target (0; 1 only in tests of the timeout path)
};

// Data that members exchange (partial sums, the entries of p) is written and
// read with device-scope accesses (cst / ldc below), which go to the device's
// coherence point instead of an XCD's own L2.  A barrier: every wave waits
// until its own stores have completed, the workgroup meets, one thread counts
// the arrival and polls until all T members have arrived (or the wait timed
// out, which marks the solve as failed and makes every later barrier return
// at once), and the workgroup meets again.  (A full agent-scope fence per
// barrier -- an L2 write-back and invalidate -- costs ~70 us here; this form
// costs 4-11 us for teams of 2-8.)
__device__ __forceinline__ void cst(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void cst(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ldc(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ldc(const float* p) {
  return __hip_atomic_load(const_cast<float*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int BT>
__device__ void team_barrier(Team& tm, Lds<BT>& L) {
  __builtin_amdgcn_s_waitcnt(0);   // this wave's stores have completed
  __syncthreads();
  ++tm.nbar;
  if (threadIdx.x == 0 && !L.team_fail) {
    __hip_atomic_fetch_add(tm.cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int target = tm.nbar * tm.T + tm.skew;
    long polls = 0;
    while (__hip_atomic_load(tm.cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (++polls > tm.spin_limit) {
        L.team_fail = 1;
        break;
      }
    }
  }
  __syncthreads();
}

// v[0..len) (LDS, this member's partial sums) <- the sum over members, in member order.
template <int BT>
__device__ void team_sum(double* v, int len, Team& tm, Lds<BT>& L) {
  if (tm.T == 1) return;
  double* region = tm.small + (int64_t)tm.parity * tm.T * SLD;
  for (int i = threadIdx.x; i < len; i += BT) cst(region + tm.member * SLD + i, v[i]);
  team_barrier(tm, L);
  for (int i = threadIdx.x; i < len; i += BT) {
    double s = 0.0;
    for (int mm = 0; mm < tm.T; ++mm) s += ldc(region + mm * SLD + i);
    v[i] = s;
  }
  tm.parity ^= 1;
  __syncthreads();
}

template <int BT>
__device__ double team_sum_scalar(double x, Team& tm, Lds<BT>& L) {
  if (tm.T == 1) return x;
  if (threadIdx.x == 0) L.scal = x;
  __syncthreads();
  team_sum(&L.scal, 1, tm, L);
  const double r = L.scal;
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- products
// w[i] = A[i, :] p - c * qprev[i] for rows i in [lo, hi) (qprev may be null);
// each wave owns 4 rows at a time, lanes stride the columns with 16-byte
// loads (4 rows x 2 vectors in flight).
// p is in LDS (PLDS, a team's copy) or in global memory.
template <int BT, bool PLDS>
__device__ void bgemv_n_body(const BatchProblem& P, const float* p_, const float* qprev_, double c, double* w_, int lo,
                        int hi) {
  constexpr int NW = BT / 64;
  constexpr int R = 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool vec = ((P.lda & 3) == 0) && ((reinterpret_cast<uintptr_t>(P.A) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(p_) & 15) == 0);
  using PT = typename std::conditional<PLDS, const LMEM float*, const GMEM float*>::type;
  using P4 = typename std::conditional<PLDS, const LMEM f4*, const GMEM f4*>::type;
  const PT p = (PT)p_;
  const GMEM float* qprev = gc(qprev_);
  GMEM double* w = gw(w_);
  const GMEM float* A = gc(P.A);
  for (int i0 = lo + wave * R; i0 < hi; i0 += NW * R) {
    const GMEM float* rows[R];
#pragma unroll
    for (int r = 0; r < R; ++r) rows[r] = A + (int64_t)min(i0 + r, hi - 1) * P.lda;
    // lane r < R fetches qprev of row i0 + r now, so that writing the row's
    // result after its reduction does not wait for a load
    const float qp = (qprev_ != nullptr && lane < R && i0 + lane < hi) ? qprev[i0 + lane] : 0.f;
    float a[R] = {};
    int jt = 0;
    if (vec) {
      const int nv = P.n >> 2;
      for (int v0 = lane; v0 < nv; v0 += 128) {
        const int v1 = v0 + 64;
        const bool ok1 = v1 < nv;
        const f4 p0 = ((P4)p)[v0];
        f4 p1 = {0.f, 0.f, 0.f, 0.f};
        if (ok1) p1 = ((P4)p)[v1];
        f4 x0[R], x1[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          x0[r] = ((const GMEM f4*)rows[r])[v0];
          x1[r] = f4{0.f, 0.f, 0.f, 0.f};
          if (ok1) x1[r] = ((const GMEM f4*)rows[r])[v1];
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
          a[r] += x0[r].x * p0.x + x0[r].y * p0.y + x0[r].z * p0.z + x0[r].w * p0.w +
                  x1[r].x * p1.x + x1[r].y * p1.y + x1[r].z * p1.z + x1[r].w * p1.w;
      }
      jt = nv << 2;
    }
    for (int j = jt + lane; j < P.n; j += 64) {
      const float pj = p[j];
#pragma unroll
      for (int r = 0; r < R; ++r) a[r] += rows[r][j] * pj;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double sr = wsum((double)a[r]);
      if (lane == r && i0 + r < hi) w[i0 + r] = sr - (qprev_ ? c * (double)qp : 0.0);
    }
  }
  __syncthreads();
}

// out[j] = sum_{i in [lo, hi)} A[i, j] q[i] - c * pprev[j] for all j < n
// (pprev may be null); threads own 4-column groups, G row groups split the
// rows (8 rows in flight per thread), partial sums meet in LDS and are added
// in group order.
template <int BT, bool COHERENT, bool DEEP>
__device__ void bgemv_t_body(const BatchProblem& P, const float* q_, const float* pprev_, double c, double* out, int lo,
                        int hi, Lds<BT>& L) {
  const int tid = threadIdx.x;
  const GMEM float* q = gc(q_);
  const GMEM float* pprev = gc(pprev_);
  // 16-byte loads need aligned rows; columns n .. 4 ceil(n / 4) - 1 must be
  // readable (the plan stages every matrix that does not satisfy this)
  const bool vec = ((P.lda & 3) == 0) && ((reinterpret_cast<uintptr_t>(P.A) & 15) == 0) &&
                   (((P.n & 3) == 0) || P.padded);
  const int VN = vec ? 4 : 1;
  const int ncg = (P.n + VN - 1) / VN;
  const int npad = ncg * VN;               // row stride of the partial sums
  const int G = ncg >= BT ? 1 : BT / ncg;  // G * npad <= 4 * BT
  const int g = ncg >= BT ? 0 : tid / ncg;
  for (int cg = ncg >= BT ? tid : tid % ncg; cg < ncg && g < G; cg += (ncg >= BT ? BT : ncg)) {
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    const GMEM float* base = gc(P.A) + cg * VN;
    int i = lo + g;
    if (vec) {
      // TR rows in flight per thread (16 TR bytes): enough outstanding loads
      // per CU to keep streaming when every CU competes for HBM
      constexpr int TR = DEEP ? 16 : 8;
      for (; i + (TR - 1) * G < hi; i += TR * G) {
        f4 a[TR];
        float qq[TR];
#pragma unroll
        for (int u = 0; u < TR; ++u) {
          qq[u] = q[i + u * G];
          a[u] = *(const GMEM f4*)(base + (int64_t)(i + u * G) * P.lda);
        }
#pragma unroll
        for (int u = 0; u < TR; ++u) {
          acc[0] += a[u].x * qq[u];
          acc[1] += a[u].y * qq[u];
          acc[2] += a[u].z * qq[u];
          acc[3] += a[u].w * qq[u];
        }
      }
      for (; i < hi; i += G) {
        const float qi = q[i];
        const f4 a0 = *(const GMEM f4*)(base + (int64_t)i * P.lda);
        acc[0] += a0.x * qi;
        acc[1] += a0.y * qi;
        acc[2] += a0.z * qi;
        acc[3] += a0.w * qi;
      }
    } else {
      for (; i + 3 * G < hi; i += 4 * G)
        acc[0] += base[(int64_t)i * P.lda] * q[i] + base[(int64_t)(i + G) * P.lda] * q[i + G] +
                  base[(int64_t)(i + 2 * G) * P.lda] * q[i + 2 * G] + base[(int64_t)(i + 3 * G) * P.lda] * q[i + 3 * G];
      for (; i < hi; i += G) acc[0] += base[(int64_t)i * P.lda] * q[i];
    }
    if (ncg >= BT) {
      for (int e = 0; e < VN; ++e) {
        const int j = cg * VN + e;
        if (j < P.n) {
          const double o = (double)acc[e] - (pprev_ ? c * (double)pprev[j] : 0.0);
          if (COHERENT) cst(out + j, o);
          else out[j] = o;
        }
      }
    } else {
      for (int e = 0; e < VN; ++e) L.tpart[g * npad + cg * VN + e] = acc[e];
    }
  }
  __syncthreads();
  if (ncg < BT) {
    for (int j = tid; j < P.n; j += BT) {
      double s = 0.0;
      for (int gg = 0; gg < G; ++gg) s += (double)L.tpart[gg * npad + j];
      const double o = s - (pprev_ ? c * (double)pprev[j] : 0.0);
      if (COHERENT) cst(out + j, o);
      else out[j] = o;
    }
    __syncthreads();
  }
}

// The products in two forms: inline, or out of line (OUT), where they get
// registers of their own instead of sharing the solver's: worth a call's
// register save and restore when the rows are long enough to stream from HBM
// (on short, cache-resident problems the calls cost more than they save).
// Out of line they also keep more loads in flight (DEEP), which inline
// would only add to the solver's spills.
template <int BT, bool PLDS>
__device__ __noinline__ void bgemv_n_ool(const BatchProblem& P, const float* p_, const float* qprev_, double c,
                                         double* w_, int lo, int hi) {
  bgemv_n_body<BT, PLDS>(P, p_, qprev_, c, w_, lo, hi);
}
template <int BT, bool OUT, bool PLDS>
__device__ __forceinline__ void bgemv_n(const BatchProblem& P, const float* p_, const float* qprev_, double c,
                                        double* w_, int lo, int hi) {
  if constexpr (OUT) bgemv_n_ool<BT, PLDS>(P, p_, qprev_, c, w_, lo, hi);
  else bgemv_n_body<BT, PLDS>(P, p_, qprev_, c, w_, lo, hi);
}
template <int BT, bool COHERENT>
__device__ __noinline__ void bgemv_t_ool(const BatchProblem& P, const float* q_, const float* pprev_, double c,
                                         double* out, int lo, int hi, Lds<BT>& L) {
  bgemv_t_body<BT, COHERENT, true>(P, q_, pprev_, c, out, lo, hi, L);
}
template <int BT, bool OUT, bool COHERENT = false>
__device__ __forceinline__ void bgemv_t(const BatchProblem& P, const float* q_, const float* pprev_, double c,
                                        double* out, int lo, int hi, Lds<BT>& L) {
  if constexpr (OUT) bgemv_t_ool<BT, COHERENT>(P, q_, pprev_, c, out, lo, hi, L);
  else bgemv_t_body<BT, COHERENT, false>(P, q_, pprev_, c, out, lo, hi, L);
}

// z[j] = (A^T q)[j] - c * pprev[j] for this member's entries j in [plo, phi);
// q is read on the member's rows [qlo, qhi) only.
template <int BT, bool OUT>
__device__ void team_gemv_t(const BatchProblem& P, const float* q, const float* pprev, double c, double* z,
                            int qlo, int qhi, int plo, int phi, Team& tm, Lds<BT>& L) {
  if (tm.T == 1) {
    bgemv_t<BT, OUT>(P, q, pprev, c, z, 0, P.m, L);
    return;
  }
  double* mine = tm.zpart + (int64_t)tm.member * P.n;
  bgemv_t<BT, OUT, true>(P, q, nullptr, 0.0, mine, qlo, qhi, L);
  team_barrier(tm, L);
  for (int j = plo + threadIdx.x; j < phi; j += BT) {
    double s = 0.0;
    for (int mm = 0; mm < tm.T; ++mm) s += ldc(tm.zpart + (int64_t)mm * P.n + j);
    z[j] = s - (pprev ? c * (double)pprev[j] : 0.0);
  }
  __syncthreads();
}

// ---------------------------------------------------------------- Gram-Schmidt
// L.h[j] = V[lo:hi, j] . x[lo:hi] for j < t (waves own columns, lanes own rows).
template <int BT, bool DEEP>
__device__ void bdots_body(const float* V_, int ldv, int t, int lo, int hi, const double* x_, Lds<BT>& L) {
  constexpr int NW = BT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const GMEM float* V = gc(V_);
  const GMEM double* x = gc(x_);
  constexpr int U = DEEP ? 8 : 1;   // rows in flight per lane; the sum keeps its sequential order
  for (int j = wave; j < t; j += NW) {
    const GMEM float* col = V + (int64_t)j * ldv;
    double a = 0.0;
    int i = lo + lane;
    for (; i + (U - 1) * 64 < hi; i += U * 64) {
      float v[U];
      double xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        v[u] = col[i + u * 64];
        xv[u] = x[i + u * 64];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) a += (double)v[u] * xv[u];
    }
    for (; i < hi; i += 64) a += (double)col[i] * x[i];
    a = wsum(a);
    if (lane == 0) L.h[j] = a;
  }
  __syncthreads();
}

// x[lo:hi] -= V[lo:hi, 0:t] h; returns the member's part of ||x||^2 after the update.
template <int BT, bool DEEP>
__device__ double bupdate_body(const float* V_, int ldv, int t, int lo, int hi, double* x_, const double* h, Lds<BT>& L) {
  const GMEM float* V = gc(V_);
  GMEM double* x = gw(x_);
  double ss = 0.0;
  constexpr int U = DEEP ? 8 : 1;   // columns in flight per thread; the update keeps its sequential order
  for (int i = lo + threadIdx.x; i < hi; i += BT) {
    double xi = x[i];
    int j = 0;
    for (; j + U <= t; j += U) {
      float v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = V[(int64_t)(j + u) * ldv + i];
#pragma unroll
      for (int u = 0; u < U; ++u) xi -= (double)v[u] * h[j + u];
    }
    for (; j < t; ++j) xi -= (double)V[(int64_t)j * ldv + i] * h[j];
    x[i] = xi;
    ss += xi * xi;
  }
  __syncthreads();
  return block_sum(ss, L);
}

template <int BT>
__device__ __noinline__ void bdots_ool(const float* V_, int ldv, int t, int lo, int hi, const double* x_,
                                       Lds<BT>& L) {
  bdots_body<BT, true>(V_, ldv, t, lo, hi, x_, L);
}
template <int BT, bool OUT>
__device__ __forceinline__ void bdots(const float* V_, int ldv, int t, int lo, int hi, const double* x_, Lds<BT>& L) {
  if constexpr (OUT) bdots_ool<BT>(V_, ldv, t, lo, hi, x_, L);
  else bdots_body<BT, false>(V_, ldv, t, lo, hi, x_, L);
}
template <int BT>
__device__ __noinline__ double bupdate_ool(const float* V_, int ldv, int t, int lo, int hi, double* x_,
                                           const double* h, Lds<BT>& L) {
  return bupdate_body<BT, true>(V_, ldv, t, lo, hi, x_, h, L);
}
template <int BT, bool OUT>
__device__ __forceinline__ double bupdate(const float* V_, int ldv, int t, int lo, int hi, double* x_,
                                          const double* h, Lds<BT>& L) {
  if constexpr (OUT) return bupdate_ool<BT>(V_, ldv, t, lo, hi, x_, h, L);
  else return bupdate_body<BT, false>(V_, ldv, t, lo, hi, x_, h, L);
}

// Two classical Gram-Schmidt passes of x against V[:, 0:t] on the member's
// range; returns the team-wide ||x||^2.
template <int BT, bool OUT>
__device__ double bcgs2(const float* V, int ldv, int t, int lo, int hi, double* x, Team& tm, Lds<BT>& L) {
  double ss;
  if (t > 0) {
    bdots<BT, OUT>(V, ldv, t, lo, hi, x, L);
    team_sum(L.h, t, tm, L);
    bupdate<BT, OUT>(V, ldv, t, lo, hi, x, L.h, L);
    bdots<BT, OUT>(V, ldv, t, lo, hi, x, L);
    team_sum(L.h, t, tm, L);
    ss = bupdate<BT, OUT>(V, ldv, t, lo, hi, x, L.h, L);
  } else {
    ss = 0.0;
    const GMEM double* xg = gc(x);
    for (int i = lo + threadIdx.x; i < hi; i += BT) ss += xg[i] * xg[i];
    ss = block_sum(ss, L);
  }
  return team_sum_scalar(ss, tm, L);
}

template <int BT>
__device__ void bscale(const double* x_, int lo, int hi, double nrm, float* out, bool coherent) {
  const GMEM double* x = gc(x_);
  if (coherent) {
    for (int i = lo + threadIdx.x; i < hi; i += BT) cst(out + i, (float)(x[i] / nrm));
  } else {
    GMEM float* o = gw(out);
    for (int i = lo + threadIdx.x; i < hi; i += BT) o[i] = (float)(x[i] / nrm);
  }
  __syncthreads();
}

// The team's current p, read from the coherence point into LDS (n <= BATCH_TEAM_NMAX).
template <int BT>
__device__ const float* team_load_p(const float* p, int n, Lds<BT>& L) {
  for (int j = threadIdx.x; j < n; j += BT) L.pvec[j] = ldc(p + j);
  __syncthreads();
  return L.pvec;
}

// One-sided Jacobi SVD of the nq x np matrix in L.Hs (columns), accumulating
// the right rotations in L.Vs; afterwards sv[c] = column norms and perm sorts
// them descending (ties by index).  Pairs follow the round-robin ordering so
// each round's pairs are disjoint; one wave per pair.  The ordering: player 0
// stays, players 1 .. N-1 move one seat on each round, and seat c meets seat
// N - 1 - c; the seat of a player is computed, not stored.
template <int BT>
__device__ void bjacobi(int nq, int np, Lds<BT>& L) {
  constexpr int NW = BT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < np * KMAX; e += BT) L.Vs[e] = 0.0;
  __syncthreads();
  for (int c = tid; c < np; c += BT) L.Vs[c * KMAX + c] = 1.0;
  const int N = (np + 1) & ~1;  // even number of players (index np is a bye)
  // the player in seat c after `round` moves
  auto seat = [N](int c, int round) { return c == 0 ? 0 : 1 + ((c - 1 - round) % (N - 1) + (N - 1)) % (N - 1); };
  for (int s = 0; s < 60; ++s) {
    if (tid == 0) L.rotated = 0;
    __syncthreads();
    for (int round = 0; round < N - 1; ++round) {
      for (int pr = wave; pr < N / 2; pr += NW) {
        const int pa = seat(pr, round), pb = seat(N - 1 - pr, round);
        const int i = min(pa, pb);
        const int j = max(pa, pb);
        if (j >= np) continue;
        double* hi = L.Hs + i * HLD;
        double* hj = L.Hs + j * HLD;
        double a = 0.0, b = 0.0, c = 0.0;
        for (int r = lane; r < nq; r += 64) {
          a += hi[r] * hi[r];
          b += hj[r] * hj[r];
          c += hi[r] * hj[r];
        }
        a = wsum(a);
        b = wsum(b);
        c = wsum(c);
        if (c != 0.0 && fabs(c) > 1e-15 * sqrt(a * b)) {
          const double zeta = (b - a) / (2.0 * c);
          const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
          for (int r = lane; r < nq; r += 64) {
            const double x = hi[r], y = hj[r];
            hi[r] = cs * x - sn * y;
            hj[r] = sn * x + cs * y;
          }
          double* vi = L.Vs + i * KMAX;
          double* vj = L.Vs + j * KMAX;
          for (int r = lane; r < np; r += 64) {
            const double x = vi[r], y = vj[r];
            vi[r] = cs * x - sn * y;
            vj[r] = sn * x + cs * y;
          }
          if (lane == 0) L.rotated = 1;
        }
      }
      __syncthreads();
    }
    const int rot = L.rotated;
    __syncthreads();
    if (!rot) break;
  }
  // column norms, normalised left vectors, descending order
  for (int c = wave; c < np; c += NW) {
    double a = 0.0;
    for (int r = lane; r < nq; r += 64) a += L.Hs[c * HLD + r] * L.Hs[c * HLD + r];
    a = wsum(a);
    const double nr = sqrt(a);
    if (lane == 0) L.sv[c] = nr;
    for (int r = lane; r < nq; r += 64) L.Hs[c * HLD + r] = nr > 0 ? L.Hs[c * HLD + r] / nr : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    for (int c = 0; c < np; ++c) L.perm[c] = c;
    for (int a = 0; a < np; ++a) {
      int best = a;
      for (int b = a + 1; b < np; ++b)
        if (L.sv[L.perm[b]] > L.sv[L.perm[best]]) best = b;
      const int tmp = L.perm[a];
      L.perm[a] = L.perm[best];
      L.perm[best] = tmp;
    }
  }
  __syncthreads();
}

// out[lo:hi, c] = V[lo:hi, 0..kk) * M[0..kk, perm[c]] for c < ncols, M column-major in LDS
// (column stride mld); V column-major (ldv), out column-major (ldo).
template <int BT>
__device__ void bgemm_small(const float* V_, int ldv, int lo, int hi, int kk, const double* M, int mld,
                            const int* perm, int ncols, float* out_, int ldo) {
  const GMEM float* V = gc(V_);
  GMEM float* out = gw(out_);
  for (int i = lo + threadIdx.x; i < hi; i += BT) {
    for (int c0 = 0; c0 < ncols; c0 += 8) {
      double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int j = 0; j < kk; ++j) {
        const double v = (double)V[(int64_t)j * ldv + i];
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (c0 + e < ncols) acc[e] += v * M[perm[c0 + e] * mld + j];
      }
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (c0 + e < ncols) out[(int64_t)(c0 + e) * ldo + i] = (float)acc[e];
    }
  }
  __syncthreads();
}

// Normalise x[lo:hi] into out with the breakdown test (nrm2 is the team-wide
// squared norm, so every member decides alike); returns false on breakdown
// (L.flag set).  thr = eps * sig (relative) or eps.
template <int BT>
__device__ bool bnormalize(const double* x, int lo, int hi, double nrm2, double thr, float* out, int code, int idx,
                           Lds<BT>& L, bool coherent = false) {
  const double nrm = sqrt(nrm2);
  if (!(nrm < INFINITY)) {
    if (threadIdx.x == 0) {
      L.flag = 3;
      L.flag_idx = idx;
    }
    __syncthreads();
    return false;
  }
  if (nrm <= thr) {
    if (threadIdx.x == 0) {
      L.flag = code;
      L.flag_idx = idx;
    }
    __syncthreads();
    return false;
  }
  bscale<BT>(x, lo, hi, nrm, out, coherent);
  return true;
}

// Philox4x32-10 start vector (same definition as the single-problem path).
__device__ double philox_normal(int64_t i, uint64_t seed) {
  uint32_t c[4] = {(uint32_t)(i & 0xffffffffu), (uint32_t)((uint64_t)i >> 32), 0u, 0u};
  uint32_t k[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  for (int r = 0; r < 10; ++r) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
    const uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k[0], n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    if (r < 9) {
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
  }
  const double two32 = 4294967296.0;
  const double u0 = ((double)c[0] + 1.0) / two32, u1 = ((double)c[1] + 1.0) / two32;
  return 2.0 + sqrt(-2.0 * log(u0)) * cos(6.283185307179586 * u1);
}

// Solve one problem as member `member` of its team (all threads of the workgroup).
template <int BT, bool OUT>
__device__ void solve_one(const BatchProblem& P, int member, const BatchParams& prm, Lds<BT>& L) {
  const unsigned long long t_start = wall_clock64();
  const int tid = threadIdx.x;
  const int ldq = P.ldq, ldp = P.ldp;   // basis column strides (multiples of 4: 16-byte aligned columns)
  float* Qb[2] = {prm.pool + P.offQ, prm.pool + P.offQ + (int64_t)(P.k + 1) * ldq};
  float* Pb[2] = {prm.pool + P.offP, prm.pool + P.offP + (int64_t)(P.k + 1) * ldp};
  double* w = prm.work + P.offW;
  double* z = w + P.m;
  const int m = P.m, n = P.n, k = P.k, r = P.r, l = P.l;
  Team tm;
  tm.T = P.team;
  tm.member = member;
  tm.cnt = prm.team_cnt + (P.team > 1 ? P.team_id : 0);
  tm.zpart = prm.team_buf + P.offTeam;
  tm.small = tm.zpart + (int64_t)P.team * n;
  tm.nbar = 0;
  tm.parity = 0;
  tm.spin_limit = prm.spin_limit;
  tm.skew = prm.barrier_skew;
  const int qlo = (int)((int64_t)member * m / tm.T), qhi = (int)((int64_t)(member + 1) * m / tm.T);
  const int plo = (int)((int64_t)member * n / tm.T), phi = (int)((int64_t)(member + 1) * n / tm.T);
  int cur = 0;
  auto Qc = [&](int j) { return Qb[cur] + (int64_t)j * ldq; };
  auto Pc = [&](int j) { return Pb[cur] + (int64_t)j * ldp; };
  const double eps = prm.eps_break;
  double sig = 0.0;  // running largest accepted coefficient / Ritz value
  int64_t matvecs = 0;
  int restarts = 0, nconv = 0, r_eff = 0, status = 0;
  if (tid == 0) {
    L.flag = 0;
    L.flag_idx = 0;
    L.team_fail = 0;
  }
  __syncthreads();
  // start: q ~ N(2,1) (Philox, seed + problem index) or caller's vector
  for (int i = qlo + tid; i < qhi; i += BT) w[i] = prm.q1 ? prm.q1[P.offQ1 + i] : philox_normal(i, prm.seed + P.index);
  __syncthreads();
  double ss = 0.0;
  for (int i = qlo + tid; i < qhi; i += BT) ss += w[i] * w[i];
  ss = team_sum_scalar(block_sum(ss, L), tm, L);
  if (!bnormalize(w, qlo, qhi, ss, 0.0, Qc(0), 1, 0, L)) {
    status = -1;
  }
  int nq = 0, np = 0;        // shape of the projected matrix of the cycle
  double alpha_res = 0.0;
  bool first = true;
  bool done = status != 0;
  while (!done) {
    // ---------------- one cycle
    int jstart = first ? 0 : l;
    int np_now = 0;
    bool early = false;
    if (first) {
      team_gemv_t<BT, OUT>(P, Qc(0), nullptr, 0.0, z, qlo, qhi, plo, phi, tm, L);
      ++matvecs;
      ss = bcgs2<BT, OUT>(nullptr, ldp, 0, plo, phi, z, tm, L);
      if (!bnormalize(z, plo, phi, ss, 0.0, Pc(0), 2, 0, L, tm.T > 1)) {
        // A^T q1 = 0
        nq = 1;
        np = 0;
        break;
      }
      if (tid == 0) L.pc[0] = sqrt(ss);
      sig = fmax(sig, sqrt(ss));
      if (tm.T > 1) team_barrier(tm, L);   // p_1 complete before A p_1
      __syncthreads();
    }
    for (int j = jstart; j < k; ++j) {
      if (L.team_fail) break;
      // q side
      const int qi = first ? j + 1 : j;     // new Q column
      const float* qprev = first ? Qc(j) : (j == l ? nullptr : Qc(j - 1));
      const double cprev = (first || j != l) ? L.pc[j] : 0.0;
      if (tm.T > 1)
        bgemv_n<BT, OUT, true>(P, team_load_p(Pc(j), n, L), qprev, cprev, w, qlo, qhi);
      else
        bgemv_n<BT, OUT, false>(P, Pc(j), qprev, cprev, w, qlo, qhi);
      if (!first) {
        if (j == l) bupdate<BT, OUT>(Qc(0), ldq, l, qlo, qhi, w, L.rho, L);
      }
      ++matvecs;
      ss = bcgs2<BT, OUT>(Qc(0), ldq, qi, qlo, qhi, w, tm, L);
      if (!bnormalize(w, qlo, qhi, ss, prm.relative ? eps * sig : eps, Qc(qi), 1, qi, L)) break;
      const double beta = sqrt(ss);
      if (tid == 0) L.qc[qi] = beta;
      sig = fmax(sig, beta);
      // p side
      team_gemv_t<BT, OUT>(P, Qc(qi), Pc(j), beta, z, qlo, qhi, plo, phi, tm, L);
      ++matvecs;
      ss = bcgs2<BT, OUT>(Pc(0), ldp, j + 1, plo, phi, z, tm, L);
      if (!bnormalize(z, plo, phi, ss, prm.relative ? eps * sig : eps, Pc(j + 1), 2, j + 1, L, tm.T > 1)) break;
      const double alpha = sqrt(ss);
      if (tid == 0) L.pc[j + 1] = alpha;
      sig = fmax(sig, alpha);
      if (tm.T > 1) team_barrier(tm, L);   // p_{j+2} complete before the next A p
      __syncthreads();
      np_now = j + 1;
      if (prm.check_every > 0 && np_now < k && np_now >= r && np_now % prm.check_every == 0) {
        // in-cycle convergence test on the partial projected matrix
        const int cq = first ? np_now + 1 : np_now;
        for (int e = tid; e < np_now * HLD; e += BT) L.Hs[e] = 0.0;
        __syncthreads();
        if (tid == 0) {
          if (first) {
            for (int c = 0; c < np_now; ++c) {
              L.Hs[c * HLD + c] = L.pc[c];
              L.Hs[c * HLD + c + 1] = L.qc[c + 1];
            }
          } else {
            for (int i = 0; i < l; ++i) {
              L.Hs[i * HLD + i] = L.sres[i];
              L.Hs[l * HLD + i] = L.rho[i];
            }
            for (int c = l; c < np_now; ++c) {
              L.Hs[c * HLD + c] = L.qc[c];
              if (c + 1 < np_now) L.Hs[(c + 1) * HLD + c] = L.pc[c + 1];
            }
          }
        }
        __syncthreads();
        bjacobi(cq, np_now, L);
        const double thr = prm.relative ? eps * sig : eps;
        int avail = 0;
        for (int c = 0; c < np_now; ++c)
          if (L.sv[L.perm[c]] > thr) ++avail;
        const int re = min(r, avail);
        const double s0 = L.sv[L.perm[0]];
        int nc = 0;
        for (int c = 0; c < re; ++c)
          if (alpha * fabs(L.Hs[L.perm[c] * HLD + cq - 1]) <= prm.tol * s0) ++nc;
        if (re == r && nc == r) {
          early = true;
          nq = cq;
          np = np_now;
          alpha_res = alpha;
          break;
        }
      }
    }
    const int fl = L.flag, fidx = L.flag_idx;
    __syncthreads();
    if (L.team_fail) {
      status = GKB_ERR_TIMEOUT;
      break;
    }
    if (fl == 3) {
      status = -3;
      break;
    }
    if (!early) {
      // assemble the projected matrix (same rules as the host driver)
      if (fl == 0) {
        np = k;
        nq = first ? k + 1 : k;
        alpha_res = L.pc[k];
      } else if (first) {
        if (fl == 1) {
          nq = np = fidx;
        } else {
          np = fidx;
          nq = fidx + 1;
        }
        alpha_res = 0.0;
      } else {
        if (fl == 1) {
          nq = fidx;
          np = fidx + 1;
        } else {
          nq = np = fidx;
        }
        alpha_res = 0.0;
      }
      for (int e = tid; e < np * HLD; e += BT) L.Hs[e] = 0.0;
      __syncthreads();
      if (tid == 0) {
        if (first) {
          for (int c = 0; c < np; ++c) {
            L.Hs[c * HLD + c] = L.pc[c];
            if (c + 1 < nq) L.Hs[c * HLD + c + 1] = L.qc[c + 1];
          }
        } else {
          for (int i = 0; i < l && i < nq; ++i) {
            if (i < np) L.Hs[i * HLD + i] = L.sres[i];
            if (l < np) L.Hs[l * HLD + i] = L.rho[i];
          }
          for (int c = l; c < nq; ++c) {
            L.Hs[c * HLD + c] = L.qc[c];
            if (c + 1 < np) L.Hs[(c + 1) * HLD + c] = L.pc[c + 1];
          }
        }
      }
      __syncthreads();
      if (np > 0) bjacobi(nq, np, L);
    }
    // convergence test
    const double thr = prm.relative ? eps * sig : eps;
    int avail = 0;
    for (int c = 0; c < np; ++c)
      if (L.sv[L.perm[c]] > thr) ++avail;
    r_eff = min(r, avail);
    const double s0 = np > 0 ? L.sv[L.perm[0]] : 0.0;
    nconv = 0;
    for (int c = 0; c < r_eff; ++c)
      if (alpha_res * fabs(L.Hs[L.perm[c] * HLD + nq - 1]) <= prm.tol * s0) ++nconv;
    const bool conv = r_eff == r && nconv == r;
    if (fl != 0 || conv || restarts >= prm.max_restarts || k == r || early) {
      done = true;
      break;
    }
    // ---------------- thick restart (each member its own rows of Q and entries of P)
    sig = fmax(sig, s0);
    const int nb = 1 - cur;
    // P~ = P Y_l (Y = Vs, columns by perm), Q~ = Q X_l (X = Hs normalised)
    bgemm_small<BT>(Pb[cur], ldp, plo, phi, np, L.Vs, KMAX, L.perm, l, Pb[nb], ldp);
    bgemm_small<BT>(Qb[cur], ldq, qlo, qhi, nq, L.Hs, HLD, L.perm, l, Qb[nb], ldq);
    for (int i = plo + tid; i < phi; i += BT) cst(Pb[nb] + (int64_t)l * ldp + i, Pb[cur][(int64_t)np * ldp + i]);
    if (tid < l) {
      L.sres[tid] = L.sv[L.perm[tid]];
      L.rho[tid] = alpha_res * L.Hs[L.perm[tid] * HLD + nq - 1];
    }
    __syncthreads();
    if (tm.T > 1) team_barrier(tm, L);   // the new P complete before A p_{l+1}
    cur = nb;
    ++restarts;
    first = false;
    if (tid == 0) {
      L.flag = 0;
      L.flag_idx = 0;
    }
    __syncthreads();
  }
  // a team barrier that timed out voids the solve, whichever way it ended
  if (L.team_fail) status = GKB_ERR_TIMEOUT;
  // ---------------- outputs (each member its rows of U and entries of V)
  const int pi = P.index;
  if (status == 0 && np > 0) {
    float* U = prm.U + P.offU;
    float* V = prm.V + P.offV;
    bgemm_small<BT>(Pb[cur], ldp, plo, phi, np, L.Vs, KMAX, L.perm, r_eff, V, n);
    bgemm_small<BT>(Qb[cur], ldq, qlo, qhi, nq, L.Hs, HLD, L.perm, r_eff, U, m);
    if (member == 0 && tid < r) prm.sigma[P.offS + tid] = tid < r_eff ? L.sv[L.perm[tid]] : 0.0;
  } else if (member == 0 && tid < r) {
    prm.sigma[P.offS + tid] = 0.0;
  }
  if (member == 0 && tid == 0) {
    int st = status;
    if (st == 0) st = r_eff < r ? 2 : (nconv == r ? 0 : 1);
    prm.info[4 * pi + 0] = st;
    prm.info[4 * pi + 1] = nconv;
    prm.info[4 * pi + 2] = restarts;
    prm.info[4 * pi + 3] = (int)matvecs;
    prm.ticks[pi] = wall_clock64() - t_start;
  }
  __syncthreads();
}

}  // namespace

template <int BT, bool OUT>
__global__ __launch_bounds__(BT) void k_batched_gk(BatchParams prm) {
  extern __shared__ double lds_raw[];
  Lds<BT>& L = *reinterpret_cast<Lds<BT>*>(lds_raw);
  while (true) {
    if (threadIdx.x == 0) {
      const int slot = atomicAdd(prm.counter, 1);
      L.problem = slot < prm.ntickets ? prm.order[slot] : -1;
      L.member = slot < prm.ntickets ? prm.member[slot] : 0;
    }
    __syncthreads();
    const int p = L.problem, mem = L.member;
    __syncthreads();
    if (p < 0) break;
    const BatchProblem P = prm.problems[p];
    solve_one<BT, OUT>(P, mem, prm, L);
  }
}

// Zero the queue head and the team barrier counters.
__global__ void k_batched_reset(int* counter, int* team_cnt, int nteams) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nteams; i += gridDim.x * blockDim.x) team_cnt[i] = 0;
}

// Copy the matrices listed in the stage table into 16-byte aligned rows of
// 4 ceil(n / 4) floats with zero padding: one wave per row, rows of all
// entries numbered consecutively (row_start is the prefix sum of m).
__global__ __launch_bounds__(256) void k_batched_stage(const StageCopy* __restrict__ tab, int ntab,
                                                        int64_t total_rows) {
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); row < total_rows; row += nwaves) {
    int lo = 0, hi = ntab - 1;  // last entry with row_start <= row
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tab[mid].row_start <= row) lo = mid;
      else hi = mid - 1;
    }
    const StageCopy& t = tab[lo];
    const int64_t i = row - t.row_start;
    const float* src = t.src + i * t.lds;
    float* dst = t.dst + i * t.ldd;
    for (int j = lane; j < t.ldd; j += 64) dst[j] = j < t.n ? src[j] : 0.f;
  }
}

size_t batched_lds_bytes(int threads) { return threads == 512 ? sizeof(Lds<512>) : sizeof(Lds<1024>); }

hipError_t launch_batched(const BatchParams& prm, int grid, int threads, hipStream_t st) {
  hipLaunchKernelGGL(k_batched_reset, dim3(1), dim3(256), 0, st, prm.counter, prm.team_cnt, prm.nteams);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (prm.nstage > 0) {
    const int64_t blocks = std::min<int64_t>((prm.stage_rows + 3) / 4, 8192);
    hipLaunchKernelGGL(k_batched_stage, dim3((unsigned)blocks), dim3(256), 0, st, prm.stage, prm.nstage,
                       prm.stage_rows);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (threads == 512) {
    if (prm.outline) hipLaunchKernelGGL((k_batched_gk<512, true>), dim3(grid), dim3(512), sizeof(Lds<512>), st, prm);
    else hipLaunchKernelGGL((k_batched_gk<512, false>), dim3(grid), dim3(512), sizeof(Lds<512>), st, prm);
  } else {
    if (prm.outline)
      hipLaunchKernelGGL((k_batched_gk<1024, true>), dim3(grid), dim3(1024), sizeof(Lds<1024>), st, prm);
    else hipLaunchKernelGGL((k_batched_gk<1024, false>), dim3(grid), dim3(1024), sizeof(Lds<1024>), st, prm);
  }
  return hipGetLastError();
}

hipError_t batched_setup() {
  const void* kernels[4] = {reinterpret_cast<const void*>(&k_batched_gk<512, false>),
                            reinterpret_cast<const void*>(&k_batched_gk<512, true>),
                            reinterpret_cast<const void*>(&k_batched_gk<1024, false>),
                            reinterpret_cast<const void*>(&k_batched_gk<1024, true>)};
  const int lds[4] = {(int)sizeof(Lds<512>), (int)sizeof(Lds<512>), (int)sizeof(Lds<1024>), (int)sizeof(Lds<1024>)};
  for (int i = 0; i < 4; ++i) {
    const hipError_t e = hipFuncSetAttribute(kernels[i], hipFuncAttributeMaxDynamicSharedMemorySize, lds[i]);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace gkb
