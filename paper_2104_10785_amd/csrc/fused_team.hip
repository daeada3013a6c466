// One sweep of A for both products of a Golub-Kahan step on rows longer than
// the single-workgroup sweep holds (n > FUSED_NMAX), and on float64 rows: a
// team of workgroups per range of rows, each member owning a slice of the
// columns.
//
// The single-workgroup sweep keeps its float64 partial of A^T w in registers,
// which bounds the row length.  Here the 16-byte column groups are cut into C
// near-equal slices of at most 8192 columns (4096 for float64 rows, 16384
// for bfloat16: 32 KB of a row in each case), and C workgroups -- a team --
// share a range of rows.
// Member c streams its slice of each row, forms the slice's part of the row's
// dot product with p (reduced across the workgroup in a fixed order) and
// publishes it; once all C parts of a row are in, every member adds them in
// member order (so every member holds the same w_i) and adds a_i[slice] w_i
// into its float64 partial of A^T w.  The team's partial is one row of the partial-sum array, which
// the consumers add in team order, as they add the workgroups' partials of
// the single-workgroup sweep.
//
// Exchange.  Each part (a double) goes to a mailbox in device memory as two
// 64-bit words, (high half << 32 | tag) and (low half << 32 | tag), with
// device-scope stores; a reader loads both with device-scope loads and takes
// them once both carry the tag.  So the two stores need no order between
// them and no fence, and publishing a part never waits.  The tag is the
// launch's generation + 1: a counter in the mailbox header that the last
// workgroup to finish a launch advances, so the words of earlier launches
// read as stale; every step of a launch has slots of its own (nothing is
// reused within a launch).  The header and slots are zeroed once before the
// first launch (launch_team_reset).
//
// Pipeline.  Iteration s loads the words of step s - D + NB - 2, issues the
// row loads of step s + NB - 1, forms and publishes the parts of step s, then
// checks the words of step s - D and adds that step's rows: NB + D steps of
// rows stay in registers (loading, being reduced, waiting for the exchange),
// and a step's parts have about D + 1 - NB iterations to arrive before they
// are loaded.  The words are loaded before the row loads of their iteration,
// so waiting for them never waits for rows not yet in use.  As in the pipelined
// single-workgroup sweep every load is issued on one path (clamped buffer
// ranges, clamped mailbox slots) and the only barrier is an LDS one, so the
// compiler's in-order memory counting never waits for rows still loading;
// the parts are stored by lanes 0 .. 2R - 1 of every wave (the same values),
// so every wave runs the same instruction stream.
//
// Members of a team must run at the same time: the grid has at most one
// workgroup per compute unit and every CU holds at least one of them, so the
// whole grid is resident once the device is free.  A wait is bounded
// (TM_SPIN_LIMIT polls, about a second); on a timeout the flag is set to 4,
// the member's outputs are set to NaN, and the wave stops waiting.  For
// tests of that path the environment variable GKB_TEAM_STALL_POLLS = P > 0
// makes every wait time out after P polls: readers then look for a tag that
// no member writes (every kernel still runs to its end).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <type_traits>

#include "device_common.h"
#include "fused.h"
#include "fused_device.h"
#include "gemv.h"
#include "lds_attr.h"

namespace gkb {

namespace {

using fdev::Elems;
using fdev::f4;
using fdev::lds_barrier;
using fdev::RSRC_WORD3;
using fdev::wsum_dpp;

constexpr int TM_T = 512;          // threads per member
constexpr int TM_R = 1;            // rows per step
constexpr int TM_CMAX = 32;        // members per team (C R parts per step, one per lane)
constexpr long TM_SPIN_LIMIT = 1L << 20;
static_assert(TM_CMAX * TM_R <= 64, "a step's parts are read one per lane");

// Per element type: columns per member at most (32 KB of a row per step:
// 8192 float32, 4096 float64, 16384 bfloat16), steps of rows in flight (NB)
// and steps between a step's parts and their use (D), as measured; the
// bfloat16 form holds twice the partial sums per thread, so one step fewer
// in flight.
constexpr int slice_cols(int dtype) { return dtype == 0 ? 4096 : (dtype == 2 ? 16384 : 8192); }
template <typename TA> constexpr int tm_dtype() { return sizeof(TA) == 8 ? 0 : (sizeof(TA) == 2 ? 2 : 1); }
template <typename TA> constexpr int tm_slice() { return slice_cols(tm_dtype<TA>()); }
template <typename TA> constexpr int tm_u() { return tm_slice<TA>() / (TM_T * Elems<TA>::VN); }
template <typename TA> constexpr int tm_nb() { return sizeof(TA) == 2 ? 2 : 3; }
template <typename TA> constexpr int tm_d() { return 5; }

__device__ __forceinline__ uint64_t ld_dev(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double part_of(uint64_t hi, uint64_t lo) {
  return __longlong_as_double((long long)(((hi >> 32) << 32) | (lo >> 32)));
}
__device__ __forceinline__ double readlane_d(double v, int l) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, l);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// T threads, U 16-byte groups per thread (thread t owns groups t + u T of the
// member's slice), R rows per step.  GIVEN_W: y = A^T win (no dot products,
// no exchange; win is loaded with the rows).  ctr[0]: generation, ctr[1]:
// workgroups finished in this launch; mbox: teams x nsteps x C x R x 2 words.
// spin_limit bounds each wait; readers accept the launch's tag + skew
// (skew 0 except in tests of the timeout path).
template <int T, int U, int R, int NB, int D, typename TA, typename TP, bool GIVEN_W>
__global__ __launch_bounds__(T) void k_gemv_fused_team(const TA* __restrict__ A, int64_t lda, int m, int64_t n,
                                                       const TP* __restrict__ p, const double* __restrict__ win,
                                                       int C, int rpt, int nsteps, double* __restrict__ w,
                                                       double* __restrict__ ypart, int64_t ldy, int* flag,
                                                       const int* __restrict__ run_if,
                                                       const double* __restrict__ qprev,
                                                       const double* __restrict__ coef, uint64_t* mbox,
                                                       uint32_t* ctr, long spin_limit, uint32_t skew) {
  constexpr int DD = GIVEN_W ? 0 : D;
  constexpr int K = NB + DD;   // row buffers
  // a step's words are loaded LL iterations before they are checked, before
  // that iteration's row loads: the check then waits for no rows that are
  // not already in use (the memory counter is in order)
  constexpr int LL = NB - 2;
  static_assert(NB >= 2 && LL <= 1 && (GIVEN_W || LL == 0 || K % 2 == 0), "mailbox words alternate by step parity");
  constexpr int NWV = T / 64;
  constexpr int VN = Elems<TA>::VN;
  if (flag != nullptr && flag[0] != 0) return;
  if (run_if != nullptr && run_if[0] == 0) return;
  const int team = blockIdx.x / C, member = blockIdx.x - team * C;
  const int ng = (int)(n / VN);
  const int g0 = (int)((int64_t)member * ng / C);
  const int sg = (int)((int64_t)(member + 1) * ng / C) - g0;   // groups of this slice (<= U T)
  __shared__ double red[2][R][NWV];                              // [parity][row][wave]
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t tag = GIVEN_W ? 0u : __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
  const uint32_t expect = tag + skew;   // the tag a reader takes
  // the slice of p, zero padded to U T groups (the dot products read it from
  // LDS): float32 for bfloat16 rows (float32 dot products), float64 otherwise
  // (for float32 rows: p rounded to float32 once, then widened exactly, so
  // the dot products convert only the row's elements)
  using PL = typename std::conditional<Elems<TA>::F32DOT, float, double>::type;
  extern __shared__ __align__(16) unsigned char pl_raw[];
  PL* pl = reinterpret_cast<PL*>(pl_raw);
  if constexpr (!GIVEN_W) {
    for (int j = tid; j < U * T * VN; j += T)
      pl[j] = j < sg * VN ? (sizeof(TA) == 8 ? (PL)p[(int64_t)g0 * VN + j] : (PL)(float)p[(int64_t)g0 * VN + j])
                          : (PL)0;
    __syncthreads();
  }
  const int r0 = team * rpt;
  const int r1 = std::min(m, r0 + rpt);
  const int last = r1 - 1;   // no team is empty
  const int64_t ldb = lda * (int64_t)sizeof(TA);
  const char* Ab = reinterpret_cast<const char*>(A) + (int64_t)g0 * 16;
  const int slice_bytes = sg * 16;
  const int off0 = tid * 16;
  const int CR = C * R;
  uint64_t* mb = mbox + (int64_t)team * nsteps * CR * 2;
  const int mlane = lane < CR ? lane : 0;

  // rows i .. i + R - 1 of the slice: group u through a resource that starts
  // at the slice's group u T and ends at the slice's end (nothing for rows
  // past the team's range, which read as zeros)
  auto load_step = [&](int i, f4 (&dst)[R][U], double (&wv)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool live = i + r <= last;
      const int ri = __builtin_amdgcn_readfirstlane(std::min(i + r, last));
      const char* row = Ab + (int64_t)ri * ldb;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int nrec = __builtin_amdgcn_readfirstlane(live ? std::max(slice_bytes - u * T * 16, 0) : 0);
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void*)(row + u * T * 16), (short)0, nrec, RSRC_WORD3);
        dst[r][u] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, off0, 0, 2));
      }
      if constexpr (GIVEN_W) wv[r] = win[ri];
    }
  };
  // this lane's part (entry mlane) of step `step` (clamped into the launch's steps)
  auto mail_load = [&](int step, uint64_t (&dst)[2]) {
    const int sc = std::min(std::max(step, 0), nsteps - 1);
    const uint64_t* a = mb + ((int64_t)sc * CR + mlane) * 2;
    dst[0] = ld_dev(a);
    dst[1] = ld_dev(a + 1);
  };

  double y[U][VN];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int e = 0; e < VN; ++e) y[u][e] = 0.0;
  f4 B[K][R][U];
  double WV[K][R];
  uint64_t MW[2][2];
  int par = 0;
  bool failed = false;

  // the parts of step s: partial dot products over the slice, reduced over the
  // workgroup in wave order, stored by lanes 0 .. 2R - 1 of every wave
  auto publish = [&](f4 (&rows)[R][U], int s) {
    double d[R];
    if constexpr (Elems<TA>::F32DOT) {
      float df[R];
#pragma unroll
      for (int r = 0; r < R; ++r) df[r] = 0.f;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int g = tid + u * T;
#pragma unroll
        for (int h = 0; h < VN / 4; ++h) {
          const f4 pv = reinterpret_cast<const f4*>(pl)[(VN / 4) * g + h];
#pragma unroll
          for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int r = 0; r < R; ++r) df[r] = fmaf(Elems<TA>::at(rows[r][u], 4 * h + e), pv[e], df[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) d[r] = (double)df[r];
    } else if constexpr (sizeof(TA) == 8) {
#pragma unroll
      for (int r = 0; r < R; ++r) d[r] = 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const fdev::d2 pv = reinterpret_cast<const fdev::d2*>(pl)[tid + u * T];
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
          for (int r = 0; r < R; ++r) d[r] += Elems<TA>::at(rows[r][u], e) * pv[e];
      }
    } else {
      // float32 rows: p in LDS as float64 (two 16-byte reads per group)
#pragma unroll
      for (int r = 0; r < R; ++r) d[r] = 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int g = tid + u * T;
        const fdev::d2 p0 = reinterpret_cast<const fdev::d2*>(pl)[2 * g];
        const fdev::d2 p1 = reinterpret_cast<const fdev::d2*>(pl)[2 * g + 1];
        const double pe[4] = {p0[0], p0[1], p1[0], p1[1]};
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int r = 0; r < R; ++r) d[r] += (double)Elems<TA>::at(rows[r][u], e) * pe[e];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      d[r] = wsum_dpp(d[r]);
      if (lane == 0) red[par][r][wave] = d[r];
    }
    // an empty register constraint: the update D steps later converts the
    // rows anew instead of keeping their float64 forms live until then
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int u = 0; u < U; ++u) asm volatile("" : "+v"(rows[r][u]));
    lds_barrier();
    double v = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < NWV; ++k) t += red[par][r][k];
      if ((lane >> 1) == r) v = t;
    }
    par ^= 1;   // the next step writes the other half of red: one barrier per step
    if (lane < 2 * R) {
      const uint64_t bits = (uint64_t)__double_as_longlong(v);
      const uint64_t pay = (lane & 1) ? (bits & 0xffffffffull) : (bits >> 32);
      st_dev(mb + (((int64_t)s * C + member) * R) * 2 + lane, (pay << 32) | tag);
    }
  };
  // w of step s from its parts (lane l < C R holds entry l = c R + r), added
  // in member order; waits (bounded) for parts not yet in
  auto gather = [&](uint64_t (&mw)[2], int s, double (&wi)[R]) {
    bool ok = lane >= CR || ((uint32_t)mw[0] == expect && (uint32_t)mw[1] == expect);
    if (!failed && __builtin_amdgcn_ballot_w64(!ok) != 0) {
      // every exit follows the test of the words just loaded, so no poll is
      // left in flight where this path rejoins the one that did not wait
      for (long polls = 0;; ++polls) {
        __builtin_amdgcn_s_sleep(2);
        mail_load(s, mw);
        ok = lane >= CR || ((uint32_t)mw[0] == expect && (uint32_t)mw[1] == expect);
        if (__builtin_amdgcn_ballot_w64(!ok) == 0) break;
        if (polls >= spin_limit) {
          failed = true;
          break;
        }
      }
    }
    const double dl = part_of(mw[0], mw[1]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double t = 0.0;
      for (int c = 0; c < C; ++c) t += readlane_d(dl, c * R + r);
      wi[r] = t;
    }
  };
  auto update = [&](const f4 (&rows)[R][U], const double (&wi)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < VN; ++e) y[u][e] += (double)Elems<TA>::at(rows[r][u], e) * wi[r];
  };

#pragma unroll
  for (int k = 0; k < NB - 1; ++k) {
    load_step(r0 + k * R, B[k], WV[k]);
    asm volatile("" ::: "memory");   // issued in step order, as in the loop
  }
  const int iters = nsteps + DD;
  for (int s0 = 0; s0 < iters; s0 += K) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int s = s0 + k;
      if constexpr (!GIVEN_W) mail_load(s - DD + LL, MW[(k - DD + LL + 2 * K) % 2]);
      load_step(r0 + (s + NB - 1) * R, B[(k + NB - 1) % K], WV[(k + NB - 1) % K]);
      if constexpr (GIVEN_W) {
        update(B[k], WV[k]);
      } else {
        if (s < nsteps) publish(B[k], s);
        if (s >= DD) {
          double wi[R];
          gather(MW[(k - DD + 2 * K) % 2], s - DD, wi);
          update(B[(k - DD + K) % K], wi);
        }
      }
    }
  }

  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  if constexpr (!GIVEN_W) {
    // a wave that timed out: the whole workgroup's results are invalid
    __shared__ int any_failed;
    if (tid == 0) any_failed = 0;
    __syncthreads();
    if (failed && lane == 0) any_failed = 1;
    __syncthreads();
    failed = any_failed != 0;
    if (failed && tid == 0 && flag != nullptr)
      __hip_atomic_store(flag, 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  double* yp = ypart + (int64_t)team * ldy + (int64_t)g0 * VN;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int g = tid + u * T;
    if (g < sg)
#pragma unroll
      for (int e = 0; e < VN; ++e) yp[VN * g + e] = failed ? nan : y[u][e];
  }
  if constexpr (!GIVEN_W) {
    // w of the team's rows from the mailbox (every part of the launch is in:
    // each member has taken every step's), in the same member order
    const int nrows = r1 - r0;
    for (int j = member + C * tid; j < nrows; j += C * T) {
      const int s = j / R, r = j - s * R;
      double t = 0.0;
      for (int c = 0; c < C; ++c) {
        const uint64_t* a = mb + (((int64_t)s * C + c) * R + r) * 2;
        t += part_of(ld_dev(a), ld_dev(a + 1));
      }
      w[r0 + j] = failed ? nan : (qprev != nullptr ? t - coef[0] * qprev[r0 + j] : t);
    }
    // the last workgroup to finish advances the generation
    __syncthreads();
    if (tid == 0) {
      const uint32_t done = __hip_atomic_fetch_add(ctr + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (done == gridDim.x - 1) {
        __hip_atomic_store(ctr + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(ctr, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

__global__ void k_team_zero(uint64_t* p, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (int64_t)gridDim.x * 256) p[i] = 0;
}

template <typename TA, typename TP, bool GIVEN_W>
hipError_t launch_team_t(const TA* A, int64_t lda, int64_t m, int64_t n, const TP* p, const double* win, double* w,
                         double* ypart, int64_t ldy, const int* flag, const int* run_if, const double* qprev,
                         const double* coef, void* team, hipStream_t st) {
  constexpr int U = tm_u<TA>(), NB = tm_nb<TA>(), D = tm_d<TA>();
  const TeamShape ts = team_shape(m, n, tm_dtype<TA>());
  if (ts.C == 0 || team == nullptr) return hipErrorInvalidValue;
  uint32_t* ctr = reinterpret_cast<uint32_t*>(team);
  uint64_t* mbox = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(team) + 256);
  long spin_limit = TM_SPIN_LIMIT;
  uint32_t skew = 0;
  if (const char* e = std::getenv("GKB_TEAM_STALL_POLLS")) {   // test of the timeout path
    const long polls = std::atol(e);
    if (polls > 0) {
      spin_limit = polls;
      skew = 1;
    }
  }
  const size_t lds = GIVEN_W ? 0 : (size_t)U * TM_T * Elems<TA>::VN * (Elems<TA>::F32DOT ? 4 : 8);
  if constexpr (!GIVEN_W) {
    const hipError_t attr = allow_dynamic_lds(
        reinterpret_cast<const void*>(&k_gemv_fused_team<TM_T, U, TM_R, NB, D, TA, TP, GIVEN_W>), (int)lds);
    if (attr != hipSuccess) return attr;
  }
  hipLaunchKernelGGL((k_gemv_fused_team<TM_T, U, TM_R, NB, D, TA, TP, GIVEN_W>), dim3(ts.nteams * ts.C),
                     dim3(TM_T), lds, st, A, lda, (int)m, n, p, win, ts.C, ts.rpt, ts.nsteps, w, ypart, ldy,
                     const_cast<int*>(flag), run_if, qprev, coef, mbox, ctr, spin_limit, skew);
  return hipGetLastError();
}

}  // namespace

TeamShape team_shape(int64_t m, int64_t n, int dtype) {
  // C = ceil(n / slice) members: near-equal slices of the 16-byte groups then
  // hold at most `slice` columns
  TeamShape ts{0, 0, 0, 0};
  const int64_t slice = slice_cols(dtype);
  const int64_t C = (n + slice - 1) / slice;
  const int slots = device_cus();   // one member per compute unit
  if (m < 1 || n < 1 || C > TM_CMAX || C > slots) return ts;
  const int64_t want = std::max<int64_t>(1, std::min<int64_t>(slots / C, (m + TM_R - 1) / TM_R));
  const int64_t rpt = (m + want - 1) / want;
  ts.C = (int)C;
  ts.nteams = (int)((m + rpt - 1) / rpt);   // none empty
  ts.rpt = (int)rpt;
  ts.nsteps = (int)((rpt + TM_R - 1) / TM_R);
  return ts;
}

size_t team_bytes(int64_t m, int64_t n, int dtype) {
  const TeamShape ts = team_shape(m, n, dtype);
  if (ts.C == 0) return 0;
  return 256 + (size_t)ts.nteams * ts.nsteps * ts.C * TM_R * 2 * sizeof(uint64_t);
}

hipError_t launch_team_reset(void* team, int64_t m, int64_t n, int dtype, hipStream_t st) {
  const size_t bytes = team_bytes(m, n, dtype);
  if (bytes == 0 || team == nullptr) return hipErrorInvalidValue;
  const int64_t words = (int64_t)(bytes / 8);
  const unsigned blocks = (unsigned)std::min<int64_t>((words + 255) / 256, 1024);
  hipLaunchKernelGGL(k_team_zero, dim3(blocks), dim3(256), 0, st, reinterpret_cast<uint64_t*>(team), words);
  return hipGetLastError();
}

template <typename TP>
hipError_t launch_gemv_fused_team(const void* A, int dtype, int64_t lda, int64_t m, int64_t n, const TP* p,
                                  const double* win, double* w, double* ypart, int64_t ldy, const int* flag,
                                  hipStream_t st, const int* run_if, const double* qprev, const double* coef,
                                  void* team) {
  if (dtype == 0) {
    const double* Ad = reinterpret_cast<const double*>(A);
    return win != nullptr
               ? launch_team_t<double, TP, true>(Ad, lda, m, n, p, win, w, ypart, ldy, flag, run_if, qprev, coef, team,
                                                 st)
               : launch_team_t<double, TP, false>(Ad, lda, m, n, p, win, w, ypart, ldy, flag, run_if, qprev, coef,
                                                  team, st);
  }
  if (dtype == 2) {
    const bf16* Ab = reinterpret_cast<const bf16*>(A);
    return win != nullptr
               ? launch_team_t<bf16, TP, true>(Ab, lda, m, n, p, win, w, ypart, ldy, flag, run_if, qprev, coef, team, st)
               : launch_team_t<bf16, TP, false>(Ab, lda, m, n, p, win, w, ypart, ldy, flag, run_if, qprev, coef, team,
                                                st);
  }
  const float* Af = reinterpret_cast<const float*>(A);
  return win != nullptr
             ? launch_team_t<float, TP, true>(Af, lda, m, n, p, win, w, ypart, ldy, flag, run_if, qprev, coef, team, st)
             : launch_team_t<float, TP, false>(Af, lda, m, n, p, win, w, ypart, ldy, flag, run_if, qprev, coef, team,
                                               st);
}

template hipError_t launch_gemv_fused_team<float>(const void*, int, int64_t, int64_t, int64_t, const float*,
                                                  const double*, double*, double*, int64_t, const int*, hipStream_t,
                                                  const int*, const double*, const double*, void*);
template hipError_t launch_gemv_fused_team<double>(const void*, int, int64_t, int64_t, int64_t, const double*,
                                                   const double*, double*, double*, int64_t, const int*, hipStream_t,
                                                   const int*, const double*, const double*, void*);

}  // namespace gkb
