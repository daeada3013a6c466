// w = A p and y = A^T w in one sweep of A (float32 or bfloat16 storage,
// float64 sums), and the small kernels of the one-sweep Golub-Kahan step.
//
// A Golub-Kahan step needs A p_t and then A^T q_{t+1}; since q_{t+1} is
// A p_t minus multiples of earlier q's (eq. (2.2) and the Gram-Schmidt
// passes), A^T q_{t+1} follows from A^T A p_t and the stored A^T q_j of those
// earlier vectors.  The sweep streams each row of A once: a workgroup owns a
// contiguous range of rows, keeps p in LDS, and for each row forms the dot
// product (reduced across the workgroup in a fixed order) and adds a_i * w_i
// into its float64 partial of A^T w held in registers, while the next rows
// are already loading.  Two forms: the pipelined one (k_gemv_fused_pipe),
// whose row loads stay in flight across each row's reduction, and the
// per-row one (k_gemv_fused), kept for the shapes where it measured faster
// and for the given-w sweep.  The partials of all workgroups are added in
// workgroup order by the consumer (the reduction, recovery or fix-up kernel).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "device_common.h"
#include "fused.h"
#include "fused_device.h"
#include "gemv.h"
#include "lds_attr.h"

namespace gkb {

namespace {

using fdev::f4;
using fdev::wsum;
using fdev::Elems;
using fdev::lds_barrier;
using fdev::RSRC_WORD3;

inline unsigned nblk(int64_t work, int64_t per) { return (unsigned)((work + per - 1) / per); }

// T threads; U = 16-byte column groups per thread (thread t owns groups
// t, t + T, ...); R rows per step, the next D groups of R rows already
// loading.  The float64 partial of A^T w (VN U doubles per thread) stays in
// registers; the rows are converted to float64 once for the dot products and
// again for the update after the barrier, so that only their 16-byte form
// stays live across it (fewer registers, more waves per CU).
// GIVEN_W: w is an input (y = A^T win) and no row needs a reduction.
// TA: float (4 per 16-byte group) or bfloat16 (8 per group, widened exactly
// to float32; Elems).
template <int T, int U, int R, int D, typename TA, typename TP, bool GIVEN_W>
__global__ __launch_bounds__(T) void k_gemv_fused(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                  const TP* __restrict__ p, const double* __restrict__ win,
                                                  int64_t rows_per_block, double* __restrict__ w,
                                                  double* __restrict__ ypart, int64_t ldy,
                                                  const int* __restrict__ flag, const int* __restrict__ run_if,
                                                  const double* __restrict__ qprev,
                                                  const double* __restrict__ coef) {
  constexpr int NWV = T / 64;
  constexpr int VN = Elems<TA>::VN;
  if (flag != nullptr && flag[0] != 0) return;
  if (run_if != nullptr && run_if[0] == 0) return;
  extern __shared__ float pl[];                  // p as float32, n entries (not GIVEN_W)
  __shared__ double red[2][R][NWV];              // [parity][row][wave]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t ng = n / VN;                     // 16-byte groups per row
  if constexpr (!GIVEN_W) {
    // each thread stages the p entries of its own column groups (the only
    // ones it reads back); the loads are independent, so all are in flight
    // together rather than one round trip per entry
    constexpr int UC = U < 4 ? U : 4;   // groups per batch of loads (bounds the temporaries)
#pragma unroll
    for (int u0 = 0; u0 < (U <= 6 ? U : 0); u0 += UC) {
      float v[UC][VN];
#pragma unroll
      for (int c = 0; c < UC; ++c) {
        // clamped to an entry in bounds; stored only if the group exists
        const int64_t g = std::min<int64_t>(tid + (int64_t)(u0 + c) * T, ng - 1);
#pragma unroll
        for (int e = 0; e < VN; ++e) v[c][e] = (float)p[VN * g + e];
      }
#pragma unroll
      for (int c = 0; c < UC; ++c) {
        const int64_t g = tid + (int64_t)(u0 + c) * T;
        if (u0 + c < U && g < ng)
#pragma unroll
          for (int e = 0; e < VN; ++e) pl[VN * g + e] = v[c][e];
      }
    }
    if constexpr (U > 6) {   // the widest shape has no registers to spare: a plain strided copy
#pragma unroll 8
      for (int64_t j = tid; j < n; j += T) pl[j] = (float)p[j];
    }
    __syncthreads();
  }
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = std::min<int64_t>(m, r0 + rows_per_block);
  double y[U][VN];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int e = 0; e < VN; ++e) y[u][e] = 0.0;
  f4 cur[R][U], nxt[R][U], nx2[R][U];
  auto load_rows = [&](int64_t i, f4 (&dst)[R][U]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool ok = i + r < r1;
      const f4* row = reinterpret_cast<const f4*>(A + (ok ? i + r : r0) * lda);   // 16-byte aligned rows
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t g = tid + (int64_t)u * T;
        dst[r][u] = (ok && g < ng) ? __builtin_nontemporal_load(row + g) : f4{0.f, 0.f, 0.f, 0.f};
      }
    }
  };
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int u = 0; u < U; ++u) nxt[r][u] = f4{0.f, 0.f, 0.f, 0.f};
  // a group is loaded only if it will be processed; a stale buffer is
  // never read (the loop ends first)
  if (r0 < r1) load_rows(r0, cur);
  if constexpr (D == 2) {
    if (r0 + R < r1) load_rows(r0 + R, nxt);
  }
  int par = 0;
  for (int64_t i = r0; i < r1; i += R) {
    if constexpr (D == 2) {
      if (i + 2 * R < r1) load_rows(i + 2 * R, nx2);
    } else {
      if (i + R < r1) load_rows(i + R, nxt);
    }
    double wi[R];
    if constexpr (GIVEN_W) {
#pragma unroll
      for (int r = 0; r < R; ++r) wi[r] = i + r < r1 ? win[i + r] : 0.0;
    } else {
      double d[R];
      if constexpr (Elems<TA>::F32DOT) {
        float df[R];
#pragma unroll
        for (int r = 0; r < R; ++r) df[r] = 0.f;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t g = tid + (int64_t)u * T;
          if (g < ng) {
#pragma unroll
            for (int h = 0; h < VN / 4; ++h) {
              const f4 pv = reinterpret_cast<const f4*>(pl)[(VN / 4) * g + h];
#pragma unroll
              for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int r = 0; r < R; ++r) df[r] = fmaf(Elems<TA>::at(cur[r][u], 4 * h + e), pv[e], df[r]);
            }
          }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) d[r] = (double)df[r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) d[r] = 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t g = tid + (int64_t)u * T;
          if (g < ng) {
#pragma unroll
            for (int h = 0; h < VN / 4; ++h) {
              const f4 pv = reinterpret_cast<const f4*>(pl)[(VN / 4) * g + h];
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const double pe = (double)pv[e];
#pragma unroll
                for (int r = 0; r < R; ++r) d[r] += (double)Elems<TA>::at(cur[r][u], 4 * h + e) * pe;
              }
            }
          }
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        d[r] = wsum(d[r]);
        if (lane == 0) red[par][r][wave] = d[r];
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < NWV; ++k) t += red[par][r][k];
        wi[r] = t;   // rows past r1 were loaded as zeros: their wi is 0
        // w gets the recurrence term subtracted (eq. (2.2)); A^T w below uses the plain product
        if (tid == 0 && i + r < r1) w[i + r] = qprev != nullptr ? t - coef[0] * qprev[i + r] : t;
      }
      par ^= 1;   // the next step writes the other half of red: one barrier per step
      // an empty register constraint: the update below converts the rows anew
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int u = 0; u < U; ++u) asm volatile("" : "+v"(cur[r][u]));
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < VN; ++e) y[u][e] += (double)Elems<TA>::at(cur[r][u], e) * wi[r];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        cur[r][u] = nxt[r][u];
        if constexpr (D == 2) nxt[r][u] = nx2[r][u];
      }
  }
  double* yp = ypart + (int64_t)blockIdx.x * ldy;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t g = tid + (int64_t)u * T;
    if (g < ng)
#pragma unroll
      for (int e = 0; e < VN; ++e) yp[VN * g + e] = y[u][e];
  }
}

// The same sweep, pipelined so that the loads of the next rows overlap the
// reduction and barrier of the current ones.  The vector memory counter is
// one in-order counter for loads and stores on this architecture, and the
// compiler waits for all of it (vmcnt(0)) wherever the number of loads issued
// after a value is not fixed: a load that some waves skip, a store between
// loads, two paths into the loop.  So here
//   - every load is issued: buffer loads whose resource covers exactly the
//     row's remaining bytes (0 for rows past the range), so groups past the
//     row end and padding rows read as zeros without touching memory;
//   - the loop has one path: NB buffers of R rows named statically (the loop
//     unrolled by NB), the last group of steps padded with zero rows;
//   - no global store inside the loop: w is staged in LDS and written once at
//     the end (with the recurrence term of eq. (2.2) subtracted there);
//   - the per-step barrier orders LDS only (lds_barrier).
// p is staged zero padded to U T groups, so the dot products need no bounds
// test.  NB - 1 steps of rows are in flight while one is processed.
template <int T, int U, int R, int NB, typename TA, typename TP, bool GIVEN_W>
__global__ __launch_bounds__(T) void k_gemv_fused_pipe(const TA* __restrict__ A, int64_t lda, int m, int64_t n,
                                                       const TP* __restrict__ p, const double* __restrict__ win,
                                                       int rows_per_block, double* __restrict__ w,
                                                       double* __restrict__ ypart, int64_t ldy,
                                                       const int* __restrict__ flag, const int* __restrict__ run_if,
                                                       const double* __restrict__ qprev,
                                                       const double* __restrict__ coef) {
  static_assert(NB >= 2, "at least one step of rows in flight");
  constexpr int NWV = T / 64;
  constexpr int VN = Elems<TA>::VN;
  if (flag != nullptr && flag[0] != 0) return;
  if (run_if != nullptr && run_if[0] == 0) return;
  // p as float32 zero padded to U T groups (not GIVEN_W), then w of the rows
  extern __shared__ double dyn[];
  __shared__ double red[2][R][NWV];              // [parity][row][wave]
  float* pl = reinterpret_cast<float*>(dyn);
  double* wl = dyn + (GIVEN_W ? 0 : U * T * VN / 2);
  // the wave index is uniform: scalar, so its LDS addresses take no vector registers
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ng = (int)(n / VN);
  if constexpr (!GIVEN_W) {
    // the loads of a batch are independent (in flight together); groups past
    // the row get zeros
    constexpr int UC = U < 4 ? U : 4;
#pragma unroll
    for (int u0 = 0; u0 < (U <= 6 ? U : 0); u0 += UC) {
      float v[UC][VN];
#pragma unroll
      for (int c = 0; c < UC; ++c) {
        const int g = std::min(tid + (u0 + c) * T, ng - 1);
#pragma unroll
        for (int e = 0; e < VN; ++e) v[c][e] = (float)p[(int64_t)VN * g + e];
      }
#pragma unroll
      for (int c = 0; c < UC; ++c) {
        const int g = tid + (u0 + c) * T;
        if (u0 + c < U)
#pragma unroll
          for (int e = 0; e < VN; ++e) pl[VN * g + e] = g < ng ? v[c][e] : 0.f;
      }
    }
    if constexpr (U > 6) {
#pragma unroll 8
      for (int j = tid; j < U * T * VN; j += T) pl[j] = j < n ? (float)p[j] : 0.f;
    }
    __syncthreads();
  }
  const int r0 = blockIdx.x * rows_per_block;
  const int r1 = std::min(m, r0 + rows_per_block);
  const int nrows = std::max(r1 - r0, 0);
  const int last = r1 - 1;
  const int rowbytes = (int)(n * (int64_t)sizeof(TA));
  const int64_t ldb = lda * (int64_t)sizeof(TA);
  const char* Ab = reinterpret_cast<const char*>(A);
  const int off0 = tid * 16;
  // rows i .. i + R - 1: group u of a row through a resource that starts at
  // its byte u T 16 and ends at the row's end; only the thread's own offset
  // (tid 16) is range-checked against it
  auto load_step = [&](int i, f4 (&dst)[R][U]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool live = i + r <= last;
      const int ri = __builtin_amdgcn_readfirstlane(std::min(i + r, last));
      const char* row = Ab + (int64_t)ri * ldb;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int nrec = __builtin_amdgcn_readfirstlane(live ? std::max(rowbytes - u * T * 16, 0) : 0);
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void*)(row + u * T * 16), (short)0, nrec, RSRC_WORD3);
        // aux 2: nontemporal (A is streamed once)
        dst[r][u] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, off0, 0, 2));
      }
    }
  };
  double y[U][VN];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int e = 0; e < VN; ++e) y[u][e] = 0.0;
  int par = 0;
  // rows past r1 are zeros: they add nothing, and only their w is not kept
  auto step = [&](f4 (&rows)[R][U], int i) {
    double wi[R];
    if constexpr (GIVEN_W) {
#pragma unroll
      for (int r = 0; r < R; ++r) wi[r] = i + r < r1 ? win[i + r] : 0.0;
    } else {
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
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) d[r] = 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int g = tid + u * T;
#pragma unroll
          for (int h = 0; h < VN / 4; ++h) {
            const f4 pv = reinterpret_cast<const f4*>(pl)[(VN / 4) * g + h];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const double pe = (double)pv[e];
#pragma unroll
              for (int r = 0; r < R; ++r) d[r] += (double)Elems<TA>::at(rows[r][u], 4 * h + e) * pe;
            }
          }
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        d[r] = wsum(d[r]);
        if (lane == 0) red[par][r][wave] = d[r];
      }
      lds_barrier();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < NWV; ++k) t += red[par][r][k];
        wi[r] = t;
        if (tid == 0 && i + r < r1) wl[i + r - r0] = t;
      }
      par ^= 1;   // the next step writes the other half of red: one barrier per step
      // an empty register constraint: the update below converts the rows anew
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int u = 0; u < U; ++u) asm volatile("" : "+v"(rows[r][u]));
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < VN; ++e) y[u][e] += (double)Elems<TA>::at(rows[r][u], e) * wi[r];
  };
  f4 B[NB][R][U];
  if (nrows > 0) {
#pragma unroll
    for (int k = 0; k < NB - 1; ++k) load_step(r0 + k * R, B[k]);
    const int nsteps = (nrows + R - 1) / R;
    for (int s = 0; s < nsteps; s += NB) {
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        load_step(r0 + (s + k + NB - 1) * R, B[(k + NB - 1) % NB]);
        step(B[k], r0 + (s + k) * R);
      }
    }
  }
  if constexpr (!GIVEN_W) {
    __syncthreads();   // the staged w
    for (int j = tid; j < nrows; j += T) {
      const double t = wl[j];
      w[r0 + j] = qprev != nullptr ? t - coef[0] * qprev[r0 + j] : t;
    }
  }
  double* yp = ypart + (int64_t)blockIdx.x * ldy;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int g = tid + u * T;
    if (g < ng)
#pragma unroll
      for (int e = 0; e < VN; ++e) yp[(int64_t)VN * g + e] = y[u][e];
  }
}

// Column sums of the partials with 256 threads per 64 columns: wave v adds
// the partial rows [v nb / 4, (v + 1) nb / 4) for column j = lane, and wave 0
// adds the four sums in wave order (a fixed order).  `extra` (may be null)
// gives each wave a second per-column sum to reduce the same way, over
// columns [v t / 4, (v + 1) t / 4) of G weighted by the coefficient of that
// column (coef(j)).  Returns (sum of partials, sum of extra) on wave 0.
constexpr int RCOLS = 64;

template <typename CoefF>
__device__ __forceinline__ void column_sums(const double* __restrict__ ypart, int nb, int64_t ldy, int64_t j, bool in,
                                            const double* G, int64_t ldg, int t, CoefF coef, double* out_y,
                                            double* out_g) {
  __shared__ double ps[2][4][RCOLS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double sy = 0.0, sg = 0.0;
  if (in) {
    // eight (four) independent sums, so that as many loads are in flight per
    // wave; combined in a fixed order
    const int b0 = (int)((int64_t)nb * wave / 4), b1 = (int)((int64_t)nb * (wave + 1) / 4);
    double s[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k] = 0.0;
    int b = b0;
    for (; b + 7 < b1; b += 8) {
#pragma unroll
      for (int k = 0; k < 8; ++k) s[k] += ypart[(int64_t)(b + k) * ldy + j];
    }
#pragma unroll
    for (int k = 0; k < 7; ++k)
      if (b + k < b1) s[k] += ypart[(int64_t)(b + k) * ldy + j];
    sy = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    if (G != nullptr) {
      const int c0 = t * wave / 4, c1 = t * (wave + 1) / 4;
      double g[4] = {0.0, 0.0, 0.0, 0.0};
      int c = c0;
      for (; c + 3 < c1; c += 4) {
#pragma unroll
        for (int k = 0; k < 4; ++k) g[k] += G[(int64_t)(c + k) * ldg + j] * coef(c + k);
      }
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (c + k < c1) g[k] += G[(int64_t)(c + k) * ldg + j] * coef(c + k);
      sg = (g[0] + g[1]) + (g[2] + g[3]);
    }
  }
  ps[0][wave][lane] = sy;
  ps[1][wave][lane] = sg;
  __syncthreads();
  if (wave == 0) {
    *out_y = ((ps[0][0][lane] + ps[0][1][lane]) + ps[0][2][lane]) + ps[0][3][lane];
    *out_g = ((ps[1][0][lane] + ps[1][1][lane]) + ps[1][2][lane]) + ps[1][3][lane];
  }
}

__global__ __launch_bounds__(256) void k_fused_reduce(const double* __restrict__ ypart, int nb, int64_t ldy,
                                                      int64_t n, double* __restrict__ y,
                                                      const int* __restrict__ flag, const int* __restrict__ run_if) {
  if (flag != nullptr && flag[0] != 0) return;
  if (run_if != nullptr && run_if[0] == 0) return;
  const int64_t j = (int64_t)blockIdx.x * RCOLS + (threadIdx.x & 63);
  double sy, sg;
  column_sums(ypart, nb, ldy, j, j < n, nullptr, 0, 0, [](int) { return 0.0; }, &sy, &sg);
  if (threadIdx.x < 64 && j < n) y[j] = sy;
}

template <int T, int U, int R, int D, typename TA, typename TP, bool GIVEN_W>
hipError_t launch_v(const TA* A, int64_t lda, int64_t m, int64_t n, const TP* p, const double* win, double* w,
                    double* ypart, int64_t ldy, const int* flag, const int* run_if, hipStream_t st,
                    const double* qprev = nullptr, const double* coef = nullptr) {
  if constexpr (!GIVEN_W) {
    const hipError_t attr =
        allow_dynamic_lds(reinterpret_cast<const void*>(&k_gemv_fused<T, U, R, D, TA, TP, GIVEN_W>),
                          (int)(FUSED_NMAX * 4));
    if (attr != hipSuccess) return attr;
  }
  const int nb = fused_blocks(m, n, 1);
  const int64_t rpb = (m + nb - 1) / nb;
  hipLaunchKernelGGL((k_gemv_fused<T, U, R, D, TA, TP, GIVEN_W>), dim3(nb), dim3(T), GIVEN_W ? 0 : (size_t)n * 4, st, A,
                     lda, m, n, p, win, rpb, w, ypart, ldy, flag, run_if, qprev, coef);
  return hipGetLastError();
}

template <int T, int U, int R, int D, typename TA, typename TP>
hipError_t launch_u(const TA* A, int64_t lda, int64_t m, int64_t n, const TP* p, const double* win, double* w,
                    double* ypart, int64_t ldy, const int* flag, const int* run_if, hipStream_t st,
                    const double* qprev, const double* coef) {
  if (win != nullptr)
    return launch_v<T, U, R, D, TA, TP, true>(A, lda, m, n, p, win, w, ypart, ldy, flag, run_if, st);
  return launch_v<T, U, R, D, TA, TP, false>(A, lda, m, n, p, win, w, ypart, ldy, flag, run_if, st, qprev, coef);
}

// Launch shape by row length (measured on MI355X): short rows take several
// rows per step and two or four workgroups per CU, so that enough bytes are
// in flight per barrier; long rows take one row per step with up to 1024
// threads, the per-thread share of A^T w held in registers without spills,
// and two rows ahead in flight where the registers allow it (up to 4 groups
// per thread).
struct FusedShape {
  int T, U, R, bpc;
};

FusedShape fused_shape(int64_t n) {
  const int64_t ng = n / 4;
  if (ng <= 128) return {128, 1, 16, 4};
  if (ng <= 256) return {256, 1, 8, 2};
  if (ng <= 512) return {256, 2, 4, 2};
  if (ng <= 1024) return {256, 4, 2, 2};
  if (ng <= 2048) return {512, 4, 1, 2};
  if (ng <= 5120) return {1024, (int)((ng + 1023) / 1024), 1, 1};
  return {768, 8, 1, 1};
}

// The pipelined sweep: LDS holds p (padded) and the w of the workgroup's rows.
constexpr int PIPE_LDS_MAX = 160 * 1024 - 4096;   // dynamic LDS; the rest covers red[][][]

template <int T, int U, int R, int NB, typename TA>
size_t pipe_lds(int64_t m, int64_t n, bool given_w) {
  const int nb = fused_blocks(m, n, 1);
  const int64_t rpb = (m + nb - 1) / nb;
  return given_w ? 0 : (size_t)U * T * Elems<TA>::VN * 4 + (size_t)rpb * 8;
}

// true if the pipelined form takes this launch (LDS within one workgroup's
// share of the CU; the row count in 32 bits)
template <int T, int U, int R, int NB, typename TA>
bool pipe_fits(int64_t m, int64_t n, bool given_w) {
  const int bpc = fused_shape(n).bpc;
  return m < (int64_t(1) << 30) && n / Elems<TA>::VN <= (int64_t)U * T &&
         pipe_lds<T, U, R, NB, TA>(m, n, given_w) <= (size_t)std::min(PIPE_LDS_MAX, 160 * 1024 / bpc - 4096);
}

template <int T, int U, int R, int NB, typename TA, typename TP, bool GIVEN_W>
hipError_t launch_p(const TA* A, int64_t lda, int64_t m, int64_t n, const TP* p, const double* win, double* w,
                    double* ypart, int64_t ldy, const int* flag, const int* run_if, hipStream_t st,
                    const double* qprev = nullptr, const double* coef = nullptr) {
  if (!pipe_fits<T, U, R, NB, TA>(m, n, GIVEN_W)) return hipErrorInvalidValue;
  if constexpr (!GIVEN_W) {
    const hipError_t attr =
        allow_dynamic_lds(reinterpret_cast<const void*>(&k_gemv_fused_pipe<T, U, R, NB, TA, TP, GIVEN_W>),
                          PIPE_LDS_MAX);
    if (attr != hipSuccess) return attr;
  }
  const int nb = fused_blocks(m, n, 1);
  const int rpb = (int)((m + nb - 1) / nb);
  const size_t lds = pipe_lds<T, U, R, NB, TA>(m, n, GIVEN_W);
  hipLaunchKernelGGL((k_gemv_fused_pipe<T, U, R, NB, TA, TP, GIVEN_W>), dim3(nb), dim3(T), lds, st, A, lda, (int)m,
                     n, p, win, rpb, w, ypart, ldy, flag, run_if, qprev, coef);
  return hipGetLastError();
}

template <int T, int U, int R, int NB, typename TA, typename TP>
hipError_t launch_pu(const TA* A, int64_t lda, int64_t m, int64_t n, const TP* p, const double* win, double* w,
                     double* ypart, int64_t ldy, const int* flag, const int* run_if, hipStream_t st,
                     const double* qprev, const double* coef) {
  if (win != nullptr)
    return launch_p<T, U, R, NB, TA, TP, true>(A, lda, m, n, p, win, w, ypart, ldy, flag, run_if, st);
  return launch_p<T, U, R, NB, TA, TP, false>(A, lda, m, n, p, win, w, ypart, ldy, flag, run_if, st, qprev, coef);
}

// Coefficient of column j in w = A p - Q c: the Gram-Schmidt sums c[j] plus
// the recurrence term xc[j - x0] for x0 <= j < x0 + nx.
__device__ __forceinline__ double coef_total(const double* __restrict__ c, int j, const double* __restrict__ xc,
                                             int x0, int nx) {
  const int k = j - x0;
  return (k >= 0 && k < nx) ? c[j] + xc[k] : c[j];
}

// G's columns 0..t-1 are read and column tq (>= t) is written: no overlap.
// Block 0 also runs the guard (it reads only coefficients and bounds).  With
// NORM, the launch first completes the left vector's normalisation (norm from
// the Gram-Schmidt partial sums, breakdown tests, q_tq = w / beta written by
// a grid-stride loop), so beta is its own result instead of beta[0].
template <bool NORM>
__global__ __launch_bounds__(256) void k_onepass_recover(NormArgs na, const double* __restrict__ ypart, int nb,
                                                         int64_t ldy, double* G, int64_t ldg, int t,
                                                         const double* __restrict__ c,
                                                         const double* __restrict__ xc, int x0, int nx,
                                                         const double* __restrict__ beta, int tq,
                                                         const double* __restrict__ pprev, double* __restrict__ z,
                                                         int64_t n, double* __restrict__ err,
                                                         const double* __restrict__ sig, double eps0, double tau,
                                                         int* __restrict__ refresh, int* __restrict__ flag) {
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (flag != nullptr && flag[0] != 0) {
    if (lead) refresh[0] = 0;
    return;
  }
  double b, s;
  if constexpr (NORM) {
    __shared__ double red[4];
    b = norm_test(na.normpart, na.nparts, na.sig_in, na.sig_out, na.eps, na.relative, 1, flag, na.code, na.index,
                  na.coef_out, lead, red, &s);
    if (b < 0.0) {  // breakdown or a non-finite norm: nothing to recover
      if (lead) refresh[0] = 0;
      return;
    }
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < na.len; i += (int64_t)gridDim.x * 256)
      na.out[i] = na.x[i] / b;
  } else {
    b = beta[0];
    s = sig[0];
  }
  if (lead) {
    double sce = 0.0, sc = 0.0;
    for (int j = 0; j < t; ++j) {
      const double a = fabs(coef_total(c, j, xc, x0, nx));
      sce += a * err[j];
      sc += a;
    }
    const double e = (sce + eps0 * (s * s + s * sc)) / b;
    if (e > tau * s) {
      refresh[0] = 1;
      refresh[1] += 1;
      err[tq] = eps0 * s;
    } else {
      refresh[0] = 0;
      err[tq] = e;
    }
  }
  const int64_t i = (int64_t)blockIdx.x * RCOLS + (threadIdx.x & 63);
  double y, acc;
  column_sums(ypart, nb, ldy, i, i < n, G, ldg, t, [&](int j) { return coef_total(c, j, xc, x0, nx); }, &y, &acc);
  if (threadIdx.x >= 64 || i >= n) return;
  const double g = (y - acc) / b;
  G[(int64_t)tq * ldg + i] = g;
  z[i] = g - b * pprev[i];
}

__global__ void k_err_set(double* err, int idx, const double* __restrict__ sig, double eps0,
                          const int* __restrict__ flag) {
  if (threadIdx.x != 0 || (flag != nullptr && flag[0] != 0)) return;
  err[idx] = eps0 * sig[0];
}

__global__ void k_err_restart(const double* __restrict__ src, int nq, double* __restrict__ dst, int l) {
  __shared__ double mx;
  if (threadIdx.x == 0) {
    double v = 0.0;
    for (int j = 0; j < nq; ++j) v = fmax(v, src[j]);
    mx = v * sqrt((double)nq);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < l; j += blockDim.x) dst[j] = mx;
}

__global__ __launch_bounds__(256) void k_onepass_fix(const double* __restrict__ ypart, int nb, int64_t ldy,
                                                     double* G, int64_t ldg, int tq, const double* __restrict__ beta,
                                                     const double* __restrict__ pprev, double* __restrict__ z,
                                                     int64_t n, const int* __restrict__ flag,
                                                     const int* __restrict__ refresh) {
  if ((flag != nullptr && flag[0] != 0) || refresh[0] == 0) return;
  const int64_t i = (int64_t)blockIdx.x * RCOLS + (threadIdx.x & 63);
  double g, unused;
  column_sums(ypart, nb, ldy, i, i < n, nullptr, 0, 0, [](int) { return 0.0; }, &g, &unused);
  if (threadIdx.x >= 64 || i >= n) return;
  G[(int64_t)tq * ldg + i] = g;
  z[i] = g - beta[0] * pprev[i];
}

__global__ __launch_bounds__(256) void k_narrow(const double* __restrict__ src, int64_t len,
                                                float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < len) dst[i] = (float)src[i];
}

}  // namespace

bool fused_ok(int64_t m, int64_t n, int64_t lda, const void* A, int dtype) {
  if (dtype < 0 || dtype > 2) return false;
  const int64_t vn = dtype == 2 ? 8 : (dtype == 1 ? 4 : 2);
  if (m < 1 || m >= (int64_t(1) << 30) || n < vn || n % vn != 0 || lda % vn != 0 ||
      (reinterpret_cast<uintptr_t>(A) & 15) != 0)
    return false;
  if (!team_form(n, dtype)) return true;
  return n <= (dtype == 0 ? FUSED_TEAM_NMAX_F64 : FUSED_TEAM_NMAX) && team_shape(m, n, dtype).C > 0;
}

int fused_blocks(int64_t m, int64_t n, int dtype) {
  if (team_form(n, dtype)) return std::max(1, team_shape(m, n, dtype).nteams);
  // bpc workgroups per compute unit, each an equal share of the rows
  return (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)fused_shape(n).bpc * device_cus(), m));
}

template <typename TP>
hipError_t launch_gemv_fused(const void* A, int dtype, int64_t lda, int64_t m, int64_t n, const TP* p,
                             const double* win, double* w, double* y, double* ypart, int64_t ldy, const int* flag,
                             hipStream_t st, const int* run_if, const double* qprev, const double* coef,
                             void* team) {
  const FusedShape fs = fused_shape(n);
  hipError_t e;
  const bool gw = win != nullptr;
  if (team_form(n, dtype)) {
    e = launch_gemv_fused_team<TP>(A, dtype, lda, m, n, p, win, w, ypart, ldy, flag, st, run_if, qprev, coef, team);
  } else
  // Shapes measured on MI355X (w = A p and A^T w, float64 p): the pipelined
  // form where it is faster, the per-row barrier form elsewhere and for the
  // given-w sweep (w read, no reduction), and wherever the pipelined form's
  // LDS (p and the staged w of a workgroup's rows) would not fit.
  if (dtype == 2) {
    // bfloat16: half the bytes per row, so several rows per barrier
    const bf16* Ab = reinterpret_cast<const bf16*>(A);
#define GKB_FUSED(T, U, R, D) \
  e = launch_u<T, U, R, D, bf16, TP>(Ab, lda, m, n, p, win, w, ypart, ldy, flag, run_if, st, qprev, coef)
#define GKB_PIPE_OR(T, U, R, NB, OT, OU, OR, OD)                                                      \
  if (!gw && pipe_fits<T, U, R, NB, bf16>(m, n, false))                                               \
    e = launch_p<T, U, R, NB, bf16, TP, false>(Ab, lda, m, n, p, win, w, ypart, ldy, flag, run_if, st, \
                                               qprev, coef);                                          \
  else GKB_FUSED(OT, OU, OR, OD)
    // (ms, old -> pipelined: n = 1000 2.06 -> 1.64; 2000 1.22 -> 1.01;
    // 4000 0.99 -> 0.72; 8000 1.01 -> 0.67; 16000 0.83 -> 0.65;
    // 20000 0.81 -> 0.64; 24576 0.75 -> 0.62, at 2-4 GB of A)
    if (n <= 1024) { GKB_PIPE_OR(128, 1, 16, 2, 128, 1, 16, 1); }
    else if (n <= 2048) { GKB_PIPE_OR(256, 1, 8, 2, 256, 1, 8, 1); }
    else if (n <= 4096) { GKB_PIPE_OR(256, 2, 2, 2, 256, 2, 4, 1); }
    else if (n <= 8192) { GKB_PIPE_OR(512, 2, 2, 2, 512, 2, 4, 1); }
    else if (n <= 16384) { GKB_PIPE_OR(512, 4, 2, 2, 512, 4, 3, 1); }
    else if (n <= 20480) { GKB_PIPE_OR(512, 5, 1, 2, 512, 5, 3, 1); }
    else { GKB_PIPE_OR(512, 6, 1, 3, 512, 6, 2, 1); }
#undef GKB_PIPE_OR
#undef GKB_FUSED
  } else {
    const float* Af = reinterpret_cast<const float*>(A);
#define GKB_FUSED(T, U, R, D) \
  e = launch_u<T, U, R, D, float, TP>(Af, lda, m, n, p, win, w, ypart, ldy, flag, run_if, st, qprev, coef)
#define GKB_PIPE_OR(T, U, R, NB, OT, OU, OR, OD)                                                       \
  if (!gw && pipe_fits<T, U, R, NB, float>(m, n, false))                                               \
    e = launch_p<T, U, R, NB, float, TP, false>(Af, lda, m, n, p, win, w, ypart, ldy, flag, run_if, st, \
                                                qprev, coef);                                          \
  else GKB_FUSED(OT, OU, OR, OD)
    // (ms, old -> pipelined: 16-byte groups per row <= 128 1.01 -> 0.85;
    // <= 256 1.11 -> 0.88; <= 512 0.77 -> 0.64; <= 1024 0.67 -> 0.63;
    // <= 3072 0.67 -> 0.61; <= 4096 0.62 -> 0.61; <= 5120 0.67 -> 0.62, at
    // 3-4 GB of A; the old form stays at 2048 groups (within the variation
    // between runs) and 6144 (0.67 against 1.03: the pipelined form spills),
    // and for the given-w sweep at 5000 groups (512 threads: fewer waves to
    // skip; 0.63 against 0.64))
    if (fs.T == 128) { GKB_PIPE_OR(128, 1, 8, 2, 128, 1, 16, 1); }
    else if (fs.T == 256 && fs.U == 1) { GKB_PIPE_OR(256, 1, 8, 2, 256, 1, 8, 1); }
    else if (fs.T == 256 && fs.U == 2) { GKB_PIPE_OR(256, 2, 2, 2, 256, 2, 4, 1); }
    else if (fs.T == 256) { GKB_PIPE_OR(256, 4, 1, 2, 256, 4, 2, 1); }
    else if (fs.T == 512) GKB_FUSED(512, 4, 1, 2);
    else if (fs.T == 768) GKB_FUSED(768, 8, 1, 1);
    else if (fs.U <= 3) { GKB_PIPE_OR(1024, 3, 1, 2, 1024, 3, 1, 2); }
    else if (fs.U == 4) { GKB_PIPE_OR(512, 8, 1, 2, 1024, 4, 1, 2); }
    else if (gw) e = launch_v<512, 10, 1, 1, float, TP, true>(Af, lda, m, n, p, win, w, ypart, ldy, flag, run_if, st);
    else { GKB_PIPE_OR(512, 10, 1, 2, 1024, 5, 1, 1); }
#undef GKB_PIPE_OR
#undef GKB_FUSED
  }
  if (e != hipSuccess || y == nullptr) return e;
  hipLaunchKernelGGL(k_fused_reduce, dim3(nblk(n, RCOLS)), dim3(256), 0, st, ypart, fused_blocks(m, n, dtype), ldy, n, y,
                     flag, run_if);
  return hipGetLastError();
}

template hipError_t launch_gemv_fused<float>(const void*, int, int64_t, int64_t, int64_t, const float*, const double*,
                                             double*, double*, double*, int64_t, const int*, hipStream_t,
                                             const int*, const double*, const double*, void*);
template hipError_t launch_gemv_fused<double>(const void*, int, int64_t, int64_t, int64_t, const double*,
                                              const double*, double*, double*, double*, int64_t, const int*,
                                              hipStream_t, const int*, const double*, const double*, void*);

hipError_t launch_onepass_recover(const double* ypart, int nb, int64_t ldy, double* G, int64_t ldg, int t,
                                  const double* c, const double* xc, int x0, int nx, const double* beta, int tq,
                                  const double* pprev, double* z, int64_t n, double* err, const double* sig,
                                  double eps0, double tau, int* refresh, int* flag, hipStream_t st,
                                  const NormArgs* norm) {
  if (norm != nullptr)
    hipLaunchKernelGGL(k_onepass_recover<true>, dim3(nblk(n, RCOLS)), dim3(256), 0, st, *norm, ypart, nb, ldy, G, ldg,
                       t, c, xc, x0, nx, beta, tq, pprev, z, n, err, sig, eps0, tau, refresh, flag);
  else
    hipLaunchKernelGGL(k_onepass_recover<false>, dim3(nblk(n, RCOLS)), dim3(256), 0, st, NormArgs(), ypart, nb, ldy, G,
                       ldg, t, c, xc, x0, nx, beta, tq, pprev, z, n, err, sig, eps0, tau, refresh, flag);
  return hipGetLastError();
}

hipError_t launch_err_set(double* err, int idx, const double* sig, double eps0, const int* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_err_set, dim3(1), dim3(64), 0, st, err, idx, sig, eps0, flag);
  return hipGetLastError();
}

hipError_t launch_err_restart(const double* src, int nq, double* dst, int l, hipStream_t st) {
  hipLaunchKernelGGL(k_err_restart, dim3(1), dim3(64), 0, st, src, nq, dst, l);
  return hipGetLastError();
}

hipError_t launch_onepass_fix(const double* ypart, int nb, int64_t ldy, double* G, int64_t ldg, int tq,
                              const double* beta, const double* pprev, double* z, int64_t n, const int* flag,
                              const int* refresh, hipStream_t st) {
  hipLaunchKernelGGL(k_onepass_fix, dim3(nblk(n, RCOLS)), dim3(256), 0, st, ypart, nb, ldy, G, ldg, tq, beta, pprev,
                     z, n, flag, refresh);
  return hipGetLastError();
}

hipError_t launch_narrow(const double* src, int64_t len, float* dst, hipStream_t st) {
  if (len <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_narrow, dim3(nblk(len, 256)), dim3(256), 0, st, src, len, dst);
  return hipGetLastError();
}

}  // namespace gkb
