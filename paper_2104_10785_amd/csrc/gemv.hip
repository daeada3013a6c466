// The two products of the Golub-Kahan recurrence (eq. 2.2) for gfx950:
//
//   gemv_n   w = A p - alpha q        (first line of eq. 2.2)
//   gemv_t   z = A^T q - beta p       (second line), in two deterministic
//            phases: per-row-block partial sums, then a column reduction with
//            the recurrence term fused in
//
// A is row-major (m x n, lda) in float64, float32 or bfloat16; the vectors are
// in the basis precision; outputs and coefficients are float64.  Both kernels
// stream A once with 16-byte non-temporal loads; every reduction has a fixed
// order, so two runs on the same input are bitwise identical.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>

#include "device_common.h"
#include "kernels.h"

namespace gkb {

// ---------------------------------------------------------------- gemv_n
// w[i] = sum_j A[i, j] p[j] - coef[cidx] * qprev[i]  (qprev may be null).
// One wave owns R consecutive rows; lanes stride the row with 16-byte loads
// (VECTOR) or scalars, and p is loaded once per column chunk for all R rows.
template <typename TA, typename TB, int R, bool VECTOR>
__global__ __launch_bounds__(256) void k_gemv_n(const TA* __restrict__ A, int64_t lda, int64_t m,
                                                int64_t n, const TB* __restrict__ p,
                                                const TB* __restrict__ qprev,
                                                const double* __restrict__ coef, int cidx,
                                                double* __restrict__ w, const int* __restrict__ flag) {
  if (flag != nullptr && flag[0] != 0) return;
  using ACC = typename Acc<TA>::type;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * R;
  if (row0 >= m) return;
  const TA* rows[R];
#pragma unroll
  for (int r = 0; r < R; ++r) rows[r] = A + (row0 + r < m ? row0 + r : m - 1) * lda;
  ACC acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0;
  int64_t jtail = 0;
  if (VECTOR) {
    constexpr int VN = Pack<TA>::VN;
    const int64_t nv = n / VN;
    constexpr int U = 2;
    for (int64_t v0 = lane; v0 < nv; v0 += 64 * U) {
      uint4 a[U][R];
      ACC pv[U][VN];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t v = v0 + 64 * u;
        const bool ok = v < nv;
#pragma unroll
        for (int r = 0; r < R; ++r) a[u][r] = ok ? ld_stream(rows[r] + v * VN) : make_uint4(0, 0, 0, 0);
        load_vec<TB, VN>(p + v * VN, ok, pv[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          ACC av[VN];
          Pack<TA>::unpack(a[u][r], av);
#pragma unroll
          for (int e = 0; e < VN; ++e) acc[r] += av[e] * pv[u][e];
        }
      }
    }
    jtail = nv * VN;
  }
  for (int64_t j = jtail + lane; j < n; j += 64) {
    const ACC pj = (ACC)p[j];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] += to_acc(rows[r][j]) * pj;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = wave_sum(acc[r]);
  const double c = (qprev != nullptr) ? coef[cidx] : 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = row0 + r;
    if (lane == r && i < m) {
      double v = (double)acc[r];
      if (qprev != nullptr) v -= c * (double)qprev[i];
      w[i] = v;
    }
  }
}

// ---------------------------------------------------------------- gemv_t
// Phase 1: part[b * ldpart + j] = sum_{i in row block b} A[i, j] q[i].
// A block of 256 threads owns a tile of 256 * VN * VPT consecutive columns:
// thread t reads the VN-element vectors at tile + v * 256 * VN + t * VN for
// v < VPT, so each of the VPT loads of a row is one contiguous 256 * 16-byte
// segment per block.  U rows are in flight per lane.  Few, tall row blocks
// (about two blocks per compute unit in total) keep each block's stream long.
// The vector form needs n to be a multiple of VN (the launcher checks).
template <typename TA, typename TB, bool VECTOR>
__global__ __launch_bounds__(256) void k_gemv_t_part(const TA* __restrict__ A, int64_t lda, int64_t m,
                                                     int64_t n, const TB* __restrict__ q,
                                                     int64_t rows_per_block,
                                                     typename Acc<TA>::type* __restrict__ part,
                                                     int64_t ldpart, const int* __restrict__ flag) {
  if (flag != nullptr && flag[0] != 0) return;
  using ACC = typename Acc<TA>::type;
  constexpr int VN = VECTOR ? Pack<TA>::VN : 1;
  constexpr int VPT = VECTOR ? 2 : 1;
  constexpr int U = VECTOR ? 4 : 4;
  const int64_t tile0 = (int64_t)blockIdx.x * 256 * VN * VPT;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_block;
  int64_t r1 = r0 + rows_per_block;
  if (r1 > m) r1 = m;
  ACC acc[VPT][VN];
#pragma unroll
  for (int v = 0; v < VPT; ++v)
#pragma unroll
    for (int e = 0; e < VN; ++e) acc[v][e] = 0;
  int64_t col[VPT];
  bool full[VPT], any = false;
#pragma unroll
  for (int v = 0; v < VPT; ++v) {
    col[v] = tile0 + (int64_t)v * 256 * VN + (int64_t)threadIdx.x * VN;
    full[v] = col[v] + VN <= n;
    any = any || col[v] < n;
  }
  if (any) {
    for (int64_t i = r0; i < r1; i += U) {
      if (VECTOR) {
        uint4 a[U][VPT];
        ACC qv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool ok = i + u < r1;
          qv[u] = ok ? (ACC)q[i + u] : (ACC)0;
#pragma unroll
          for (int v = 0; v < VPT; ++v)
            a[u][v] = (ok && full[v]) ? ld_stream(A + (i + u) * lda + col[v]) : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
          for (int v = 0; v < VPT; ++v) {
            ACC av[Pack<TA>::VN];
            Pack<TA>::unpack(a[u][v], av);
#pragma unroll
            for (int e = 0; e < VN; ++e) acc[v][e] += av[e] * qv[u];
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (i + u < r1) {
            const ACC qi = (ACC)q[i + u];
            const TA* row = A + (i + u) * lda;
#pragma unroll
            for (int v = 0; v < VPT; ++v)
#pragma unroll
              for (int e = 0; e < VN; ++e)
                if (col[v] + e < n) acc[v][e] += to_acc(row[col[v] + e]) * qi;
          }
        }
      }
    }
  }
  ACC* out = part + (int64_t)blockIdx.y * ldpart;
#pragma unroll
  for (int v = 0; v < VPT; ++v)
#pragma unroll
    for (int e = 0; e < VN; ++e)
      if (col[v] + e < n) out[col[v] + e] = acc[v][e];
}

// Phase 2: z[j] = sum_b part[b][j] - coef[cidx] * pprev[j]  (pprev may be null).
template <typename ACC, typename TB>
__global__ __launch_bounds__(256) void k_gemv_t_reduce(const ACC* __restrict__ part, int64_t ldpart,
                                                       int nb, int64_t n, const TB* __restrict__ pprev,
                                                       const double* __restrict__ coef, int cidx,
                                                       double* __restrict__ z,
                                                       const int* __restrict__ flag) {
  if (flag != nullptr && flag[0] != 0) return;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int b = 0;
  for (; b + 4 <= nb; b += 4) {
    s0 += (double)part[(int64_t)b * ldpart + j];
    s1 += (double)part[(int64_t)(b + 1) * ldpart + j];
    s2 += (double)part[(int64_t)(b + 2) * ldpart + j];
    s3 += (double)part[(int64_t)(b + 3) * ldpart + j];
  }
  for (; b < nb; ++b) s0 += (double)part[(int64_t)b * ldpart + j];
  double s = (s0 + s1) + (s2 + s3);
  if (pprev != nullptr) s -= coef[cidx] * (double)pprev[j];
  z[j] = s;
}

// ================================================================ launchers
template <typename TA, typename TB>
hipError_t launch_gemv_n_t(const TA* A, int64_t lda, int64_t m, int64_t n, const TB* p, const TB* qprev,
                           const double* coef, int cidx, double* w, const int* flag, hipStream_t st) {
  constexpr int R = 4;
  const bool vec = ((lda % Pack<TA>::VN) == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(p) & 15) == 0);
  dim3 grid(nblocks(m, 4 * R));
  if (vec)
    hipLaunchKernelGGL((k_gemv_n<TA, TB, R, true>), grid, dim3(256), 0, st, A, lda, m, n, p, qprev, coef,
                       cidx, w, flag);
  else
    hipLaunchKernelGGL((k_gemv_n<TA, TB, R, false>), grid, dim3(256), 0, st, A, lda, m, n, p, qprev, coef,
                       cidx, w, flag);
  return hipGetLastError();
}

int device_cus() {
  // queried once per device (a partitioned GPU exposes fewer compute units);
  // 256 if the query fails
  constexpr int kDevs = 64;
  static std::atomic<int> cached[kDevs];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (dev >= 0 && dev < kDevs) {
    const int c = cached[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  if (dev >= 0 && dev < kDevs) cached[dev].store(cus, std::memory_order_relaxed);
  return cus;
}

GemvTShape gemv_t_shape(int64_t m, int64_t n, int dtype_bytes) {
  GemvTShape s;
  const int vn = 16 / dtype_bytes;
  s.col_tiles = nblocks(n, 256 * 2 * (int64_t)vn);
  // Two blocks per compute unit in total (never more), so every CU streams
  // the same amount: an extra partial wave of blocks would leave a tail.
  int64_t want = (2 * (int64_t)device_cus()) / s.col_tiles;
  int64_t maxnb = (m + 63) / 64;
  if (want > maxnb) want = maxnb;
  if (want > GEMV_T_MAX_BLOCKS) want = GEMV_T_MAX_BLOCKS;
  if (want < 1) want = 1;
  s.rows_per_block = (m + want - 1) / want;
  s.nb = (int)((m + s.rows_per_block - 1) / s.rows_per_block);
  return s;
}

template <typename TA, typename TB>
hipError_t launch_gemv_t_t(const TA* A, int64_t lda, int64_t m, int64_t n, const TB* q, const TB* pprev,
                           const double* coef, int cidx, double* z, void* part, int64_t ldpart,
                           const int* flag, hipStream_t st) {
  using ACC = typename Acc<TA>::type;
  const bool vec = ((lda % Pack<TA>::VN) == 0) && ((n % Pack<TA>::VN) == 0) &&
                   ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  GemvTShape s = gemv_t_shape(m, n, (int)sizeof(TA));
  ACC* pa = reinterpret_cast<ACC*>(part);
  if (vec) {
    dim3 grid(s.col_tiles, s.nb);
    hipLaunchKernelGGL((k_gemv_t_part<TA, TB, true>), grid, dim3(256), 0, st, A, lda, m, n, q,
                       s.rows_per_block, pa, ldpart, flag);
  } else {
    dim3 grid(nblocks(n, 256), s.nb);
    hipLaunchKernelGGL((k_gemv_t_part<TA, TB, false>), grid, dim3(256), 0, st, A, lda, m, n, q,
                       s.rows_per_block, pa, ldpart, flag);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || z == nullptr) return e;  // z == NULL: the partial sums only
  hipLaunchKernelGGL((k_gemv_t_reduce<ACC, TB>), dim3(nblocks(n, 256)), dim3(256), 0, st, pa, ldpart, s.nb,
                     n, pprev, coef, cidx, z, flag);
  return hipGetLastError();
}

template <typename TB>
hipError_t launch_gemv_n(const MatrixRef& A, const TB* p, const TB* qprev, const double* coef, int cidx,
                         double* w, const int* flag, hipStream_t st) {
  switch (A.dtype) {
    case 0:
      return launch_gemv_n_t<double, TB>((const double*)A.data, A.lda, A.m, A.n, p, qprev, coef, cidx, w,
                                         flag, st);
    case 1:
      return launch_gemv_n_t<float, TB>((const float*)A.data, A.lda, A.m, A.n, p, qprev, coef, cidx, w,
                                        flag, st);
    default:
      return launch_gemv_n_t<bf16, TB>((const bf16*)A.data, A.lda, A.m, A.n, p, qprev, coef, cidx, w,
                                       flag, st);
  }
}

template <typename TB>
hipError_t launch_gemv_t(const MatrixRef& A, const TB* q, const TB* pprev, const double* coef, int cidx,
                         double* z, void* part, int64_t ldpart, const int* flag, hipStream_t st) {
  switch (A.dtype) {
    case 0:
      return launch_gemv_t_t<double, TB>((const double*)A.data, A.lda, A.m, A.n, q, pprev, coef, cidx, z,
                                         part, ldpart, flag, st);
    case 1:
      return launch_gemv_t_t<float, TB>((const float*)A.data, A.lda, A.m, A.n, q, pprev, coef, cidx, z,
                                        part, ldpart, flag, st);
    default:
      return launch_gemv_t_t<bf16, TB>((const bf16*)A.data, A.lda, A.m, A.n, q, pprev, coef, cidx, z,
                                       part, ldpart, flag, st);
  }
}

template hipError_t launch_gemv_n<double>(const MatrixRef&, const double*, const double*, const double*, int,
                                          double*, const int*, hipStream_t);
template hipError_t launch_gemv_n<float>(const MatrixRef&, const float*, const float*, const double*, int,
                                         double*, const int*, hipStream_t);
template hipError_t launch_gemv_t<double>(const MatrixRef&, const double*, const double*, const double*, int,
                                          double*, void*, int64_t, const int*, hipStream_t);
template hipError_t launch_gemv_t<float>(const MatrixRef&, const float*, const float*, const double*, int,
                                         double*, void*, int64_t, const int*, hipStream_t);

}  // namespace gkb
