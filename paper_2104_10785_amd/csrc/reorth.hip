// Full reorthogonalisation of a new Golub-Kahan vector against the basis built
// so far (Algorithm 1's projection steps; two classical Gram-Schmidt passes)
// in three launches instead of one launch per dot product, reduction and
// update.
//
// A workgroup owns a contiguous slice of the vector (gs_split) and keeps it in
// LDS for the whole launch.  Each pass needs the full coefficient vector
// h = V^T x, a reduction over all slices; that reduction is the launch
// boundary: a launch writes its slices' partial dot products, and the next
// launch has every workgroup add all partials in the same fixed order, so all
// of them hold bitwise the same h without a separate reduction launch.  The
// middle launch updates its slice with the first pass's h and forms the
// second pass's partial dots from the updated slice, reading the basis slice
// once into LDS for both uses when it fits.  Every sum has a fixed order, so
// results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "device_common.h"
#include "kernels.h"
#include "lds_attr.h"
#include "reorth.h"

namespace gkb {

GsSplit gs_split(int64_t len) {
  int64_t G = std::min<int64_t>(GS_MAX_G, std::max<int64_t>(1, (len + 255) / 256));
  if ((len + G - 1) / G > GS_MAX_ROWS) G = (len + GS_MAX_ROWS - 1) / GS_MAX_ROWS;
  GsSplit s;
  s.G = (int)G;
  s.rows = std::max<int64_t>(1, (len + G - 1) / G);
  return s;
}

int64_t gs_partial_rows(int64_t len) {
  return std::max<int64_t>(2 * (int64_t)gs_split(len).G, dots_chunks(len)) + 1;
}

namespace {

constexpr int GS_T = 256;                 // threads per workgroup
constexpr int GS_HCH = 1024;              // coefficients held in LDS at a time
constexpr int GS_COLS = 32;               // columns per workgroup in the first launch's dots
constexpr size_t GS_STAGE_BYTES = 120 * 1024;  // basis slice staged in LDS up to this size
constexpr size_t GS_LDS_MAX = 160 * 1024;
// below GS_WIDE_G slices, a pass with more than GS_WIDE_WORK basis entries per
// slice spreads its columns over workgroups instead (see launch_gs2)
constexpr int GS_WIDE_G = 64;
constexpr int GS_SHORT_G = 16;  // fewer slices than this: always the column-spread kernels
// longer slices than this (vectors over 256 x 512 entries): the column-spread
// kernels too, whose dots run over many more workgroups; a slice's dots and
// update would run as long chains of dependent loads in its four waves
// (measured: the sparse 1000000 x 200000 solve, slices of 3907 and 782 rows,
// 103 ms against 75 ms)
constexpr int64_t GS_SLICE_MAX = 512;
constexpr int64_t GS_WIDE_WORK = 32768;

// LDS of a launch: the slice (rows doubles), a chunk of coefficients, the
// reduction buffer (4 x 64) and the column-part buffer (256), then the staged
// basis slice.
size_t gs_lds_base(int64_t rows) { return (size_t)rows * 8 + (size_t)(GS_HCH + 512) * 8; }

// h[j] = sum over the G partial rows of P (row stride ldh) of column j, j < t:
// one wave per column, lanes stride the rows with four accumulators (rows b =
// lane + 64 (4q + r) into a_r), combined as (a0 + a1) + (a2 + a3) and then by
// a fixed-order wave reduction.  acc (optional): acc[j] = h[j] (add = 0) or
// acc[j] += h[j] (add = 1).
__global__ __launch_bounds__(256) void k_gs_reduce(const double* __restrict__ P, int ldh, int G, int t,
                                                   double* __restrict__ h, double* __restrict__ acc, int add,
                                                   const int* __restrict__ flag) {
  if (flag != nullptr && flag[0] != 0) return;
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= t) return;
  const double* col = P + j;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = lane; b < G; b += 256) {
    double v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = b + 64 * r < G ? col[(int64_t)(b + 64 * r) * ldh] : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] += v[r];
  }
  const double s = wave_sum((a[0] + a[1]) + (a[2] + a[3]));
  if (lane == 0) {
    h[j] = s;
    if (acc != nullptr) acc[j] = add ? acc[j] + s : s;
  }
}

// Basis entry (column j, slice row i): from the staged copy or from memory.
template <typename TB, bool STAGED>
__device__ __forceinline__ double vat(const TB* __restrict__ V, int64_t ldv, const TB* Vs, int nr, int64_t r0,
                                      int j, int i) {
  if constexpr (STAGED) return (double)Vs[(int64_t)j * nr + i];
  return (double)V[(int64_t)j * ldv + r0 + i];
}

// xs[i] -= sum_{j in [c0, c0 + nc)} V[j][i] hs[j - c0] over the slice rows.
// Slices of up to 64 (128) rows split the columns into four (two) contiguous
// parts whose corrections are added in part order; longer slices give each
// thread whole rows.
template <typename TB, bool STAGED>
__device__ void gs_update(const TB* __restrict__ V, int64_t ldv, const TB* Vs, int c0, int nc, int64_t r0, int nr,
                          double* xs, const double* hs, double* cp) {
  const int RS = nr <= 64 ? 64 : (nr <= 128 ? 128 : GS_T);
  const int NCP = GS_T / RS;
  const int part = threadIdx.x / RS, slot = threadIdx.x % RS;
  const int per = (nc + NCP - 1) / NCP;
  const int j0 = part * per;
  const int j1 = min(nc, j0 + per);
  for (int i = slot; i < nr; i += RS) {
    double c = 0.0;
    int j = j0;
    for (; j + 8 <= j1; j += 8) {  // eight loads in flight, then the products in column order
      double v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = vat<TB, STAGED>(V, ldv, Vs, nr, r0, c0 + j + k, i);
#pragma unroll
      for (int k = 0; k < 8; ++k) c += v[k] * hs[j + k];
    }
    for (; j < j1; ++j) c += vat<TB, STAGED>(V, ldv, Vs, nr, r0, c0 + j, i) * hs[j];
    if (NCP == 1)
      xs[i] -= c;
    else
      cp[part * RS + slot] = c;
  }
  __syncthreads();
  if (NCP > 1 && part == 0 && slot < nr) {
    double c = cp[slot] + cp[RS + slot];
    if (NCP == 4) c = (cp[slot] + cp[RS + slot]) + (cp[2 * RS + slot] + cp[3 * RS + slot]);
    xs[slot] -= c;
  }
  __syncthreads();
}

// Pout[j] = sum over the slice rows of V[j][i] xs[i], jb <= j < je (default
// all t): wave w takes columns jb + w*8 .. jb + w*8+7, then +32; lanes stride
// the rows, two rows per lane at a time, so sixteen loads per lane are in
// flight; one wave reduction per column.
template <typename TB, bool STAGED>
__device__ void gs_dots(const TB* __restrict__ V, int64_t ldv, const TB* Vs, int t, int64_t r0, int nr,
                        const double* xs, double* __restrict__ Pout, int jb = 0, int je = -1) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (je < 0) je = t;
  for (int j0 = jb + wave * 8; j0 < je; j0 += 32) {
    const int nj = min(8, je - j0);
    double a[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) a[c] = 0.0;
    for (int i = lane; i < nr; i += 128) {
      const int i2 = i + 64;
      const bool in2 = i2 < nr;
      const double x1 = xs[i];
      const double x2 = in2 ? xs[i2] : 0.0;
      double v1[8], v2[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        v1[c] = c < nj ? vat<TB, STAGED>(V, ldv, Vs, nr, r0, j0 + c, i) : 0.0;
        v2[c] = (c < nj && in2) ? vat<TB, STAGED>(V, ldv, Vs, nr, r0, j0 + c, i2) : 0.0;
      }
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        a[c] += v1[c] * x1;
        a[c] += v2[c] * x2;
      }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) a[c] = wave_sum(a[c]);
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c < nj) Pout[j0 + c] = a[c];
    }
  }
}

struct Slice {
  int64_t r0;
  int nr;
};
__device__ __forceinline__ Slice slice_of(int64_t len, int64_t rows) {
  Slice s;
  s.r0 = (int64_t)blockIdx.x * rows;
  const int64_t left = len - s.r0;
  s.nr = (int)(left <= 0 ? 0 : (left < rows ? left : rows));
  return s;
}

// First launch: form the slice (pre-step), then the first pass's partial dots.
template <typename TB, typename TP, int PRE>
__global__ __launch_bounds__(GS_T) void k_gs_first(const TB* __restrict__ V, int64_t ldv, int t, int64_t len,
                                                   int64_t rows, double* __restrict__ x, double* __restrict__ P1,
                                                   int ldh, const double* __restrict__ rho, int l,
                                                   const TP* __restrict__ part, int64_t ldpart, int nparts,
                                                   const TB* __restrict__ prev, const double* __restrict__ coef,
                                                   int cidx, const int* __restrict__ run_if,
                                                   double* __restrict__ gcol, const int* __restrict__ flag) {
  if (flag != nullptr && flag[0] != 0) return;
  extern __shared__ double sm[];
  double* xs = sm;
  double* hs = xs + rows;
  double* cp = hs + GS_HCH + 256;
  const Slice S = slice_of(len, rows);
  // blockIdx.y: a block of 32 columns of the dots; every column block forms the
  // slice (the same values), the first one writes it back
  const bool writer = blockIdx.y == 0;
  const bool sum_parts = PRE == GS_PRE_TSUM || (PRE == GS_PRE_FIX && run_if[0] != 0);
  for (int i = threadIdx.x; i < S.nr; i += GS_T) {
    const int64_t gi = S.r0 + i;
    double v;
    if (sum_parts) {
      // the row-block partial sums of A^T q, added as eight interleaved sums
      // (eight loads in flight per thread), combined in a fixed order
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = 0.0;
      for (int b = 0; b < nparts; b += 8) {
        double pv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) pv[u] = b + u < nparts ? (double)part[(int64_t)(b + u) * ldpart + gi] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += pv[u];
      }
      v = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
      if (PRE == GS_PRE_FIX && writer) gcol[gi] = v;
      if (prev != nullptr) v -= coef[cidx] * (double)prev[gi];
    } else {
      v = x[gi];
    }
    xs[i] = v;
  }
  if constexpr (PRE == GS_PRE_RHO) {
    for (int j = threadIdx.x; j < l; j += GS_T) hs[j] = rho[j];
  }
  __syncthreads();
  if constexpr (PRE == GS_PRE_RHO) gs_update<TB, false>(V, ldv, nullptr, 0, l, S.r0, S.nr, xs, hs, cp);
  if (writer && (PRE == GS_PRE_RHO || sum_parts)) {
    for (int i = threadIdx.x; i < S.nr; i += GS_T) x[S.r0 + i] = xs[i];
  }
  const int jb = blockIdx.y * GS_COLS;
  gs_dots<TB, false>(V, ldv, nullptr, t, S.r0, S.nr, xs, P1 + (int64_t)blockIdx.x * ldh, jb, min(t, jb + GS_COLS));
}

// Middle launch: slice -= V h1, then the partial dots P2 of the updated slice.
template <typename TB, bool STAGED>
__global__ __launch_bounds__(GS_T) void k_gs_mid(const TB* __restrict__ V, int64_t ldv, int t, int64_t len,
                                                 int64_t rows, double* __restrict__ x,
                                                 const double* __restrict__ h1, double* __restrict__ P2, int ldh,
                                                 const int* __restrict__ flag) {
  if (flag != nullptr && flag[0] != 0) return;
  extern __shared__ double sm[];
  double* xs = sm;
  double* hs = xs + rows;
  double* cp = hs + GS_HCH + 256;
  TB* Vs = reinterpret_cast<TB*>(hs + GS_HCH + 512);
  const Slice S = slice_of(len, rows);
  for (int i = threadIdx.x; i < S.nr; i += GS_T) xs[i] = x[S.r0 + i];
  if constexpr (STAGED) {
    // the basis slice into LDS, eight loads in flight per thread
    const int64_t tot = (int64_t)t * S.nr;
    for (int64_t e0 = threadIdx.x; e0 < tot; e0 += 8 * GS_T) {
      TB vv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t e = e0 + (int64_t)u * GS_T;
        const int j = (int)(e / S.nr);
        const int i = (int)(e - (int64_t)j * S.nr);
        vv[u] = e < tot ? V[(int64_t)j * ldv + S.r0 + i] : (TB)0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t e = e0 + (int64_t)u * GS_T;
        if (e < tot) Vs[e] = vv[u];
      }
    }
  }
  for (int c0 = 0; c0 < t; c0 += GS_HCH) {
    const int nc = min(GS_HCH, t - c0);
    __syncthreads();
    for (int j = threadIdx.x; j < nc; j += GS_T) hs[j] = h1[c0 + j];
    __syncthreads();
    gs_update<TB, STAGED>(V, ldv, Vs, c0, nc, S.r0, S.nr, xs, hs, cp);
  }
  gs_dots<TB, STAGED>(V, ldv, Vs, t, S.r0, S.nr, xs, P2 + (int64_t)blockIdx.x * ldh);
  for (int i = threadIdx.x; i < S.nr; i += GS_T) x[S.r0 + i] = xs[i];
}

// Last launch: slice -= V h2, npart[b] = sum of the slice's squares (per-thread
// sums in row order, then the fixed block order).
template <typename TB>
__global__ __launch_bounds__(GS_T) void k_gs_last(const TB* __restrict__ V, int64_t ldv, int t, int64_t len,
                                                  int64_t rows, double* __restrict__ x,
                                                  const double* __restrict__ h2, double* __restrict__ npart,
                                                  const int* __restrict__ flag) {
  if (flag != nullptr && flag[0] != 0) return;
  extern __shared__ double sm[];
  double* xs = sm;
  double* hs = xs + rows;
  double* red = hs + GS_HCH;
  double* cp = red + 256;
  const Slice S = slice_of(len, rows);
  for (int i = threadIdx.x; i < S.nr; i += GS_T) xs[i] = x[S.r0 + i];
  for (int c0 = 0; c0 < t; c0 += GS_HCH) {
    const int nc = min(GS_HCH, t - c0);
    __syncthreads();
    for (int j = threadIdx.x; j < nc; j += GS_T) hs[j] = h2[c0 + j];
    __syncthreads();
    gs_update<TB, false>(V, ldv, nullptr, c0, nc, S.r0, S.nr, xs, hs, cp);
  }
  __syncthreads();
  double ss = 0.0;
  for (int i = threadIdx.x; i < S.nr; i += GS_T) {
    const double v = xs[i];
    x[S.r0 + i] = v;
    ss += v * v;
  }
  const double tot = block_sum256(ss, red);
  if (threadIdx.x == 0) npart[blockIdx.x] = tot;
}

// Allow launches of this kernel to use up to GS_LDS_MAX bytes of LDS on the
// current device.
template <typename K>
hipError_t allow_lds(K kernel) {
  return allow_dynamic_lds(reinterpret_cast<const void*>(kernel), (int)GS_LDS_MAX);
}

template <typename TB, typename TP, int PRE>
hipError_t launch_first(const TB* V, int64_t ldv, int t, int64_t len, const GsSplit& s, double* x, double* P1,
                        int ldh, const GsPreArgs& pre, const int* flag, hipStream_t st) {
  auto kern = k_gs_first<TB, TP, PRE>;
  const hipError_t attr = allow_lds(kern);
  if (attr != hipSuccess) return attr;
  const unsigned cb = (unsigned)std::max(1, (t + GS_COLS - 1) / GS_COLS);
  hipLaunchKernelGGL(kern, dim3(s.G, cb), dim3(GS_T), gs_lds_base(s.rows), st, V, ldv, t, len, s.rows, x, P1, ldh,
                     pre.rho, pre.l, reinterpret_cast<const TP*>(pre.part), pre.ldpart, pre.nparts,
                     reinterpret_cast<const TB*>(pre.prev), pre.coef, pre.cidx, pre.run_if, pre.gcol, flag);
  return hipGetLastError();
}

template <typename TB, bool STAGED>
hipError_t launch_mid(const TB* V, int64_t ldv, int t, int64_t len, const GsSplit& s, double* x, const double* h1,
                      double* P2, int ldh, const int* flag, hipStream_t st) {
  auto kern = k_gs_mid<TB, STAGED>;
  const hipError_t attr = allow_lds(kern);
  if (attr != hipSuccess) return attr;
  const size_t lds = gs_lds_base(s.rows) + (STAGED ? (size_t)t * s.rows * sizeof(TB) : 0);
  hipLaunchKernelGGL(kern, dim3(s.G), dim3(GS_T), lds, st, V, ldv, t, len, s.rows, x, h1, P2, ldh, flag);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* P, int ldh, int G, int t, double* h, double* acc, int add, const int* flag,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_gs_reduce, dim3((unsigned)((t + 3) / 4)), dim3(256), 0, st, P, ldh, G, t, h, acc, add, flag);
  return hipGetLastError();
}

}  // namespace

template <typename TB>
hipError_t launch_gs2(const TB* V, int64_t ldv, int t, int64_t len, double* x, double* gsp, int ldh,
                      double* npart, double* acc, int pre_kind, const GsPreArgs& pre, const int* flag,
                      hipStream_t st, int* nparts) {
  if (len < 1 || t < 0 || (t > 0 && ldh < t)) return hipErrorInvalidValue;
  if (pre_kind == GS_PRE_RHO && (pre.l < 1 || pre.l > GS_HCH || pre.rho == nullptr)) return hipErrorInvalidValue;
  if ((pre_kind == GS_PRE_TSUM || pre_kind == GS_PRE_FIX) && (pre.part == nullptr || pre.nparts < 1))
    return hipErrorInvalidValue;
  if (pre_kind == GS_PRE_FIX && (pre.run_if == nullptr || pre.gcol == nullptr)) return hipErrorInvalidValue;
  const GsSplit s = gs_split(len);
  if (gs_lds_base(s.rows) > GS_LDS_MAX) return hipErrorInvalidValue;
  double* P1 = gsp;
  double* P2 = gsp + (int64_t)s.G * ldh;
  double* h = gsp + (gs_partial_rows(len) - 1) * ldh;  // the reduced coefficients of the current pass
  hipError_t e = hipSuccess;
  const bool spread = s.G < GS_SHORT_G || s.rows > GS_SLICE_MAX ||
                      (s.G < GS_WIDE_G && (int64_t)t * s.rows > GS_WIDE_WORK);
  if (t > 0 && spread) {
    // A short vector (few slices), a long one (long slices), or few slices and
    // many columns: a slice's dot products would run one after another in a
    // few waves, so the passes use the kernels that spread the columns over
    // workgroups (dots over row
    // chunks x column blocks, a reduction, an update per 64 rows, the second
    // update leaving the norm partials, one per 64 rows).  P1 holds the
    // dots_chunks(len) chunk partials (gs_partial_rows counts them), h follows.
    if (pre_kind != GS_PRE_NONE) {
      e = pre_kind == GS_PRE_RHO
              ? launch_first<TB, double, GS_PRE_RHO>(V, ldv, 0, len, s, x, P1, ldh, pre, flag, st)
          : pre_kind == GS_PRE_FIX
              ? launch_first<TB, double, GS_PRE_FIX>(V, ldv, 0, len, s, x, P1, ldh, pre, flag, st)
          : pre.part_f64 ? launch_first<TB, double, GS_PRE_TSUM>(V, ldv, 0, len, s, x, P1, ldh, pre, flag, st)
                         : launch_first<TB, float, GS_PRE_TSUM>(V, ldv, 0, len, s, x, P1, ldh, pre, flag, st);
      if (e != hipSuccess) return e;
    }
    for (int pass = 0; pass < 2; ++pass) {
      e = launch_dots<TB>(V, ldv, t, len, x, P1, ldh, h, flag, st, acc, pass);
      if (e != hipSuccess) return e;
      e = launch_update<TB>(V, ldv, t, len, x, h, pass == 1 ? npart : nullptr, flag, st);
      if (e != hipSuccess) return e;
    }
    if (nparts != nullptr) *nparts = update_blocks(len);
    return hipSuccess;
  } else {
    if (pre_kind == GS_PRE_RHO) {
      e = launch_first<TB, double, GS_PRE_RHO>(V, ldv, t, len, s, x, P1, ldh, pre, flag, st);
    } else if (pre_kind == GS_PRE_TSUM) {
      e = pre.part_f64 ? launch_first<TB, double, GS_PRE_TSUM>(V, ldv, t, len, s, x, P1, ldh, pre, flag, st)
                       : launch_first<TB, float, GS_PRE_TSUM>(V, ldv, t, len, s, x, P1, ldh, pre, flag, st);
    } else if (pre_kind == GS_PRE_FIX) {
      e = launch_first<TB, double, GS_PRE_FIX>(V, ldv, t, len, s, x, P1, ldh, pre, flag, st);
    } else if (t > 0) {
      e = launch_first<TB, double, GS_PRE_NONE>(V, ldv, t, len, s, x, P1, ldh, pre, flag, st);
    }
    if (e != hipSuccess) return e;
    if (t > 0) {
      e = launch_reduce(P1, ldh, s.G, t, h, acc, 0, flag, st);
      if (e != hipSuccess) return e;
      const bool staged = (size_t)t * s.rows * sizeof(TB) <= GS_STAGE_BYTES;
      e = staged ? launch_mid<TB, true>(V, ldv, t, len, s, x, h, P2, ldh, flag, st)
                 : launch_mid<TB, false>(V, ldv, t, len, s, x, h, P2, ldh, flag, st);
      if (e != hipSuccess) return e;
      e = launch_reduce(P2, ldh, s.G, t, h, acc, 1, flag, st);
      if (e != hipSuccess) return e;
    }
  }
  auto kern = k_gs_last<TB>;
  const hipError_t attr = allow_lds(kern);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(kern, dim3(s.G), dim3(GS_T), gs_lds_base(s.rows), st, V, ldv, t, len, s.rows, x, h, npart,
                     flag);
  if (nparts != nullptr) *nparts = s.G;
  return hipGetLastError();
}

template hipError_t launch_gs2<double>(const double*, int64_t, int, int64_t, double*, double*, int, double*,
                                       double*, int, const GsPreArgs&, const int*, hipStream_t, int*);
template hipError_t launch_gs2<float>(const float*, int64_t, int, int64_t, double*, double*, int, double*,
                                      double*, int, const GsPreArgs&, const int*, hipStream_t, int*);

}  // namespace gkb
