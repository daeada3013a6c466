// HIP kernels for gfx950 (CDNA4): the Golub-Kahan bidiagonalization hot path
// apart from the two products of eq. 2.2 (those are in gemv.hip).
//
//   dots/update   classical Gram-Schmidt projection x <- x - V (V^T x)
//                 (Algorithm 1's reorthogonalisation), float64 coefficients
//   normalize     norm, breakdown test, scaling into the basis
//   gemm_tall     C = A B for a tall column-major A and a small B on MFMA
//                 (Ritz vectors V = P Y, U = Q X, and the restart GEMMs)
//   cast_bf16     float32 -> bfloat16, round to nearest even
//   philox_start  q ~ N(2, 1)^m from Philox4x32-10 + Box-Muller
//
// A is row-major (m x n, lda).  Bases are column-major with each vector
// contiguous.  Every reduction has a fixed order (no float atomics), so two
// runs on the same input are bitwise identical.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "device_common.h"
#include "kernels.h"

namespace gkb {

// ---------------------------------------------------------------- CGS
// hpart[c * ldh + j] = sum_{i in chunk c} V[j * ldv + i] x[i]  for j < t.
// Chunk = 64 * DE rows; each lane keeps its DE entries of x in registers and
// each wave reduces one column at a time.
constexpr int DE = 4;
constexpr int DCOLS = 16;  // columns per block (4 per wave)
template <typename TB>
__global__ __launch_bounds__(256) void k_dots(const TB* __restrict__ V, int64_t ldv, int t, int64_t len,
                                              const double* __restrict__ x, double* __restrict__ hpart,
                                              int ldh, const int* __restrict__ flag) {
  if (flag != nullptr && flag[0] != 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * 64 * DE;
  double xr[DE];
#pragma unroll
  for (int e = 0; e < DE; ++e) {
    const int64_t i = base + e * 64 + lane;
    xr[e] = i < len ? x[i] : 0.0;
  }
  const int j0 = blockIdx.y * DCOLS;
  int j1 = j0 + DCOLS;
  if (j1 > t) j1 = t;
  for (int j = j0 + wave; j < j1; j += 4) {
    const TB* col = V + (int64_t)j * ldv;
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < DE; ++e) {
      const int64_t i = base + e * 64 + lane;
      if (i < len) acc += (double)col[i] * xr[e];
    }
    acc = wave_sum(acc);
    if (lane == 0) hpart[(int64_t)blockIdx.x * ldh + j] = acc;
  }
}

// h[j] = sum_c hpart[c * ldh + j]: one wave per column, lanes stride the
// chunks, then a fixed-order wave reduction.
// h[j] = sum of the chunk partials; acc (if given) gets h (acc_add = 0) or
// adds it (acc_add = 1).
__global__ __launch_bounds__(64) void k_dots_reduce(const double* __restrict__ hpart, int ldh, int nchunks,
                                                    int t, double* __restrict__ h,
                                                    const int* __restrict__ flag, double* __restrict__ acc,
                                                    int acc_add) {
  if (flag != nullptr && flag[0] != 0) return;
  const int j = blockIdx.x;
  if (j >= t) return;
  double s = 0.0;
  for (int c = threadIdx.x; c < nchunks; c += 64) s += hpart[(int64_t)c * ldh + j];
  s = wave_sum(s);
  if (threadIdx.x == 0) {
    h[j] = s;
    if (acc != nullptr) acc[j] = acc_add ? acc[j] + s : s;
  }
}

// x[i] -= sum_{j<t} V[j * ldv + i] h[j] for the block's 64 rows (lane = row).
// The four waves take contiguous quarters of the columns and their partial
// corrections are added in a fixed order through LDS.  If normpart is
// non-null, normpart[block] = sum over the block's rows of the updated x^2.
constexpr int UROWS = 64;
template <typename TB>
__global__ __launch_bounds__(256) void k_update(const TB* __restrict__ V, int64_t ldv, int t, int64_t len,
                                                double* __restrict__ x, const double* __restrict__ h,
                                                double* __restrict__ normpart,
                                                const int* __restrict__ flag) {
  if (flag != nullptr && flag[0] != 0) return;
  __shared__ double part[3][UROWS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * UROWS + lane;
  const bool in = i < len;
  const int per = (t + 3) / 4;
  const int j0 = wave * per;
  int j1 = j0 + per;
  if (j1 > t) j1 = t;
  double c0 = 0.0, c1 = 0.0;
  int j = j0;
  for (; j + 4 <= j1; j += 4) {
    const TB* v0 = V + (int64_t)j * ldv;
    const TB* v1 = v0 + ldv;
    const TB* v2 = v1 + ldv;
    const TB* v3 = v2 + ldv;
    if (in) {
      c0 += (double)v0[i] * h[j];
      c1 += (double)v1[i] * h[j + 1];
      c0 += (double)v2[i] * h[j + 2];
      c1 += (double)v3[i] * h[j + 3];
    }
  }
  for (; j < j1; ++j)
    if (in) c0 += (double)V[(int64_t)j * ldv + i] * h[j];
  const double c = c0 + c1;
  if (wave > 0) part[wave - 1][lane] = c;
  __syncthreads();
  if (wave == 0) {
    double xi = 0.0;
    if (in) {
      xi = x[i] - (((c + part[0][lane]) + part[1][lane]) + part[2][lane]);
      x[i] = xi;
    }
    if (normpart != nullptr) {
      const double ss = wave_sum(xi * xi);
      if (lane == 0) normpart[blockIdx.x] = ss;
    }
  }
}

// nrm = sqrt(sum normpart).  Breakdown if nrm <= thr (thr = eps * sig_in or
// eps), NaN/Inf -> numeric flag.  Otherwise out[i] = x[i] / nrm.  Block 0
// records coef_out = nrm and sig_out = max(sig_in, nrm) (or sig_in when
// !track).  Every block computes nrm identically, so all take the same branch.
template <typename TB>
__global__ __launch_bounds__(256) void k_normalize(const double* __restrict__ x, int64_t len,
                                                   const double* __restrict__ normpart, int nparts,
                                                   TB* __restrict__ out, double* __restrict__ coef_out,
                                                   const double* __restrict__ sig_in,
                                                   double* __restrict__ sig_out, double eps,
                                                   int relative, int track, int* __restrict__ flag,
                                                   int code, int index) {
  if (flag[0] != 0) return;
  __shared__ double red[4];
  const double nrm = norm_test(normpart, nparts, sig_in, sig_out, eps, relative, track, flag, code, index,
                               coef_out, blockIdx.x == 0 && threadIdx.x == 0, red);
  if (nrm < 0.0) return;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256)
    out[i] = (TB)(x[i] / nrm);
}

__global__ void k_init_cycle(int* flag, double* sig0, double v) {
  if (threadIdx.x == 0) {
    flag[0] = 0;
    flag[1] = 0;
    *sig0 = v;
  }
}

template <typename TB>
__global__ __launch_bounds__(256) void k_copy_to_f64(const TB* __restrict__ src, int64_t len,
                                                     double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < len) dst[i] = (double)src[i];
}

template <typename TB>
__global__ __launch_bounds__(256) void k_copy_vec(const TB* __restrict__ src, int64_t len,
                                                  TB* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < len) dst[i] = src[i];
}

// ---------------------------------------------------------------- MFMA GEMM
// C (M x N, column-major, ldc) = A (M x K, column-major, lda) * B (K x N,
// column-major, ldb).  One wave computes a 16 x (16 * NT) tile with the
// 16x16x4 MFMA: lane l supplies A[r0 + l % 16][k0 + l / 16] and
// B[k0 + l / 16][c0 + l % 16].  Accumulator element v of lane l holds
// D[row][l % 16] with row = 4 * (l / 16) + v for the float32 instruction and
// row = 4 * v + l / 16 for the float64 one (lane layouts checked on gfx950).
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> struct V4;
template <> struct V4<double> {
  using type = v4d;
  __device__ __forceinline__ static int row(int lk, int v) { return 4 * v + lk; }
};
template <> struct V4<float> {
  using type = v4f;
  __device__ __forceinline__ static int row(int lk, int v) { return 4 * lk + v; }
};

// Tall-skinny product C = A B with M >> K, N.  A block (4 waves) owns a
// 64 x 64 tile of C; wave w computes rows [16w, 16w + 16) of it as four
// 16 x 16 MFMA tiles.  K advances in chunks of GT_KC: the A chunk (64 rows x
// GT_KC columns; each column slice is 64 contiguous elements, loaded 16 bytes
// per lane) and the B chunk (GT_KC x 64) are staged in LDS; the next chunk's
// loads are issued into registers before the MFMAs of the current one, so a
// block keeps one chunk in flight while it computes.  (Measured on gfx950 at
// 50000 x 120 x 50: this form beats both a 64-wide chunk and direct register
// loads of A.)
constexpr int GT_BM = 64, GT_BN = 64, GT_KC = 32;
template <typename T> struct Vec16;
template <> struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int E = 4;
};
template <> struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int E = 2;
};

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_tall(const T* __restrict__ A, int64_t lda, int64_t M, int K,
                                                   const T* __restrict__ B, int64_t ldb, int N,
                                                   T* __restrict__ C, int64_t ldc, int vec_a, int vec_c,
                                                   int kchunk, int64_t cslice) {
  using VT = typename V4<T>::type;
  using V16 = typename Vec16<T>::type;
  constexpr int E = Vec16<T>::E;
  constexpr int APAD = 64 / (int)sizeof(T);        // row padding of the LDS tiles
  constexpr int GROUPS = GT_BM / E;                 // 16-byte groups per A column slice
  constexpr int NA = GT_KC * GROUPS / 256;          // A vectors per thread per chunk
  constexpr int NB = GT_KC * GT_BN / 256;           // B elements per thread per chunk
  __shared__ __align__(16) T As[GT_KC][GT_BM + APAD];
  __shared__ __align__(16) T Bs[GT_KC][GT_BN + APAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * GT_BM;
  const int c0 = blockIdx.y * GT_BN;
  const int li = lane & 15, lk = lane >> 4;
  // split-K: slice z sums k in [kb, ke) into its own copy of C
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  C += blockIdx.z * cslice;

  V16 ra[NA];
  T rb[NB];
  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int idx = tid + i * 256;
      const int kk = idx / GROUPS, g = idx % GROUPS;
      const int k = k0 + kk;
      const int64_t row = r0 + g * E;
      V16 v;
      if (k < ke && vec_a && row + E <= M) {
        v = *reinterpret_cast<const V16*>(A + (int64_t)k * lda + row);
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = (k < ke && row + e < M) ? A[(int64_t)k * lda + row + e] : (T)0;
      }
      ra[i] = v;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int idx = tid + i * 256;
      const int c = idx / GT_KC, kk = idx % GT_KC;   // consecutive threads walk down a column of B
      const int col = c0 + c, k = k0 + kk;
      rb[i] = (col < N && k < ke) ? B[(int64_t)col * ldb + k] : (T)0;
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int idx = tid + i * 256;
      const int kk = idx / GROUPS, g = idx % GROUPS;
      *reinterpret_cast<V16*>(&As[kk][g * E]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int idx = tid + i * 256;
      Bs[idx % GT_KC][idx / GT_KC] = rb[i];
    }
  };

  VT acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = VT{0, 0, 0, 0};
  load_chunk(kb);
  for (int k0 = kb; k0 < ke; k0 += GT_KC) {
    store_chunk();
    __syncthreads();
    if (k0 + GT_KC < ke) load_chunk(k0 + GT_KC);
#pragma unroll
    for (int ks = 0; ks < GT_KC; ks += 4) {
      const T a = As[ks + lk][wave * 16 + li];
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = mfma16(a, Bs[ks + lk][t * 16 + li], acc[t]);
    }
    __syncthreads();
  }

  const int64_t rw = r0 + wave * 16;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int col = c0 + t * 16 + li;
    if (col >= N) continue;
    T* cc = C + (int64_t)col * ldc;
    if constexpr (sizeof(T) == 4) {
      // float32 layout: lane (li, lk) holds rows 4 lk .. 4 lk + 3 of column li
      const int64_t row = rw + 4 * lk;
      if (vec_c && row + 4 <= M) {
        *reinterpret_cast<v4f*>(cc + row) = acc[t];
        continue;
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = rw + V4<T>::row(lk, v);
      if (row < M) cc[row] = acc[t][v];
    }
  }
}

// C[col * ldc + row] = sum over s of P[s * M * N + col * M + row], in slice order.
template <typename T>
__global__ __launch_bounds__(256) void k_sum_slices(const T* __restrict__ P, int S, int64_t M, int N,
                                                    T* __restrict__ C, int64_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= M * N) return;
  const int64_t col = e / M, row = e % M;
  T acc = 0;
  for (int s2 = 0; s2 < S; ++s2) acc += P[(int64_t)s2 * M * N + e];
  C[col * ldc + row] = acc;
}

// ---------------------------------------------------------------- row-major GEMM
// C (M x N, column-major, ldc) = A (M x K, row-major, lda, float32) *
// B (K x N, column-major, ldb, float32), on the float32 16x16x4 MFMA.
// A block (4 waves) computes a BM x BN tile of C: wave w owns rows
// [w BM/4, (w + 1) BM/4) (BM/64 16-row MFMA tiles) and the block's BN
// columns (BN/16 16-column tiles).  K advances in chunks of 32: the chunk in
// LDS (A: BM rows of 128 contiguous bytes; B: BN columns of 128 contiguous
// bytes; row stride padded to 36 floats) feeds the MFMAs while the next
// chunk's loads are in flight into registers.  Tiles: 64 x 32 for N <= 32
// with the K range split in two (more workgroups for the narrow sketch),
// 128 x 64 for N <= 64, 64 x 112 for N <= 112 (one column tile, so A is read
// once), 64 x 128 above.  Used for the Rayleigh-Ritz block product W = A V and the sketch
// S = A Omega.
constexpr int RM_BK = 32, RM_LD = RM_BK + 4;
// C[col * ldc + row] = 0 for row < M, col < N.
__global__ __launch_bounds__(256) void k_zero_cols(float* __restrict__ C, int64_t ldc, int64_t M, int N) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= M * N) return;
  const int64_t col = e / M, row = e - col * M;
  C[col * ldc + row] = 0.f;
}
template <int BM, int BN, bool SPLIT2>
__global__ __launch_bounds__(256) void k_gemm_rm(const float* __restrict__ A, int64_t lda, int64_t M, int64_t K,
                                                 const float* __restrict__ B, int64_t ldb, int N,
                                                 float* __restrict__ C, int64_t ldc) {
  constexpr int TM = BM / 64;                   // 16-row tiles per wave
  constexpr int TN = BN / 16;                   // 16-column tiles
  constexpr int NA = BM * 8 / 256;              // float4 of an A chunk per thread
  constexpr int NB = (BN * 8 + 255) / 256;      // float4 of a B chunk per thread (the last partly idle)
  static_assert(BM % 64 == 0 && BN % 16 == 0 && (BM * 8) % 256 == 0, "tile shape");
  __shared__ float As[BM * RM_LD];
  __shared__ float Bs[BN * RM_LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.x * BM;
  const int n0 = blockIdx.y * BN;
  const int li = lane & 15, lk = lane >> 4;
  // SPLIT2: workgroup z of 2 takes K range [kb, ke) (the halves split at a
  // multiple of the chunk width) and adds its product into C, which the launch
  // has zeroed; two addends on zero give the same sum in either order
  const int64_t khalf = K / (2 * RM_BK) * RM_BK;
  const int64_t kb = SPLIT2 && blockIdx.z == 1 ? khalf : 0;
  const int64_t ke = SPLIT2 && blockIdx.z == 0 ? khalf : K;
  v4f acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = v4f{0, 0, 0, 0};
  const bool avec = ((lda & 3) == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  const bool bvec = ((ldb & 3) == 0) && ((reinterpret_cast<uintptr_t>(B) & 15) == 0);
  float4 ra[NA], rb[NB];
  // rows past M and columns past N (and the idle part of the last B slot)
  // are zeros; the same for every chunk
  bool oka[NA], okb[NB];
#pragma unroll
  for (int it = 0; it < NA; ++it) oka[it] = m0 + ((tid + it * 256) >> 3) < M;
#pragma unroll
  for (int it = 0; it < NB; ++it) {
    const int idx = tid + it * 256;
    okb[it] = idx < BN * 8 && n0 + (idx >> 3) < N;
  }
  // Full 32-wide chunk k0 of aligned operands into registers with no branch
  // and no use of the values: rows past M and columns past N load row M - 1
  // / column N - 1 (zeroed when stored to LDS), so the loads stay in flight
  // through the MFMAs of the current chunk.
  auto fetch_full = [&](int64_t k0) {
#pragma unroll
    for (int it = 0; it < NA; ++it) {
      const int idx = tid + it * 256;
      const uint4 u = ld_stream(A + std::min(m0 + (idx >> 3), M - 1) * lda + k0 + (idx & 7) * 4);
      ra[it] = make_float4(__uint_as_float(u.x), __uint_as_float(u.y), __uint_as_float(u.z), __uint_as_float(u.w));
    }
#pragma unroll
    for (int it = 0; it < NB; ++it) {
      const int idx = std::min(tid + it * 256, BN * 8 - 1);
      const int gc = std::min(n0 + (idx >> 3), N - 1);
      rb[it] = *reinterpret_cast<const float4*>(B + (int64_t)gc * ldb + k0 + (idx & 7) * 4);
    }
  };
  // Any chunk, element by element (zeros past M, N or K): the last partial
  // chunk, or every chunk of unaligned operands.
  auto fetch_any = [&](int64_t k0) {
#pragma unroll
    for (int it = 0; it < NA; ++it) {
      const int idx = tid + it * 256;
      const int64_t gr = m0 + (idx >> 3), gk = k0 + (idx & 7) * 4;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gr < M) {
        const float* src = A + gr * lda + gk;
        if (gk < ke) v.x = src[0];
        if (gk + 1 < ke) v.y = src[1];
        if (gk + 2 < ke) v.z = src[2];
        if (gk + 3 < ke) v.w = src[3];
      }
      ra[it] = v;
    }
#pragma unroll
    for (int it = 0; it < NB; ++it) {
      const int idx = tid + it * 256;
      const int gc = n0 + (idx >> 3);
      const int64_t gk = k0 + (idx & 7) * 4;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (idx < BN * 8 && gc < N) {
        const float* src = B + (int64_t)gc * ldb + gk;
        if (gk < ke) v.x = src[0];
        if (gk + 1 < ke) v.y = src[1];
        if (gk + 2 < ke) v.z = src[2];
        if (gk + 3 < ke) v.w = src[3];
      }
      rb[it] = v;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int it = 0; it < NA; ++it) {
      const int idx = tid + it * 256;
      float* dst = As + (idx >> 3) * RM_LD + (idx & 7) * 4;
      dst[0] = oka[it] ? ra[it].x : 0.f;
      dst[1] = oka[it] ? ra[it].y : 0.f;
      dst[2] = oka[it] ? ra[it].z : 0.f;
      dst[3] = oka[it] ? ra[it].w : 0.f;
    }
#pragma unroll
    for (int it = 0; it < NB; ++it) {
      const int idx = tid + it * 256;
      if (idx < BN * 8) {
        float* dst = Bs + (idx >> 3) * RM_LD + (idx & 7) * 4;
        dst[0] = okb[it] ? rb[it].x : 0.f;
        dst[1] = okb[it] ? rb[it].y : 0.f;
        dst[2] = okb[it] ? rb[it].z : 0.f;
        dst[3] = okb[it] ? rb[it].w : 0.f;
      }
    }
  };
  auto mfma_chunk = [&]() {
#pragma unroll
    for (int kk = 0; kk < RM_BK; kk += 4) {
      float av[TM];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = As[(wave * (BM / 4) + a * 16 + li) * RM_LD + kk + lk];
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const float bv = Bs[(b * 16 + li) * RM_LD + kk + lk];
#pragma unroll
        for (int a = 0; a < TM; ++a) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv, acc[a][b], 0, 0, 0);
      }
    }
  };
  // full chunks: the next one (the last one again at the end: one spare
  // chunk load per block) loads while the current one feeds the MFMAs
  const int64_t kfull = (avec && bvec) ? kb + (ke - kb) / RM_BK * RM_BK : kb;
  if (kfull > kb) fetch_full(kb);
  for (int64_t k0 = kb; k0 < kfull; k0 += RM_BK) {
    stash();
    __syncthreads();
    fetch_full(std::min(k0 + RM_BK, kfull - RM_BK));
    __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the MFMAs
    mfma_chunk();
    __syncthreads();
  }
  for (int64_t k0 = kfull; k0 < ke; k0 += RM_BK) {
    fetch_any(k0);
    stash();
    __syncthreads();
    mfma_chunk();
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int col = n0 + b * 16 + li;
      if (col < N) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = m0 + wave * (BM / 4) + a * 16 + 4 * lk + v;
          if (row < M) {
            if constexpr (SPLIT2) atomicAdd(C + (int64_t)col * ldc + row, acc[a][b][v]);
            else C[(int64_t)col * ldc + row] = acc[a][b][v];
          }
        }
      }
    }
}

// ---------------------------------------------------------------- Gram matrix
// Gpart[c * ldg + a * d + b] = sum_{i in chunk c} W[i][a] W[i][b] for a 16 x 16
// tile (a0.., b0..) per block, W column-major float32 (m x d, ldw), products
// and sums in float64 on the 16x16x4 MFMA.  Chunk = GRAM_ROWS rows.
constexpr int GRAM_ROWS = 2048;
constexpr int GRAM_U = 8;
__global__ __launch_bounds__(64) void k_gram(const float* __restrict__ W, int64_t ldw, int64_t m, int d,
                                             double* __restrict__ Gpart, int64_t ldg) {
  const int lane = threadIdx.x;
  const int c = blockIdx.x;
  const int a0 = blockIdx.y * 16, b0 = blockIdx.z * 16;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t r0 = (int64_t)c * GRAM_ROWS;
  int64_t r1 = r0 + GRAM_ROWS;
  if (r1 > m) r1 = m;
  v4d acc = {0, 0, 0, 0};
  const int ca = a0 + li, cb = b0 + li;
  // GRAM_U groups of 4 rows loaded before their MFMAs (one memory round trip
  // per GRAM_U groups); one accumulator, so the products are added in row
  // order; rows past r1 contribute exact zeros
  for (int64_t i0 = r0; i0 < r1; i0 += 4 * GRAM_U) {
    double av[GRAM_U], bv[GRAM_U];
#pragma unroll
    for (int u = 0; u < GRAM_U; ++u) {
      const int64_t i = i0 + 4 * u + lk;
      av[u] = (i < r1 && ca < d) ? (double)W[(int64_t)ca * ldw + i] : 0.0;
      bv[u] = (i < r1 && cb < d) ? (double)W[(int64_t)cb * ldw + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < GRAM_U; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
  }
  // float64 layout: element v of lane l is row 4v + l/16, column l % 16
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int ra = a0 + 4 * v + lk;
    if (ra < d && cb < d) Gpart[(int64_t)c * ldg + (int64_t)ra * d + cb] = acc[v];
  }
}

// ---------------------------------------------------------------- bf16 cast
// Round to nearest even; NaN stays NaN (quiet bit forced).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x0040u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__global__ __launch_bounds__(256) void k_cast_bf16(const float* __restrict__ src, int64_t lds, int64_t m,
                                                   int64_t n, uint16_t* __restrict__ dst, int64_t ldd) {
  const int64_t row = blockIdx.y;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256)
    dst[row * ldd + j] = f32_to_bf16_rne(src[row * lds + j]);
}

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC 2011): counter (i, 0, 0, 0), key = seed.  Uniforms
// u = (x + 1) * 2^-32 in (0, 1]; Box-Muller on (u0, u1):
// g = sqrt(-2 ln u0) cos(2 pi u1); q_i = 2 + g.
__device__ __forceinline__ void philox_round(uint32_t* c, const uint32_t* k) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
  uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
  uint32_t n0 = hi1 ^ c[1] ^ k[0];
  uint32_t n1 = lo1;
  uint32_t n2 = hi0 ^ c[3] ^ k[1];
  uint32_t n3 = lo0;
  c[0] = n0;
  c[1] = n1;
  c[2] = n2;
  c[3] = n3;
}

__global__ __launch_bounds__(256) void k_philox_start(double* __restrict__ q, int64_t m, uint64_t seed,
                                                      double mean, double stdv) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  uint32_t c[4] = {(uint32_t)(i & 0xffffffffu), (uint32_t)((uint64_t)i >> 32), 0u, 0u};
  uint32_t k[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    philox_round(c, k);
    if (r < 9) {
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
  }
  const double two32 = 4294967296.0;
  const double u0 = ((double)c[0] + 1.0) / two32;
  const double u1 = ((double)c[1] + 1.0) / two32;
  const double g = sqrt(-2.0 * log(u0)) * cos(6.283185307179586 * u1);
  q[i] = mean + stdv * g;
}

// ================================================================ launchers
int dots_chunks(int64_t len) { return (int)nblocks(len, 64 * DE); }
int update_blocks(int64_t len) { return (int)nblocks(len, UROWS); }

template <typename TB>
hipError_t launch_dots(const TB* V, int64_t ldv, int t, int64_t len, const double* x, double* hpart,
                       int ldh, double* h, const int* flag, hipStream_t st, double* acc, int acc_add) {
  if (t <= 0) return hipSuccess;
  const int nch = dots_chunks(len);
  dim3 grid(nch, nblocks(t, DCOLS));
  hipLaunchKernelGGL((k_dots<TB>), grid, dim3(256), 0, st, V, ldv, t, len, x, hpart, ldh, flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dots_reduce, dim3(t), dim3(64), 0, st, hpart, ldh, nch, t, h, flag, acc, acc_add);
  return hipGetLastError();
}

template <typename TB>
hipError_t launch_update(const TB* V, int64_t ldv, int t, int64_t len, double* x, const double* h,
                         double* normpart, const int* flag, hipStream_t st) {
  hipLaunchKernelGGL((k_update<TB>), dim3(update_blocks(len)), dim3(256), 0, st, V, ldv, t, len, x, h,
                     normpart, flag);
  return hipGetLastError();
}

template <typename TB>
hipError_t launch_normalize(const double* x, int64_t len, const double* normpart, int nparts, TB* out,
                            double* coef_out, const double* sig_in, double* sig_out, double eps,
                            int relative, int track, int* flag, int code, int index, hipStream_t st) {
  int64_t blocks = nblocks(len, 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL((k_normalize<TB>), dim3((unsigned)blocks), dim3(256), 0, st, x, len, normpart, nparts,
                     out, coef_out, sig_in, sig_out, eps, relative, track, flag, code, index);
  return hipGetLastError();
}

hipError_t launch_init_cycle(int* flag, double* sig0, double v, hipStream_t st) {
  hipLaunchKernelGGL(k_init_cycle, dim3(1), dim3(64), 0, st, flag, sig0, v);
  return hipGetLastError();
}

template <typename TB>
hipError_t launch_copy_to_f64(const TB* src, int64_t len, double* dst, hipStream_t st) {
  hipLaunchKernelGGL((k_copy_to_f64<TB>), dim3(nblocks(len, 256)), dim3(256), 0, st, src, len, dst);
  return hipGetLastError();
}

template <typename TB>
hipError_t launch_copy_vec(const TB* src, int64_t len, TB* dst, hipStream_t st) {
  hipLaunchKernelGGL((k_copy_vec<TB>), dim3(nblocks(len, 256)), dim3(256), 0, st, src, len, dst);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gemm_tall(const T* A, int64_t lda, int64_t M, int K, const T* B, int64_t ldb, int N, T* C,
                            int64_t ldc, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid(nblocks(M, GT_BM), nblocks(N, GT_BN));
  // 16-byte accesses need 16-byte aligned column starts
  const int vec_a = (lda % (16 / (int64_t)sizeof(T)) == 0) && (reinterpret_cast<uintptr_t>(A) % 16 == 0);
  const int vec_c = (ldc % (16 / (int64_t)sizeof(T)) == 0) && (reinterpret_cast<uintptr_t>(C) % 16 == 0);
  hipLaunchKernelGGL((k_gemm_tall<T>), grid, dim3(256), 0, st, A, lda, M, K, B, ldb, N, C, ldc, vec_a, vec_c,
                     K, (int64_t)0);
  return hipGetLastError();
}

GemmSplit gemm_split(int64_t M, int64_t K, int N) {
  GemmSplit g;
  const int64_t tiles = nblocks(M, GT_BM) * nblocks(N, GT_BN);
  int64_t want = (2 * (int64_t)device_cus()) / std::max<int64_t>(tiles, 1);
  want = std::max<int64_t>(1, std::min<int64_t>({want, nblocks(K, GT_KC), 1024}));
  const int64_t chunk = nblocks(nblocks(K, want), GT_KC) * GT_KC;
  g.kchunk = (int)std::max<int64_t>(chunk, GT_KC);
  g.slices = (int)std::max<int64_t>(1, nblocks(K, g.kchunk));
  return g;
}

template <typename T>
hipError_t launch_gemm_tall_splitk(const T* A, int64_t lda, int64_t M, int K, const T* B, int64_t ldb, int N,
                                   T* C, int64_t ldc, T* partial, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const GemmSplit g = gemm_split(M, K, N);
  if (g.slices == 1) return launch_gemm_tall<T>(A, lda, M, K, B, ldb, N, C, ldc, st);
  dim3 grid(nblocks(M, GT_BM), nblocks(N, GT_BN), g.slices);
  const int vec_a = (lda % (16 / (int64_t)sizeof(T)) == 0) && (reinterpret_cast<uintptr_t>(A) % 16 == 0);
  const int vec_c = (M % (16 / (int64_t)sizeof(T)) == 0) && (reinterpret_cast<uintptr_t>(partial) % 16 == 0);
  hipLaunchKernelGGL((k_gemm_tall<T>), grid, dim3(256), 0, st, A, lda, M, K, B, ldb, N, partial, M, vec_a, vec_c,
                     g.kchunk, M * (int64_t)N);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_sum_slices<T>), dim3(nblocks(M * (int64_t)N, 256)), dim3(256), 0, st, partial, g.slices, M, N,
                     C, ldc);
  return hipGetLastError();
}
template hipError_t launch_gemm_tall_splitk<float>(const float*, int64_t, int64_t, int, const float*, int64_t, int,
                                                   float*, int64_t, float*, hipStream_t);

hipError_t launch_cast_bf16(const float* src, int64_t lds, int64_t m, int64_t n, uint16_t* dst, int64_t ldd,
                            hipStream_t st) {
  int64_t gx = nblocks(n, 256);
  if (gx > 64) gx = 64;
  // one grid row per matrix row; gridDim.y limit is 65535, so split if needed
  for (int64_t r0 = 0; r0 < m; r0 += 65535) {
    int64_t rows = m - r0 < 65535 ? m - r0 : 65535;
    hipLaunchKernelGGL(k_cast_bf16, dim3((unsigned)gx, (unsigned)rows), dim3(256), 0, st, src + r0 * lds,
                       lds, rows, n, dst + r0 * ldd, ldd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_gemm_rm(const float* A, int64_t lda, int64_t M, int64_t K, const float* B, int64_t ldb, int N,
                          float* C, int64_t ldc, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (N <= 32) {
    hipLaunchKernelGGL(k_zero_cols, dim3(nblocks(M * N, 256)), dim3(256), 0, st, C, ldc, M, N);
    hipLaunchKernelGGL((k_gemm_rm<64, 32, true>), dim3(nblocks(M, 64), 1, 2), dim3(256), 0, st, A, lda, M, K, B, ldb, N,
                       C, ldc);
  } else if (N <= 64) {
    hipLaunchKernelGGL((k_gemm_rm<128, 64, false>), dim3(nblocks(M, 128), 1), dim3(256), 0, st, A, lda, M, K, B, ldb, N, C,
                       ldc);
  } else if (N <= 112) {
    hipLaunchKernelGGL((k_gemm_rm<64, 112, false>), dim3(nblocks(M, 64), 1), dim3(256), 0, st, A, lda, M, K, B, ldb, N, C,
                       ldc);
  } else {
    hipLaunchKernelGGL((k_gemm_rm<64, 128, false>), dim3(nblocks(M, 64), nblocks(N, 128)), dim3(256), 0, st, A, lda, M, K, B,
                       ldb, N, C, ldc);
  }
  return hipGetLastError();
}

int gram_chunks(int64_t m) { return (int)nblocks(m, GRAM_ROWS); }

hipError_t launch_gram(const float* W, int64_t ldw, int64_t m, int d, double* Gpart, double* G, hipStream_t st) {
  const int nch = gram_chunks(m);
  const int64_t ldg = (int64_t)d * d;
  dim3 grid(nch, nblocks(d, 16), nblocks(d, 16));
  hipLaunchKernelGGL(k_gram, grid, dim3(64), 0, st, W, ldw, m, d, Gpart, ldg);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dots_reduce, dim3((unsigned)ldg), dim3(64), 0, st, Gpart, (int)ldg, nch, (int)ldg, G,
                     (const int*)nullptr, (double*)nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_philox_start(double* q, int64_t m, uint64_t seed, hipStream_t st) {
  hipLaunchKernelGGL(k_philox_start, dim3(nblocks(m, 256)), dim3(256), 0, st, q, m, seed, 2.0, 1.0);
  return hipGetLastError();
}

// explicit instantiations for the two basis types
#define GKB_INST(TB)                                                                                      \
  template hipError_t launch_dots<TB>(const TB*, int64_t, int, int64_t, const double*, double*, int,      \
                                      double*, const int*, hipStream_t, double*, int);                    \
  template hipError_t launch_update<TB>(const TB*, int64_t, int, int64_t, double*, const double*,         \
                                        double*, const int*, hipStream_t);                                \
  template hipError_t launch_normalize<TB>(const double*, int64_t, const double*, int, TB*, double*,      \
                                           const double*, double*, double, int, int, int*, int, int,      \
                                           hipStream_t);                                                  \
  template hipError_t launch_copy_to_f64<TB>(const TB*, int64_t, double*, hipStream_t);                   \
  template hipError_t launch_copy_vec<TB>(const TB*, int64_t, TB*, hipStream_t);                          \
  template hipError_t launch_gemm_tall<TB>(const TB*, int64_t, int64_t, int, const TB*, int64_t, int, TB*, \
                                           int64_t, hipStream_t);
GKB_INST(double)
GKB_INST(float)
#undef GKB_INST

}  // namespace gkb
