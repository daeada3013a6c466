// Kernel launchers (internal).  All launches go to the given stream; none
// allocates memory or synchronises.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gkb {

struct bf16 {
  uint16_t bits;
};

// A, row-major m x n, leading dimension lda; dtype 0 = double, 1 = float,
// 2 = bfloat16.
struct MatrixRef {
  const void* data;
  int64_t m, n, lda;
  int dtype;
};

// Most row blocks (partial sums) the gemv_t launch uses.
constexpr int GEMV_T_MAX_BLOCKS = 512;

// Compute units of the current device (256 if it cannot be queried).
int device_cus();

struct GemvTShape {
  int64_t rows_per_block;
  int nb;         // row blocks = partial vectors
  int col_tiles;  // blocks along n (vector path)
};
GemvTShape gemv_t_shape(int64_t m, int64_t n, int dtype_bytes);

int dots_chunks(int64_t len);
int update_blocks(int64_t len);

// w = A p - coef[cidx] * qprev   (qprev == nullptr: no recurrence term)
template <typename TB>
hipError_t launch_gemv_n(const MatrixRef& A, const TB* p, const TB* qprev, const double* coef, int cidx,
                         double* w, const int* flag, hipStream_t st);

// z = A^T q - coef[cidx] * pprev, through `part` (nb x ldpart accumulators)
template <typename TB>
hipError_t launch_gemv_t(const MatrixRef& A, const TB* q, const TB* pprev, const double* coef, int cidx,
                         double* z, void* part, int64_t ldpart, const int* flag, hipStream_t st);

// h[0..t) = V^T x through hpart (dots_chunks(len) x ldh)
template <typename TB>
hipError_t launch_dots(const TB* V, int64_t ldv, int t, int64_t len, const double* x, double* hpart,
                       int ldh, double* h, const int* flag, hipStream_t st);

// x -= V h; normpart[b] = partial sums of x^2 (update_blocks(len) entries) if non-null
template <typename TB>
hipError_t launch_update(const TB* V, int64_t ldv, int t, int64_t len, double* x, const double* h,
                         double* normpart, const int* flag, hipStream_t st);

template <typename TB>
hipError_t launch_normalize(const double* x, int64_t len, const double* normpart, int nparts, TB* out,
                            double* coef_out, const double* sig_in, double* sig_out, double eps,
                            int relative, int track, int* flag, int code, int index, hipStream_t st);

hipError_t launch_init_cycle(int* flag, double* sig0, double v, hipStream_t st);

template <typename TB>
hipError_t launch_copy_to_f64(const TB* src, int64_t len, double* dst, hipStream_t st);

template <typename TB>
hipError_t launch_copy_vec(const TB* src, int64_t len, TB* dst, hipStream_t st);

// C = A B; A (M x K, col-major, lda), B (K x N, col-major, ldb), C (M x N, ldc)
template <typename T>
hipError_t launch_gemm_tall(const T* A, int64_t lda, int64_t M, int K, const T* B, int64_t ldb, int N, T* C,
                            int64_t ldc, hipStream_t st);

// C (M x N, col-major) = A (M x K, row-major float32) * B (K x N, col-major float32), MFMA
hipError_t launch_gemm_rm(const float* A, int64_t lda, int64_t M, int64_t K, const float* B, int64_t ldb, int N,
                          float* C, int64_t ldc, hipStream_t st);

// G (d x d, row-major float64) = W^T W for W col-major float32 (m x d), via
// gram_chunks(m) x d*d float64 partials in Gpart
int gram_chunks(int64_t m);
hipError_t launch_gram(const float* W, int64_t ldw, int64_t m, int d, double* Gpart, double* G, hipStream_t st);

hipError_t launch_cast_bf16(const float* src, int64_t lds, int64_t m, int64_t n, uint16_t* dst, int64_t ldd,
                            hipStream_t st);

hipError_t launch_philox_start(double* q, int64_t m, uint64_t seed, hipStream_t st);

}  // namespace gkb
