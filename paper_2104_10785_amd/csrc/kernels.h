// Kernel launchers (internal).  All launches go to the given stream; none
// allocates memory or synchronises.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gemv.h"

namespace gkb {

int dots_chunks(int64_t len);
int update_blocks(int64_t len);

// h[0..t) = V^T x through hpart (dots_chunks(len) x ldh); if acc is given,
// acc[0..t) = h (acc_add = 0) or acc[0..t) += h (acc_add = 1)
template <typename TB>
hipError_t launch_dots(const TB* V, int64_t ldv, int t, int64_t len, const double* x, double* hpart,
                       int ldh, double* h, const int* flag, hipStream_t st, double* acc = nullptr,
                       int acc_add = 0);

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

// Split-K form for long K (K-range slices summed in a fixed order): partial
// must hold gemm_split(M, K, N).slices * M * N elements.
struct GemmSplit {
  int kchunk;
  int slices;
};
GemmSplit gemm_split(int64_t M, int64_t K, int N);
template <typename T>
hipError_t launch_gemm_tall_splitk(const T* A, int64_t lda, int64_t M, int K, const T* B, int64_t ldb, int N,
                                   T* C, int64_t ldc, T* partial, hipStream_t st);

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
