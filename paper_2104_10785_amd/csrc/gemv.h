// The matvec launchers (gemv.hip) and the types they share with the rest of
// the library.  All launches go to the given stream; none allocates memory or
// synchronises.
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

// w = A p - coef[cidx] * qprev   (qprev == nullptr: no recurrence term)
template <typename TB>
hipError_t launch_gemv_n(const MatrixRef& A, const TB* p, const TB* qprev, const double* coef, int cidx,
                         double* w, const int* flag, hipStream_t st);

// z = A^T q - coef[cidx] * pprev, through `part` (nb x ldpart accumulators:
// float for float and bfloat16 A, double for double A; nb =
// gemv_t_shape(m, n, element bytes).nb).  z == NULL: only the partial sums.
template <typename TB>
hipError_t launch_gemv_t(const MatrixRef& A, const TB* q, const TB* pprev, const double* coef, int cidx,
                         double* z, void* part, int64_t ldpart, const int* flag, hipStream_t st);

}  // namespace gkb
