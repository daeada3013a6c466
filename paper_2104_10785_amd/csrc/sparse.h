// Sparse products (internal): row bins and the binned CSR product kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/gkb_sparse.h"

namespace gkb {

constexpr int SP_BINS = 4;          // row lengths <= 16, <= 128, <= 1024, longer
constexpr int SP_CHUNK = 1024;      // rows per block of the binning kernels

// One direction: the CSR arrays of A (rows = m) or of A^T (rows = n), and its
// rows listed bin by bin (row order kept inside a bin).
struct SparseDir {
  const int64_t* ptr = nullptr;
  const int32_t* idx = nullptr;
  const float* val = nullptr;
  int64_t rows = 0, cols = 0;
  int32_t* list = nullptr;          // device, rows entries
  int64_t* cnt = nullptr;           // device, chunks x SP_BINS counts, then offsets
  int64_t* tot = nullptr;           // device, SP_BINS totals and the invalid-entry count
  int64_t count[SP_BINS] = {0, 0, 0, 0};   // host copies of the bin sizes
  int64_t base[SP_BINS] = {0, 0, 0, 0};
};

struct SparseRef {
  int64_t m = 0, n = 0, nnz = 0;
  SparseDir fwd, tr;
};

// bytes of one direction's bin arrays
size_t sparse_dir_bytes(int64_t rows);
// place a direction's arrays at ws (sparse_dir_bytes(rows) bytes)
void sparse_dir_place(SparseDir& D, char* ws);
// bin the rows of D on the device and count invalid offsets / indices into
// tot[SP_BINS] (the bin totals go to tot[0 .. SP_BINS))
hipError_t launch_sparse_bins(SparseDir& D, int64_t nnz, hipStream_t st);
// y[row] = sum_j val[j] x[idx[j]] - coef[cidx] * prev[row] for every row
// (prev may be null); skipped when flag[0] != 0
hipError_t launch_spmv(const SparseDir& D, const float* x, const float* prev, const double* coef, int cidx,
                       double* y, const int* flag, hipStream_t st);

}  // namespace gkb

struct gkb_sparse_plan_s {
  gkb::SparseRef ref;
};
