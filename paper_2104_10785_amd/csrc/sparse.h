// Sparse products (internal): the row schedule of a CSR matrix and the
// product kernels that follow it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/gkb_sparse.h"
#include "sparse_panels.h"

namespace gkb {

constexpr int SP_SHORT = 256;     // rows up to this length go through the stream blocks
constexpr int SP_BLOCK_NNZ = 2048;  // entries of one stream block (at most SP_SHORT rows)
constexpr int SP_HUGE = 4096;     // rows longer than this are split into chunks of this many entries

// One direction: the CSR arrays of A (rows = m) or of A^T (rows = n) and its
// schedule, built on the host from the row offsets when the plan is made:
//  * stream blocks: runs of consecutive short rows holding at most
//    SP_BLOCK_NNZ entries (first row, row count), one workgroup each;
//  * wave rows: rows of SP_SHORT + 1 .. SP_HUGE entries, one wave each;
//  * huge rows: longer rows, cut into chunks of SP_HUGE entries whose partial
//    sums are added in chunk order.
// A direction's column-panel layout on the device (sparse_panels.h).
struct PanelDev {
  int64_t R = 0, C = 0;
  int np = 0;
  const uint16_t* pidx = nullptr;
  const float* pval = nullptr;
  const int32_t* poff = nullptr;   // np x (R + 1)
  const int64_t* pbase = nullptr;  // np + 1
  const PnDesc* jobs = nullptr;
  const PnDesc* sblk = nullptr;
  const PnDesc* witem = nullptr;
  const PnDesc* segs = nullptr;
  const int32_t* lrow = nullptr;   // long rows of the stream blocks
  int64_t njobs = 0, nsegs = 0;
  float* slot = nullptr;           // chunk sums
  float* partial = nullptr;        // np x R row sums per panel (np > 1)
};

struct SparseDir {
  const int64_t* ptr = nullptr;
  const int32_t* idx = nullptr;
  const float* val = nullptr;
  int64_t rows = 0, cols = 0;
  int32_t* sblk = nullptr;     // 2 x nsblk
  int32_t* wrow = nullptr;     // nwrow
  int32_t* hrow = nullptr;     // nhrow
  int32_t* hfirst = nullptr;   // nhrow + 1: first chunk of each huge row
  int32_t* crow = nullptr;     // nchunk: the huge row of each chunk
  int64_t* cbeg = nullptr;     // nchunk: first entry of each chunk
  float* part = nullptr;       // nchunk partial sums
  int64_t nsblk = 0, nwrow = 0, nhrow = 0, nchunk = 0;
  bool panels = false;         // products through the column-panel layout
  PanelDev pn;
};

struct SparseRef {
  int64_t m = 0, n = 0, nnz = 0;
  SparseDir fwd, tr;
};

// upper bound of the device bytes of one direction's schedule
size_t sparse_dir_bytes(int64_t rows, int64_t nnz);
// Place a built panel layout in device memory at w (at most
// panel_bytes_bound bytes, 256-byte aligned) and fill P; synchronises st.
hipError_t place_panels(const PanelLayout& L, char* w, PanelDev& P, hipStream_t st);
// the panel products: what launch_spmv computes, through P
hipError_t launch_panels(const PanelDev& P, const float* x, const float* prev, const double* coef, int cidx,
                         double* y, const int* flag, hipStream_t st);
// y[row] = sum_j val[j] x[idx[j]] - coef[cidx] * prev[row] for every row
// (prev may be null); skipped when flag[0] != 0
hipError_t launch_spmv(const SparseDir& D, const float* x, const float* prev, const double* coef, int cidx,
                       double* y, const int* flag, hipStream_t st);

}  // namespace gkb

struct gkb_sparse_plan_s {
  gkb::SparseRef ref;
};
