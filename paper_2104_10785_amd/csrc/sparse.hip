// Products with a sparse A (CSR of A for A p, CSR of A^T for A^T q) and the
// row binning they use.  The bidiagonalization only touches A through these
// two products (eq. (2.1)-(2.2)); the rest of the solver is shared with the
// dense path.
//
// A row of length L is summed by G lanes (G = 4, 16, 64 by bin, or a
// 256-thread workgroup for the longest rows): lane l takes entries
// l, l + G, ..., the G partial sums meet in a fixed butterfly, so the result
// of a row does not depend on the launch.  Rows are listed bin by bin in row
// order, so neighbouring lanes read neighbouring rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>

#include "sparse.h"

namespace gkb {

namespace {

constexpr int SP_T = 256;                    // threads per block
constexpr int SP_RPT = SP_CHUNK / SP_T;      // rows per thread in the binning kernels (4)

__device__ __forceinline__ int row_bin(int64_t len) {
  return len <= 16 ? 0 : (len <= 128 ? 1 : (len <= 1024 ? 2 : 3));
}

constexpr int SP_COLS = SP_BINS + 1;          // per-chunk counts: the bins, then invalid rows

// cnt[c * SP_COLS + b] = rows of chunk c in bin b; cnt[c * SP_COLS + SP_BINS] =
// rows whose offsets are outside [0, nnz] or decreasing
__global__ __launch_bounds__(SP_T) void k_bin_count(const int64_t* __restrict__ ptr, int64_t rows, int64_t nnz,
                                                     int64_t* __restrict__ cnt) {
  __shared__ int c[SP_COLS];
  if (threadIdx.x < SP_COLS) c[threadIdx.x] = 0;
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * SP_CHUNK + threadIdx.x * SP_RPT;
  int mine[SP_COLS] = {0, 0, 0, 0, 0};
  for (int u = 0; u < SP_RPT; ++u) {
    const int64_t r = r0 + u;
    if (r < rows) {
      const int64_t b = ptr[r], e = ptr[r + 1];
      ++mine[row_bin(e - b)];
      if (b < 0 || e < b || e > nnz) ++mine[SP_BINS];
    }
  }
  for (int b = 0; b < SP_COLS; ++b)
    if (mine[b]) atomicAdd(&c[b], mine[b]);   // integer counts: order does not matter
  __syncthreads();
  if (threadIdx.x < SP_COLS) cnt[(int64_t)blockIdx.x * SP_COLS + threadIdx.x] = c[threadIdx.x];
}

// tot[SP_BINS] += indices outside [0, cols)
__global__ __launch_bounds__(SP_T) void k_check_idx(const int32_t* __restrict__ idx, int64_t nnz, int64_t cols,
                                                     int64_t* __restrict__ tot) {
  int64_t bad = 0;
  for (int64_t j = (int64_t)blockIdx.x * SP_T + threadIdx.x; j < nnz; j += (int64_t)gridDim.x * SP_T)
    bad += (idx[j] < 0 || idx[j] >= cols) ? 1 : 0;
  for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off, 64);
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd((unsigned long long*)&tot[SP_BINS], (unsigned long long)bad);
}

// In place: cnt[c * SP_COLS + b] <- rows of bin b in chunks before c; tot[b] = rows of
// bin b (b = SP_BINS: invalid rows).
__global__ void k_bin_scan(int64_t* __restrict__ cnt, int64_t nchunks, int64_t* __restrict__ tot) {
  const int b = threadIdx.x;
  if (b >= SP_COLS) return;
  int64_t s = 0;
  for (int64_t c = 0; c < nchunks; ++c) {
    const int64_t v = cnt[c * SP_COLS + b];
    cnt[c * SP_COLS + b] = s;
    s += v;
  }
  tot[b] = s;
}

// list[base_b + offset of chunk c in bin b + rank in the chunk] = row, rows in order.
__global__ __launch_bounds__(SP_T) void k_bin_scatter(const int64_t* __restrict__ ptr, int64_t rows,
                                                       const int64_t* __restrict__ cnt,
                                                       const int64_t* __restrict__ tot,
                                                       int32_t* __restrict__ list) {
  __shared__ uint64_t wsum[SP_T / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * SP_CHUNK + threadIdx.x * SP_RPT;
  int bins[SP_RPT];
  uint64_t packed = 0;   // 16-bit count per bin (at most SP_CHUNK rows per chunk)
  for (int u = 0; u < SP_RPT; ++u) {
    const int64_t r = r0 + u;
    bins[u] = r < rows ? row_bin(ptr[r + 1] - ptr[r]) : -1;
    if (bins[u] >= 0) packed += (uint64_t)1 << (16 * bins[u]);
  }
  // exclusive scan of the packed counts over the block, in thread (= row) order
  uint64_t incl = packed;
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint64_t before = incl - packed;
  for (int w = 0; w < wave; ++w) before += wsum[w];
  int64_t base[SP_BINS];
  int64_t acc = 0;
  for (int b = 0; b < SP_BINS; ++b) {
    base[b] = acc + cnt[(int64_t)blockIdx.x * SP_COLS + b] + (int64_t)((before >> (16 * b)) & 0xffff);
    acc += tot[b];
  }
  for (int u = 0; u < SP_RPT; ++u)
    if (bins[u] >= 0) list[base[bins[u]]++] = (int32_t)(r0 + u);
}

// Rows of one bin with G lanes per row (G <= 64).
template <int G>
__global__ __launch_bounds__(SP_T) void k_spmv_group(const int64_t* __restrict__ ptr,
                                                      const int32_t* __restrict__ idx,
                                                      const float* __restrict__ val,
                                                      const int32_t* __restrict__ list, int64_t count,
                                                      const float* __restrict__ x, const float* __restrict__ prev,
                                                      const double* __restrict__ coef, int cidx,
                                                      double* __restrict__ y, const int* __restrict__ flag) {
  if (flag != nullptr && flag[0] != 0) return;
  const int64_t g = ((int64_t)blockIdx.x * SP_T + threadIdx.x) / G;
  const int l = threadIdx.x % G;
  if (g >= count) return;   // uniform over the G lanes of a row
  const int32_t row = list[g];
  const int64_t b = ptr[row], e = ptr[row + 1];
  float s = 0.f;
  for (int64_t j = b + l; j < e; j += G) s += val[j] * x[idx[j]];
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, G);
  if (l == 0) y[row] = (double)s - (prev ? coef[cidx] * (double)prev[row] : 0.0);
}

// The longest rows: one workgroup per row.
__global__ __launch_bounds__(SP_T) void k_spmv_block(const int64_t* __restrict__ ptr,
                                                      const int32_t* __restrict__ idx,
                                                      const float* __restrict__ val,
                                                      const int32_t* __restrict__ list,
                                                      const float* __restrict__ x, const float* __restrict__ prev,
                                                      const double* __restrict__ coef, int cidx,
                                                      double* __restrict__ y, const int* __restrict__ flag) {
  if (flag != nullptr && flag[0] != 0) return;
  __shared__ float red[SP_T / 64];
  const int32_t row = list[blockIdx.x];
  const int64_t b = ptr[row], e = ptr[row + 1];
  float s = 0.f;
  for (int64_t j = b + threadIdx.x; j < e; j += SP_T) s += val[j] * x[idx[j]];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
#pragma unroll
    for (int w = 0; w < SP_T / 64; ++w) t += red[w];
    y[row] = (double)t - (prev ? coef[cidx] * (double)prev[row] : 0.0);
  }
}

inline unsigned nblk(int64_t work, int64_t per) { return (unsigned)((work + per - 1) / per); }
inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

size_t sparse_dir_bytes(int64_t rows) {
  const int64_t chunks = (rows + SP_CHUNK - 1) / SP_CHUNK;
  return a256((size_t)rows * 4) + a256((size_t)chunks * SP_COLS * 8) + a256(SP_COLS * 8);
}

void sparse_dir_place(SparseDir& D, char* ws) {
  const int64_t chunks = (D.rows + SP_CHUNK - 1) / SP_CHUNK;
  D.list = reinterpret_cast<int32_t*>(ws);
  ws += a256((size_t)D.rows * 4);
  D.cnt = reinterpret_cast<int64_t*>(ws);
  ws += a256((size_t)chunks * SP_COLS * 8);
  D.tot = reinterpret_cast<int64_t*>(ws);
}

hipError_t launch_sparse_bins(SparseDir& D, int64_t nnz, hipStream_t st) {
  const int64_t chunks = (D.rows + SP_CHUNK - 1) / SP_CHUNK;
  hipLaunchKernelGGL(k_bin_count, dim3((unsigned)chunks), dim3(SP_T), 0, st, D.ptr, D.rows, nnz, D.cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(64), 0, st, D.cnt, chunks, D.tot);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nnz > 0) {
    hipLaunchKernelGGL(k_check_idx, dim3((unsigned)std::min<int64_t>(nblk(nnz, SP_T), 4096)), dim3(SP_T), 0, st,
                       D.idx, nnz, D.cols, D.tot);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_bin_scatter, dim3((unsigned)chunks), dim3(SP_T), 0, st, D.ptr, D.rows, D.cnt, D.tot,
                     D.list);
  return hipGetLastError();
}

hipError_t launch_spmv(const SparseDir& D, const float* x, const float* prev, const double* coef, int cidx,
                       double* y, const int* flag, hipStream_t st) {
  const int32_t* l0 = D.list + D.base[0];
  const int32_t* l1 = D.list + D.base[1];
  const int32_t* l2 = D.list + D.base[2];
  const int32_t* l3 = D.list + D.base[3];
  if (D.count[0] > 0)
    hipLaunchKernelGGL(k_spmv_group<4>, dim3(nblk(D.count[0], SP_T / 4)), dim3(SP_T), 0, st, D.ptr, D.idx, D.val,
                       l0, D.count[0], x, prev, coef, cidx, y, flag);
  if (D.count[1] > 0)
    hipLaunchKernelGGL(k_spmv_group<16>, dim3(nblk(D.count[1], SP_T / 16)), dim3(SP_T), 0, st, D.ptr, D.idx,
                       D.val, l1, D.count[1], x, prev, coef, cidx, y, flag);
  if (D.count[2] > 0)
    hipLaunchKernelGGL(k_spmv_group<64>, dim3(nblk(D.count[2], SP_T / 64)), dim3(SP_T), 0, st, D.ptr, D.idx,
                       D.val, l2, D.count[2], x, prev, coef, cidx, y, flag);
  if (D.count[3] > 0)
    hipLaunchKernelGGL(k_spmv_block, dim3((unsigned)D.count[3]), dim3(SP_T), 0, st, D.ptr, D.idx, D.val, l3, x,
                       prev, coef, cidx, y, flag);
  return hipGetLastError();
}

}  // namespace gkb

namespace {
thread_local std::string s_err;
gkb_status sfail(gkb_status s, const std::string& m) {
  s_err = m;
  return s;
}
}  // namespace

extern "C" {

const char* gkb_sparse_last_error(void) { return s_err.c_str(); }

static gkb_status check_csr(const gkb_csr* A) {
  if (!A) return sfail(GKB_ERR_INVALID, "A is NULL");
  if (A->m < 1 || A->n < 1 || A->nnz < 0) return sfail(GKB_ERR_INVALID, "need m, n >= 1 and nnz >= 0");
  if (A->m >= ((int64_t)1 << 31) || A->n >= ((int64_t)1 << 31))
    return sfail(GKB_ERR_INVALID, "m and n must be below 2^31");
  if (!A->row_ptr || !A->col_ptr) return sfail(GKB_ERR_INVALID, "row_ptr and col_ptr must be non-NULL");
  if (A->nnz > 0 && (!A->col_idx || !A->val || !A->row_idx || !A->val_t))
    return sfail(GKB_ERR_INVALID, "index and value arrays must be non-NULL");
  return GKB_OK;
}

size_t gkb_sparse_plan_workspace_size(const gkb_csr* A) {
  if (check_csr(A) != GKB_OK) return 0;
  return gkb::sparse_dir_bytes(A->m) + gkb::sparse_dir_bytes(A->n);
}

gkb_status gkb_sparse_plan_create(const gkb_csr* A, void* ws, size_t ws_bytes, void* stream,
                                  gkb_sparse_plan* out) {
  s_err.clear();
  if (!out) return sfail(GKB_ERR_INVALID, "plan pointer is NULL");
  *out = nullptr;
  gkb_status rc = check_csr(A);
  if (rc != GKB_OK) return rc;
  const size_t need = gkb_sparse_plan_workspace_size(A);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) || ws_bytes < need)
    return sfail(GKB_ERR_WORKSPACE, "plan workspace missing, misaligned or too small (need " + std::to_string(need) +
                                        " bytes)");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // the offsets must end at nnz (a cheap check of the two pointer arrays)
  int64_t ends[2] = {-1, -1};
  if (hipMemcpyAsync(&ends[0], A->row_ptr + A->m, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(&ends[1], A->col_ptr + A->n, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return sfail(GKB_ERR_HIP, "reading the row offsets failed");
  if (ends[0] != A->nnz || ends[1] != A->nnz)
    return sfail(GKB_ERR_INVALID, "row_ptr[m] and col_ptr[n] must equal nnz");
  auto* plan = new gkb_sparse_plan_s();
  gkb::SparseRef& R = plan->ref;
  R.m = A->m;
  R.n = A->n;
  R.nnz = A->nnz;
  R.fwd.ptr = A->row_ptr;
  R.fwd.idx = A->col_idx;
  R.fwd.val = A->val;
  R.fwd.rows = A->m;
  R.fwd.cols = A->n;
  R.tr.ptr = A->col_ptr;
  R.tr.idx = A->row_idx;
  R.tr.val = A->val_t;
  R.tr.rows = A->n;
  R.tr.cols = A->m;
  char* w = reinterpret_cast<char*>(ws);
  gkb::sparse_dir_place(R.fwd, w);
  gkb::sparse_dir_place(R.tr, w + gkb::sparse_dir_bytes(A->m));
  int64_t tots[2][gkb::SP_BINS + 1];
  if (gkb::launch_sparse_bins(R.fwd, A->nnz, st) != hipSuccess || gkb::launch_sparse_bins(R.tr, A->nnz, st) != hipSuccess ||
      hipMemcpyAsync(tots[0], R.fwd.tot, sizeof(tots[0]), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(tots[1], R.tr.tot, sizeof(tots[1]), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    delete plan;
    return sfail(GKB_ERR_HIP, "binning the rows failed");
  }
  gkb::SparseDir* dirs[2] = {&R.fwd, &R.tr};
  for (int d = 0; d < 2; ++d) {
    int64_t acc = 0;
    for (int b = 0; b < gkb::SP_BINS; ++b) {
      dirs[d]->count[b] = tots[d][b];
      dirs[d]->base[b] = acc;
      acc += tots[d][b];
    }
    if (acc != dirs[d]->rows || tots[d][gkb::SP_BINS] != 0) {
      delete plan;
      return sfail(GKB_ERR_INVALID, d == 0 ? "invalid row_ptr or col_idx (offsets must be non-decreasing within "
                                             "[0, nnz], indices within [0, n))"
                                           : "invalid col_ptr or row_idx (offsets must be non-decreasing within "
                                             "[0, nnz], indices within [0, m))");
    }
  }
  *out = plan;
  return GKB_OK;
}

void gkb_sparse_plan_destroy(gkb_sparse_plan plan) { delete plan; }

gkb_status gkb_sparse_matvec(gkb_sparse_plan plan, int trans, const float* x, double* y, void* stream) {
  s_err.clear();
  if (!plan || !x || !y) return sfail(GKB_ERR_INVALID, "plan, x and y must be non-NULL");
  if (trans != 0 && trans != 1) return sfail(GKB_ERR_INVALID, "trans must be 0 or 1");
  const gkb::SparseDir& D = trans ? plan->ref.tr : plan->ref.fwd;
  if (gkb::launch_spmv(D, x, nullptr, nullptr, 0, y, nullptr, reinterpret_cast<hipStream_t>(stream)) !=
      hipSuccess)
    return sfail(GKB_ERR_HIP, "sparse product launch failed");
  return GKB_OK;
}

}  // extern "C"
