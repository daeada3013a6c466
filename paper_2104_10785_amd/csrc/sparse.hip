// Products with a sparse A (CSR of A for A p, CSR of A^T for A^T q).  The
// bidiagonalization only touches A through these two products
// (eq. (2.1)-(2.2)); the rest of the solver is shared with the dense path.
//
// Schedule (built on the host from the row offsets when the plan is made):
//  * short rows (<= SP_SHORT entries) are packed, in row order, into stream
//    blocks of consecutive rows with at most SP_BLOCK_NNZ entries: a workgroup
//    reads the block's index/value range with coalesced loads, gathers x and
//    leaves the products in LDS, then one thread per row adds its products in
//    order;
//  * medium rows (<= SP_HUGE) get a wave each: lane l takes entries
//    l, l + 64, ..., the 64 partial sums meet in a fixed butterfly;
//  * huge rows are cut into chunks of SP_HUGE entries, one workgroup per chunk,
//    and the chunk sums are added in chunk order.
// Every row sum has a fixed order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "sparse.h"

namespace gkb {

namespace {

constexpr int SP_T = 256;   // threads per workgroup
constexpr int SP_EPT = SP_BLOCK_NNZ / SP_T;   // entries per thread in a stream block (8)

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// sum over j = j0, j0 + G, ... < e of val[j] x[idx[j]], in that order; four
// entries' index and value loads are issued before their gathers.
__device__ __forceinline__ float strided_sum(const int32_t* __restrict__ idx, const float* __restrict__ val,
                                             const float* __restrict__ x, int64_t j, int64_t e, int G) {
  float s = 0.f;
  for (; j + 3 * G < e; j += 4 * G) {
    const int32_t i0 = idx[j], i1 = idx[j + G], i2 = idx[j + 2 * G], i3 = idx[j + 3 * G];
    const float v0 = val[j], v1 = val[j + G], v2 = val[j + 2 * G], v3 = val[j + 3 * G];
    const float x0 = x[i0], x1 = x[i1], x2 = x[i2], x3 = x[i3];
    s += v0 * x0;
    s += v1 * x1;
    s += v2 * x2;
    s += v3 * x3;
  }
  for (; j < e; j += G) s += val[j] * x[idx[j]];
  return s;
}

// Stream block b: blk[2b] = first row, blk[2b + 1] = row count.
__device__ __forceinline__ void spmv_stream_block(int b, const int64_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ idx, const float* __restrict__ val,
                                                  const int32_t* __restrict__ blk, const float* __restrict__ x,
                                                  const float* __restrict__ prev, const double* __restrict__ coef,
                                                  int cidx, double* __restrict__ y) {
  __shared__ float prod[SP_BLOCK_NNZ];
  __shared__ int64_t off[SP_SHORT + 1];
  const int r0 = blk[2 * b], nr = blk[2 * b + 1];
  for (int t = threadIdx.x; t <= nr; t += SP_T) off[t] = ptr[r0 + t];
  __syncthreads();
  const int64_t e0 = off[0];
  const int cnt = (int)(off[nr] - e0);
  int32_t ii[SP_EPT];
  float vv[SP_EPT];
#pragma unroll
  for (int u = 0; u < SP_EPT; ++u) {
    const int q = threadIdx.x + u * SP_T;
    ii[u] = q < cnt ? idx[e0 + q] : 0;
    vv[u] = q < cnt ? val[e0 + q] : 0.f;
  }
#pragma unroll
  for (int u = 0; u < SP_EPT; ++u) {
    const int q = threadIdx.x + u * SP_T;
    if (q < cnt) prod[q] = vv[u] * x[ii[u]];
  }
  __syncthreads();
  if (threadIdx.x < nr) {
    const int bq = (int)(off[threadIdx.x] - e0), e = (int)(off[threadIdx.x + 1] - e0);
    float s = 0.f;
    for (int q = bq; q < e; ++q) s += prod[q];
    const int row = r0 + threadIdx.x;
    y[row] = (double)s - (prev ? coef[cidx] * (double)prev[row] : 0.0);
  }
}

// Medium rows: one wave per row, 4 rows per workgroup (workgroup b).
__device__ __forceinline__ void spmv_wave_block(int b, const int64_t* __restrict__ ptr,
                                                const int32_t* __restrict__ idx, const float* __restrict__ val,
                                                const int32_t* __restrict__ rows, int64_t count,
                                                const float* __restrict__ x, const float* __restrict__ prev,
                                                const double* __restrict__ coef, int cidx, double* __restrict__ y) {
  const int64_t w = (int64_t)b * (SP_T / 64) + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (w >= count) return;   // uniform over the wave
  const int32_t row = rows[w];
  const float s = wave_sum_f(strided_sum(idx, val, x, ptr[row] + l, ptr[row + 1], 64));
  if (l == 0) y[row] = (double)s - (prev ? coef[cidx] * (double)prev[row] : 0.0);
}

// Huge rows, step 1: chunk c of row crow[c] covers entries
// [cbeg[c], min(cbeg[c] + SP_HUGE, end of the row)); part[c] = its sum.
__device__ __forceinline__ void spmv_chunk_block(int c, const int64_t* __restrict__ ptr,
                                                 const int32_t* __restrict__ idx, const float* __restrict__ val,
                                                 const int32_t* __restrict__ crow, const int64_t* __restrict__ cbeg,
                                                 const float* __restrict__ x, float* __restrict__ part) {
  __shared__ float red[SP_T / 64];
  const int64_t b = cbeg[c];
  const int64_t e = std::min<int64_t>(b + SP_HUGE, ptr[crow[c] + 1]);
  const float s = wave_sum_f(strided_sum(idx, val, x, b + threadIdx.x, e, SP_T));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
#pragma unroll
    for (int w = 0; w < SP_T / 64; ++w) t += red[w];
    part[c] = t;
  }
}

// All three row classes in one launch, so that their gathers overlap: the
// first nchunk workgroups take huge-row chunks, the next nwb medium rows (4
// per workgroup), the rest stream blocks of short rows.  Each row's sum is
// formed exactly as in its class's own schedule.
__global__ __launch_bounds__(SP_T) void k_spmv_rows(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                                                    const float* __restrict__ val, const int32_t* __restrict__ crow,
                                                    const int64_t* __restrict__ cbeg, int nchunk,
                                                    float* __restrict__ part, const int32_t* __restrict__ wrow,
                                                    int64_t nwrow, int nwb, const int32_t* __restrict__ sblk,
                                                    const float* __restrict__ x, const float* __restrict__ prev,
                                                    const double* __restrict__ coef, int cidx,
                                                    double* __restrict__ y, const int* __restrict__ flag) {
  if (flag != nullptr && flag[0] != 0) return;
  int b = (int)blockIdx.x;
  if (b < nchunk) {
    spmv_chunk_block(b, ptr, idx, val, crow, cbeg, x, part);
    return;
  }
  b -= nchunk;
  if (b < nwb) {
    spmv_wave_block(b, ptr, idx, val, wrow, nwrow, x, prev, coef, cidx, y);
    return;
  }
  spmv_stream_block(b - nwb, ptr, idx, val, sblk, x, prev, coef, cidx, y);
}

// Huge rows, step 2: y[row] = sum of its chunk sums in chunk order.
__global__ __launch_bounds__(SP_T) void k_spmv_huge_sum(const int32_t* __restrict__ hrow,
                                                         const int32_t* __restrict__ hfirst, int64_t nh,
                                                         const float* __restrict__ part,
                                                         const float* __restrict__ prev,
                                                         const double* __restrict__ coef, int cidx,
                                                         double* __restrict__ y, const int* __restrict__ flag) {
  if (flag != nullptr && flag[0] != 0) return;
  const int64_t h = (int64_t)blockIdx.x * SP_T + threadIdx.x;
  if (h >= nh) return;
  float s = 0.f;
  for (int c = hfirst[h]; c < hfirst[h + 1]; ++c) s += part[c];
  const int32_t row = hrow[h];
  y[row] = (double)s - (prev ? coef[cidx] * (double)prev[row] : 0.0);
}

// *bad += indices outside [0, cols)
__global__ __launch_bounds__(SP_T) void k_check_idx(const int32_t* __restrict__ idx, int64_t nnz, int64_t cols,
                                                     unsigned long long* __restrict__ bad) {
  unsigned long long nb = 0;
  for (int64_t j = (int64_t)blockIdx.x * SP_T + threadIdx.x; j < nnz; j += (int64_t)gridDim.x * SP_T)
    nb += (idx[j] < 0 || idx[j] >= cols) ? 1ull : 0ull;
  for (int o = 32; o > 0; o >>= 1) nb += __shfl_xor(nb, o, 64);
  if ((threadIdx.x & 63) == 0 && nb) atomicAdd(bad, nb);
}

__global__ void k_zero_u64(unsigned long long* p) {
  if (threadIdx.x == 0) *p = 0ull;
}

inline unsigned nblk(int64_t work, int64_t per) { return (unsigned)((work + per - 1) / per); }
inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

size_t sparse_dir_bytes(int64_t rows, int64_t nnz) {
  const int64_t maxh = nnz / SP_HUGE + 1;              // rows longer than SP_HUGE
  const int64_t maxc = 2 * (nnz / SP_HUGE) + 2;        // their chunks
  return a256((size_t)rows * 8) + a256((size_t)rows * 4) + a256((size_t)maxh * 4) + a256((size_t)(maxh + 1) * 4) +
         a256((size_t)maxc * 4) + a256((size_t)maxc * 8) + a256((size_t)maxc * 4) + 256;
}

// Build the schedule of D on the host from its row offsets (validated here:
// non-decreasing, within [0, nnz]); false if they are not.
bool sparse_schedule(SparseDir& D, const std::vector<int64_t>& p, int64_t nnz, std::vector<int32_t>& sblk,
                     std::vector<int32_t>& wrow, std::vector<int32_t>& hrow, std::vector<int32_t>& hfirst,
                     std::vector<int32_t>& crow, std::vector<int64_t>& cbeg) {
  if (p[0] != 0 || p[D.rows] != nnz) return false;
  int32_t run0 = -1, runn = 0;
  int64_t runnz = 0;
  auto flush = [&]() {
    if (runn > 0) {
      sblk.push_back(run0);
      sblk.push_back(runn);
    }
    runn = 0;
    runnz = 0;
  };
  hfirst.push_back(0);
  for (int64_t r = 0; r < D.rows; ++r) {
    const int64_t len = p[r + 1] - p[r];
    if (len < 0 || p[r + 1] > nnz) return false;
    if (len <= SP_SHORT) {
      if (runn == SP_SHORT || runnz + len > SP_BLOCK_NNZ) flush();
      if (runn == 0) run0 = (int32_t)r;
      ++runn;
      runnz += len;
    } else {
      flush();
      if (len <= SP_HUGE) {
        wrow.push_back((int32_t)r);
      } else {
        hrow.push_back((int32_t)r);
        for (int64_t b = p[r]; b < p[r + 1]; b += SP_HUGE) {
          crow.push_back((int32_t)r);
          cbeg.push_back(b);
        }
        hfirst.push_back((int32_t)crow.size());
      }
    }
  }
  flush();
  return true;
}

hipError_t launch_spmv(const SparseDir& D, const float* x, const float* prev, const double* coef, int cidx,
                       double* y, const int* flag, hipStream_t st) {
  if (D.panels) return launch_panels(D.pn, x, prev, coef, cidx, y, flag, st);
  const int nwb = (int)nblk(D.nwrow, SP_T / 64);
  const int64_t blocks = (int64_t)D.nchunk + nwb + D.nsblk;
  if (blocks > 0)
    hipLaunchKernelGGL(k_spmv_rows, dim3((unsigned)blocks), dim3(SP_T), 0, st, D.ptr, D.idx, D.val, D.crow, D.cbeg,
                       (int)D.nchunk, D.part, D.wrow, D.nwrow, nwb, D.sblk, x, prev, coef, cidx, y, flag);
  if (D.nhrow > 0)
    hipLaunchKernelGGL(k_spmv_huge_sum, dim3(nblk(D.nhrow, SP_T)), dim3(SP_T), 0, st, D.hrow, D.hfirst, D.nhrow,
                       D.part, prev, coef, cidx, y, flag);
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
  return gkb::sparse_dir_bytes(A->m, A->nnz) + gkb::sparse_dir_bytes(A->n, A->nnz) + 256;
}

size_t gkb_sparse_panel_workspace_size(const gkb_csr* A) {
  const size_t base = gkb_sparse_plan_workspace_size(A);
  if (base == 0) return 0;
  return base + gkb::panel_bytes_bound(A->m, A->n, A->nnz) + gkb::panel_bytes_bound(A->n, A->m, A->nnz);
}

namespace {
// Lay out a direction's schedule at w (at most sparse_dir_bytes bytes) and upload it.
hipError_t place_schedule(gkb::SparseDir& D, char* w, const std::vector<int32_t>& sblk,
                          const std::vector<int32_t>& wrow, const std::vector<int32_t>& hrow,
                          const std::vector<int32_t>& hfirst, const std::vector<int32_t>& crow,
                          const std::vector<int64_t>& cbeg, hipStream_t st) {
  auto a = [](size_t x) { return (x + 255) & ~size_t(255); };
  D.sblk = reinterpret_cast<int32_t*>(w);
  w += a(std::max<size_t>(sblk.size(), 1) * 4);
  D.wrow = reinterpret_cast<int32_t*>(w);
  w += a(std::max<size_t>(wrow.size(), 1) * 4);
  D.hrow = reinterpret_cast<int32_t*>(w);
  w += a(std::max<size_t>(hrow.size(), 1) * 4);
  D.hfirst = reinterpret_cast<int32_t*>(w);
  w += a(hfirst.size() * 4);
  D.crow = reinterpret_cast<int32_t*>(w);
  w += a(std::max<size_t>(crow.size(), 1) * 4);
  D.cbeg = reinterpret_cast<int64_t*>(w);
  w += a(std::max<size_t>(cbeg.size(), 1) * 8);
  D.part = reinterpret_cast<float*>(w);
  D.nsblk = (int64_t)sblk.size() / 2;
  D.nwrow = (int64_t)wrow.size();
  D.nhrow = (int64_t)hrow.size();
  D.nchunk = (int64_t)crow.size();
  hipError_t e = hipSuccess;
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (e == hipSuccess && bytes > 0) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
  };
  up(D.sblk, sblk.data(), sblk.size() * 4);
  up(D.wrow, wrow.data(), wrow.size() * 4);
  up(D.hrow, hrow.data(), hrow.size() * 4);
  up(D.hfirst, hfirst.data(), hfirst.size() * 4);
  up(D.crow, crow.data(), crow.size() * 4);
  up(D.cbeg, cbeg.data(), cbeg.size() * 8);
  if (e == hipSuccess) e = hipStreamSynchronize(st);   // the host vectors go out of scope
  return e;
}
}  // namespace

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
  // row offsets of both directions to the host: the schedule is built from them
  std::vector<int64_t> pf((size_t)A->m + 1), pt((size_t)A->n + 1);
  if (hipMemcpyAsync(pf.data(), A->row_ptr, pf.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(pt.data(), A->col_ptr, pt.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return sfail(GKB_ERR_HIP, "reading the row offsets failed");
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
  unsigned long long* bad = reinterpret_cast<unsigned long long*>(w);
  w += 256;
  gkb::SparseDir* dirs[2] = {&R.fwd, &R.tr};
  const std::vector<int64_t>* offs[2] = {&pf, &pt};
  for (int d = 0; d < 2; ++d) {
    std::vector<int32_t> sblk, wrow, hrow, hfirst, crow;
    std::vector<int64_t> cbeg;
    if (!gkb::sparse_schedule(*dirs[d], *offs[d], A->nnz, sblk, wrow, hrow, hfirst, crow, cbeg)) {
      delete plan;
      return sfail(GKB_ERR_INVALID, d == 0 ? "row_ptr must be non-decreasing from 0 to nnz"
                                           : "col_ptr must be non-decreasing from 0 to nnz");
    }
    if (place_schedule(*dirs[d], w, sblk, wrow, hrow, hfirst, crow, cbeg, st) != hipSuccess) {
      delete plan;
      return sfail(GKB_ERR_HIP, "uploading the schedule failed");
    }
    w += gkb::sparse_dir_bytes(dirs[d]->rows, A->nnz);
  }
  // every index in range (one pass over both index arrays)
  unsigned long long nbad = 1;
  hipLaunchKernelGGL(gkb::k_zero_u64, dim3(1), dim3(64), 0, st, bad);
  if (A->nnz > 0) {
    const unsigned g = (unsigned)std::min<int64_t>((A->nnz + 255) / 256, 4096);
    hipLaunchKernelGGL(gkb::k_check_idx, dim3(g), dim3(256), 0, st, A->col_idx, A->nnz, A->n, bad);
    hipLaunchKernelGGL(gkb::k_check_idx, dim3(g), dim3(256), 0, st, A->row_idx, A->nnz, A->m, bad);
  }
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&nbad, bad, 8, hipMemcpyDeviceToHost, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    delete plan;
    return sfail(GKB_ERR_HIP, "checking the indices failed");
  }
  if (nbad != 0) {
    delete plan;
    return sfail(GKB_ERR_INVALID, "column indices must lie in [0, n) and row indices of A^T in [0, m)");
  }
  // column panels, for the directions whose shape suits them, when the
  // workspace holds them (the bound of gkb_sparse_panel_workspace_size)
  if (ws_bytes >= gkb_sparse_panel_workspace_size(A)) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
      delete plan;
      return sfail(GKB_ERR_HIP, "querying the device failed");
    }
    const int32_t* didx[2] = {A->col_idx, A->row_idx};
    const float* dval[2] = {A->val, A->val_t};
    for (int d = 0; d < 2; ++d) {
      gkb::SparseDir& D = *dirs[d];
      const size_t bound = gkb::panel_bytes_bound(D.rows, D.cols, A->nnz);
      if (bound == 0) continue;
      std::vector<int32_t> hidx((size_t)A->nnz);
      std::vector<float> hval((size_t)A->nnz);
      if (A->nnz > 0 &&
          (hipMemcpyAsync(hidx.data(), didx[d], hidx.size() * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
           hipMemcpyAsync(hval.data(), dval[d], hval.size() * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
           hipStreamSynchronize(st) != hipSuccess)) {
        delete plan;
        return sfail(GKB_ERR_HIP, "reading the entries failed");
      }
      gkb::PanelLayout L;
      gkb::build_panels(D.rows, D.cols, A->nnz, offs[d]->data(), hidx.data(), hval.data(), cus, L);
      if (gkb::place_panels(L, w, D.pn, st) != hipSuccess) {
        delete plan;
        return sfail(GKB_ERR_HIP, "uploading the panel layout failed");
      }
      D.panels = true;
      w += bound;
    }
  }
  *out = plan;
  return GKB_OK;
}

void gkb_sparse_plan_destroy(gkb_sparse_plan plan) { delete plan; }

int gkb_sparse_plan_panels(gkb_sparse_plan plan) {
  if (!plan) return 0;
  return (plan->ref.fwd.panels ? 1 : 0) | (plan->ref.tr.panels ? 2 : 0);
}

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
