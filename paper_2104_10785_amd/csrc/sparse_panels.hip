// Products through the column-panel layout (sparse_panels.h): one workgroup
// per job loads its panel of x into LDS and streams the job's entries, so the
// gathers of x are LDS reads; the row sums of each panel go to `partial` and a
// last launch adds them in panel order (one panel: straight to y).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "sparse.h"

namespace gkb {

namespace {

constexpr int PN_EPT = PN_BLK / PN_T;                               // entries per thread in a stream block (4)
constexpr int PN_LONG = 128;                                        // long rows a block can hold
static_assert(PN_BLK / (PN_SHORT + 1) <= PN_LONG, "long-row list too short");
// the job's item descriptors (and four empty ones after them), x panel, and
// two buffers of products, row offsets and long-row lists
constexpr int PN_DSC = PN_JOB_ITEMS + 4;
constexpr int PN_LDS = PN_DSC * 16 + (PN_W + 2 * (PN_BLK + PN_ROWS + 1 + PN_LONG)) * 4;
static_assert(PN_LDS <= 160 * 1024, "panel workgroup LDS above the compute unit's 160 KB");
constexpr int PN_XV = (PN_W / 4 + PN_T - 1) / PN_T;                 // float4 of the x panel per thread
constexpr int PN_WAVE_LOADS = 8;                                     // entries per lane in flight (wave items)

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// A row's sum in panel b: into the per-panel sums, or (one panel) the result.
__device__ __forceinline__ void put_row(const PanelDev& P, int b, int64_t row, float s, const float* __restrict__ prev,
                                        const double* __restrict__ coef, int cidx, double* __restrict__ y) {
  if (P.partial != nullptr)
    P.partial[(int64_t)b * P.R + row] = s;
  else
    y[row] = (double)s - (prev ? coef[cidx] * (double)prev[row] : 0.0);
}

// One stream block's operands in registers: its descriptor, thread t's row
// offset, thread t's entry of the block's long-row list and thread t's
// entries (t + u PN_T, u < PN_EPT).
struct BlkRegs {
  PnDesc d;
  int o, lr;
  uint32_t ii[PN_EPT];
  float vv[PN_EPT];
};

__device__ __forceinline__ int blk_rows(const PnDesc& d) { return d.b & 1023; }
__device__ __forceinline__ int blk_entries(const PnDesc& d) { return (d.b >> 10) & 8191; }
__device__ __forceinline__ int blk_longs(const PnDesc& d) { return d.b >> 23; }

// Every load is issued unconditionally (indices clamped into the block, the
// values of lanes past its end zeroed afterwards), so that the compiler can
// count the loads in flight exactly and wait for one block's loads only.  An
// empty block reads the entry at its start and the padding of the long-row
// list.
__device__ __forceinline__ void blk_load(BlkRegs& B, const PnDesc* dsc, int s, const int32_t* __restrict__ po,
                                         const int32_t* __restrict__ lrow, const uint16_t* __restrict__ ci,
                                         const float* __restrict__ cv, int t) {
  B.d = dsc[s];
  const int nr = blk_rows(B.d), cnt = blk_entries(B.d), lc = blk_longs(B.d);
  B.o = po[B.d.a + min(t, nr)];
  B.lr = lrow[B.d.d + min(t, max(lc - 1, 0))];
#pragma unroll
  for (int u = 0; u < PN_EPT; ++u) {
    const int q = t + u * PN_T;
    const int qc = q < cnt ? q : 0;
    B.ii[u] = ci[B.d.c + qc];
    B.vv[u] = cv[B.d.c + qc];
  }
}

// Block s (operands in B) on LDS buffer K: its offsets, long-row list and
// products into the buffer, then B receives block s + 2 (an empty descriptor
// past the job's end), then one barrier, then the row sums: rows of at most
// PN_SHORT entries by their thread, the listed long rows by the waves.  Block
// s + 1 uses the other buffer, and the barrier of block s + 1 comes after
// every thread's sums of block s, so one barrier per block suffices.
template <int K>
__device__ __forceinline__ void blk_step(BlkRegs& B, int s, const PnDesc* dsc, const int32_t* __restrict__ po,
                                         const int32_t* __restrict__ lrow, const uint16_t* __restrict__ ci,
                                         const float* __restrict__ cv, const float* xs, float* prod, int* off,
                                         int* lst, const PanelDev& P, int b, const float* __restrict__ prev,
                                         const double* __restrict__ coef, int cidx, double* __restrict__ y, int t) {
  float* pk = prod + K * PN_BLK;
  int* ok = off + K * (PN_ROWS + 1);
  int* lk = lst + K * PN_LONG;
  const int nr = blk_rows(B.d), cnt = blk_entries(B.d), lc = blk_longs(B.d);
  if (t <= nr) ok[t] = B.o - B.d.c;
  if (t < lc) lk[t] = B.lr;
  float pr[PN_EPT];
#pragma unroll
  for (int u = 0; u < PN_EPT; ++u) pr[u] = B.vv[u] * xs[B.ii[u]];
#pragma unroll
  for (int u = 0; u < PN_EPT; ++u) {
    const int q = t + u * PN_T;
    if (q < cnt) pk[q] = pr[u];
  }
  const int r0 = B.d.a;
  blk_load(B, dsc, s + 2, po, lrow, ci, cv, t);
  __syncthreads();
  if (t < nr) {
    const int lo = ok[t], hi = ok[t + 1];
    if (hi - lo <= PN_SHORT) {
      // in entry order; eight LDS reads in flight per batch
      float acc = 0.f;
      int q = lo;
      for (; q + 8 <= hi; q += 8) {
        float pb[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) pb[k] = pk[q + k];
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += pb[k];
      }
      for (; q < hi; ++q) acc += pk[q];
      put_row(P, b, (int64_t)r0 + t, acc, prev, coef, cidx, y);
    }
  }
  for (int i = t >> 6; i < lc; i += PN_T / 64) {
    const int rt = lk[i], l = t & 63;
    const int hi = ok[rt + 1];
    float acc = 0.f;
    int q = ok[rt] + l;
    for (; q + 192 < hi; q += 256) {
      const float p0 = pk[q], p1 = pk[q + 64], p2 = pk[q + 128], p3 = pk[q + 192];
      acc += p0;
      acc += p1;
      acc += p2;
      acc += p3;
    }
    for (; q < hi; q += 64) acc += pk[q];
    acc = wave_sum(acc);
    if (l == 0) put_row(P, b, (int64_t)r0 + rt, acc, prev, coef, cidx, y);
  }
}

__global__ __launch_bounds__(PN_T) void k_panel_main(PanelDev P, const float* __restrict__ x,
                                                      const float* __restrict__ prev, const double* __restrict__ coef,
                                                      int cidx, double* __restrict__ y, const int* __restrict__ flag) {
  extern __shared__ float4 lds4[];
  PnDesc* dsc = reinterpret_cast<PnDesc*>(lds4);                       // PN_DSC
  float* xs = reinterpret_cast<float*>(lds4 + PN_DSC);                 // PN_W
  float* prod = xs + PN_W;                                             // 2 x PN_BLK
  int* off = reinterpret_cast<int*>(prod + 2 * PN_BLK);                // 2 x (PN_ROWS + 1)
  int* lst = off + 2 * (PN_ROWS + 1);                                  // 2 x PN_LONG
  if (flag != nullptr && flag[0] != 0) return;
  const PnDesc J = P.jobs[blockIdx.x];
  const int b = J.a;
  const int t = threadIdx.x;
  const int64_t c0 = (int64_t)b * PN_W;
  const int pw = (int)std::min<int64_t>(PN_W, P.C - c0);
  const int64_t base = P.pbase[b];
  const uint16_t* __restrict__ ci = P.pidx + base;
  const float* __restrict__ cv = P.pval + base;
  // the job's item descriptors and the panel of x into LDS, every load
  // issued before the first wait
  const PnDesc* jd = (J.b == 0 ? P.sblk : P.witem) + J.c;
  const int4 dl = t < J.d ? reinterpret_cast<const int4*>(jd)[t] : make_int4(0, 0, 0, 0);   // J.d <= PN_JOB_ITEMS
  const float* xp = x + c0;
  if ((reinterpret_cast<uintptr_t>(xp) & 15) == 0) {
    const int n4 = pw >> 2;
    const float4* x4 = reinterpret_cast<const float4*>(xp);
    float4 xv[PN_XV];
#pragma unroll
    for (int k = 0; k < PN_XV; ++k) {
      const int i = t + k * PN_T;
      xv[k] = i < n4 ? x4[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < PN_XV; ++k) {
      const int i = t + k * PN_T;
      if (i < n4) reinterpret_cast<float4*>(xs)[i] = xv[k];
    }
    for (int i = (n4 << 2) + t; i < pw; i += PN_T) xs[i] = xp[i];
  } else {
    for (int i = t; i < pw; i += PN_T) xs[i] = xp[i];
  }
  if (t < J.d + 4) reinterpret_cast<int4*>(dsc)[t] = dl;
  __syncthreads();

  // stream blocks {first row, rows, first entry, entries}: block s + 2's
  // offsets and entries are loaded while the rows of block s are added (two
  // register sets).  The loads and steps run unconditionally (on the empty
  // descriptors past the job's end), so that the waits for block s never
  // cover block s + 1's loads.
  if (J.b == 0) {
    const int32_t* __restrict__ po = P.poff + (int64_t)b * (P.R + 1);
    BlkRegs A, B;
    blk_load(A, dsc, 0, po, P.lrow, ci, cv, t);
    blk_load(B, dsc, 1, po, P.lrow, ci, cv, t);
    for (int s = 0; s < J.d; s += 2) {
      blk_step<0>(A, s, dsc, po, P.lrow, ci, cv, xs, prod, off, lst, P, b, prev, coef, cidx, y, t);
      blk_step<1>(B, s + 1, dsc, po, P.lrow, ci, cv, xs, prod, off, lst, P, b, prev, coef, cidx, y, t);
    }
  } else {
    // wave items {row, first entry, entries, chunk-sum slot}: a wave each
    const int w = t >> 6, l = t & 63;
    for (int i = w; i < J.d; i += PN_T / 64) {
      const PnDesc it = dsc[i];
      const uint16_t* __restrict__ ic = ci + it.b;
      const float* __restrict__ vc = cv + it.b;
      float s = 0.f;
      int j = l;
      for (; j + 64 * (PN_WAVE_LOADS - 1) < it.c; j += 64 * PN_WAVE_LOADS) {
        uint32_t ik[PN_WAVE_LOADS];
        float vk[PN_WAVE_LOADS];
#pragma unroll
        for (int k = 0; k < PN_WAVE_LOADS; ++k) {
          ik[k] = ic[j + 64 * k];
          vk[k] = vc[j + 64 * k];
        }
#pragma unroll
        for (int k = 0; k < PN_WAVE_LOADS; ++k) s += vk[k] * xs[ik[k]];
      }
      for (; j < it.c; j += 64) s += vc[j] * xs[ic[j]];
      s = wave_sum(s);
      if (l == 0) P.slot[it.d] = s;
    }
  }
}

// Segments of several chunks: their chunk sums added in chunk order.
__global__ __launch_bounds__(256) void k_panel_segsum(PanelDev P, const float* __restrict__ prev,
                                                       const double* __restrict__ coef, int cidx,
                                                       double* __restrict__ y, const int* __restrict__ flag) {
  if (flag != nullptr && flag[0] != 0) return;
  const int64_t h = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (h >= P.nsegs) return;
  const PnDesc g = P.segs[h];
  float s = 0.f;
  for (int c = 0; c < g.d; ++c) s += P.slot[g.c + c];
  put_row(P, g.a, g.b, s, prev, coef, cidx, y);
}

// y[row] = the row's panel sums added in panel order, minus coef * prev.
__global__ __launch_bounds__(256) void k_panel_rowsum(PanelDev P, const float* __restrict__ prev,
                                                       const double* __restrict__ coef, int cidx,
                                                       double* __restrict__ y, const int* __restrict__ flag) {
  if (flag != nullptr && flag[0] != 0) return;
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= P.R) return;
  float s = P.partial[r];
  for (int b = 1; b < P.np; ++b) s += P.partial[(int64_t)b * P.R + r];
  y[r] = (double)s - (prev ? coef[cidx] * (double)prev[r] : 0.0);
}

inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

hipError_t place_panels(const PanelLayout& L, char* w, PanelDev& P, hipStream_t st) {
  P = PanelDev();
  P.R = L.R;
  P.C = L.C;
  P.np = L.np;
  hipError_t e = hipSuccess;
  auto put = [&](const void* src, size_t bytes) -> char* {
    char* at = w;
    if (e == hipSuccess && bytes > 0) e = hipMemcpyAsync(at, src, bytes, hipMemcpyHostToDevice, st);
    w += a256(bytes);
    return at;
  };
  P.pidx = reinterpret_cast<const uint16_t*>(put(L.pidx.data(), L.pidx.size() * 2));
  P.pval = reinterpret_cast<const float*>(put(L.pval.data(), L.pval.size() * 4));
  P.poff = reinterpret_cast<const int32_t*>(put(L.poff.data(), L.poff.size() * 4));
  P.pbase = reinterpret_cast<const int64_t*>(put(L.pbase.data(), L.pbase.size() * 8));
  P.jobs = reinterpret_cast<const PnDesc*>(put(L.jobs.data(), L.jobs.size() * 16));
  P.sblk = reinterpret_cast<const PnDesc*>(put(L.sblk.data(), L.sblk.size() * 16));
  P.witem = reinterpret_cast<const PnDesc*>(put(L.witem.data(), L.witem.size() * 16));
  P.segs = reinterpret_cast<const PnDesc*>(put(L.segs.data(), L.segs.size() * 16));
  P.lrow = reinterpret_cast<const int32_t*>(put(L.lrow.data(), L.lrow.size() * 4));
  P.njobs = (int64_t)L.jobs.size();
  P.nsegs = (int64_t)L.segs.size();
  P.slot = reinterpret_cast<float*>(w);
  w += a256((size_t)L.nslot * 4);
  P.partial = L.np > 1 ? reinterpret_cast<float*>(w) : nullptr;
  if (e == hipSuccess) e = hipStreamSynchronize(st);   // the host arrays may go once this returns
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_panel_main), hipFuncAttributeMaxDynamicSharedMemorySize,
                            PN_LDS);
  return e;
}

hipError_t launch_panels(const PanelDev& P, const float* x, const float* prev, const double* coef, int cidx,
                         double* y, const int* flag, hipStream_t st) {
  if (P.njobs > 0)
    hipLaunchKernelGGL(k_panel_main, dim3((unsigned)P.njobs), dim3(PN_T), PN_LDS, st, P, x, prev, coef, cidx, y, flag);
  if (P.nsegs > 0)
    hipLaunchKernelGGL(k_panel_segsum, dim3((unsigned)((P.nsegs + 255) / 256)), dim3(256), 0, st, P, prev, coef,
                       cidx, y, flag);
  if (P.np > 1)
    hipLaunchKernelGGL(k_panel_rowsum, dim3((unsigned)((P.R + 255) / 256)), dim3(256), 0, st, P, prev, coef, cidx,
                       y, flag);
  return hipGetLastError();
}

}  // namespace gkb
