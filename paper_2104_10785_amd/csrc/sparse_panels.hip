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

constexpr int PN_EPT = PN_BLK / PN_T;                               // entries per thread in a stream block (8)
constexpr int PN_LONG = PN_BLK / (PN_SHORT + 1) + 1;                // long rows a block can hold
constexpr int PN_LDS = (PN_W + PN_BLK + PN_ROWS + 1 + 1 + PN_LONG) * 4;   // x panel, products, row offsets, long rows
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

__global__ __launch_bounds__(PN_T) void k_panel_main(PanelDev P, const float* __restrict__ x,
                                                      const float* __restrict__ prev, const double* __restrict__ coef,
                                                      int cidx, double* __restrict__ y, const int* __restrict__ flag) {
  extern __shared__ float lds[];
  float* xs = lds;                                   // PN_W
  float* prod = lds + PN_W;                          // PN_BLK
  int* off = reinterpret_cast<int*>(prod + PN_BLK);  // PN_ROWS + 1
  int* nlong = off + PN_ROWS + 1;                    // 1
  int* lrow = nlong + 1;                             // PN_LONG
  if (flag != nullptr && flag[0] != 0) return;
  const PnDesc J = P.jobs[blockIdx.x];
  const int b = J.a;
  const int t = threadIdx.x;
  const int64_t c0 = (int64_t)b * PN_W;
  const int pw = (int)std::min<int64_t>(PN_W, P.C - c0);
  const int64_t base = P.pbase[b];
  const uint16_t* __restrict__ ci = P.pidx + base;
  const float* __restrict__ cv = P.pval + base;
  // stream blocks {first row, rows, first entry, entries}: the first block's
  // offsets and entries are loaded before the panel of x, each next block's
  // while the rows of the current one are added
  const int32_t* __restrict__ po = P.poff + (int64_t)b * (P.R + 1);
  const PnDesc* sd = P.sblk + J.c;
  PnDesc d = {0, 0, 0, 0};
  int o = 0;
  uint32_t ii[PN_EPT];
  float vv[PN_EPT];
  if (J.b == 0) {
    d = sd[0];
    o = t <= d.b ? po[d.a + t] : 0;
#pragma unroll
    for (int u = 0; u < PN_EPT; ++u) {
      const int q = t + u * PN_T;
      ii[u] = q < d.d ? ci[d.c + q] : 0u;
      vv[u] = q < d.d ? cv[d.c + q] : 0.f;
    }
  }
  const float* xp = x + c0;
  if ((reinterpret_cast<uintptr_t>(xp) & 15) == 0) {
    const int n4 = pw >> 2;
    const float4* x4 = reinterpret_cast<const float4*>(xp);
    for (int i = t; i < n4; i += PN_T) reinterpret_cast<float4*>(xs)[i] = x4[i];
    for (int i = (n4 << 2) + t; i < pw; i += PN_T) xs[i] = xp[i];
  } else {
    for (int i = t; i < pw; i += PN_T) xs[i] = xp[i];
  }
  __syncthreads();

  if (J.b == 0) {
    for (int s = 0; s < J.d; ++s) {
      if (t <= d.b) off[t] = o - d.c;
#pragma unroll
      for (int u = 0; u < PN_EPT; ++u) {
        const int q = t + u * PN_T;
        if (q < d.d) prod[q] = vv[u] * xs[ii[u]];
      }
      const PnDesc dc = d;
      if (s + 1 < J.d) {
        d = sd[s + 1];
        o = t <= d.b ? po[d.a + t] : 0;
#pragma unroll
        for (int u = 0; u < PN_EPT; ++u) {
          const int q = t + u * PN_T;
          ii[u] = q < d.d ? ci[d.c + q] : 0u;
          vv[u] = q < d.d ? cv[d.c + q] : 0.f;
        }
      }
      if (t == 0) *nlong = 0;
      __syncthreads();
      // short rows: a thread each; long rows are listed for the waves (the
      // list order varies, each long row's sum does not)
      if (t < dc.b) {
        const int lo = off[t], hi = off[t + 1];
        if (hi - lo <= PN_SHORT) {
          float acc = 0.f;
          for (int q = lo; q < hi; ++q) acc += prod[q];
          put_row(P, b, (int64_t)dc.a + t, acc, prev, coef, cidx, y);
        } else {
          lrow[atomicAdd(nlong, 1)] = t;
        }
      }
      __syncthreads();
      const int nl = *nlong;
      for (int i = t >> 6; i < nl; i += PN_T / 64) {
        const int rt = lrow[i], l = t & 63;
        const int hi = off[rt + 1];
        float acc = 0.f;
        for (int q = off[rt] + l; q < hi; q += 64) acc += prod[q];
        acc = wave_sum(acc);
        if (l == 0) put_row(P, b, (int64_t)dc.a + rt, acc, prev, coef, cidx, y);
      }
      __syncthreads();
    }
  } else {
    // wave items {row, first entry, entries, chunk-sum slot}: a wave each
    const PnDesc* wd = P.witem + J.c;
    const int w = t >> 6, l = t & 63;
    for (int i = w; i < J.d; i += PN_T / 64) {
      const PnDesc it = wd[i];
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
