// Learned start vector for sequences of slowly changing matrices.
//
// A two-layer network maps, row by row, the features
//   x_i = [ S_i / c_S ,  sqrt(m) * s_j * U_prev[i, j] ]      (S = A Omega, the sketch;
//   U_prev = the previous solve's left Ritz vectors, each column signed so its
//   largest-magnitude entry is positive; c_S = RMS of S)
// to z_i = w2 . relu(W1 x_i + b1) + b2, and q1 = z / ||z|| starts the Golub-Kahan
// recurrence (eq. (2.1)).  Training minimises the energy of q1 outside the
// target left subspace U_t:  L = 1 - ||U_t^T z||^2 / ||z||^2.
//
// Kernels: feature statistics and assembly, forward, loss statistics,
// per-row backward (dL/dz, dL/dh), parameter gradients as MFMA GEMMs over the
// rows (gkb_gemm_tall with a ones column for the biases), gradient packing,
// Adam.  Every reduction has a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/gkb.h"
#include "../../include/gkb_learned.h"
#include "kernels.h"

namespace gkb {
namespace {

constexpr int XLD = 64;  // feature row stride: in features, a ones column, padding

inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
inline unsigned nblk(int64_t w, int64_t per) { return (unsigned)((w + per - 1) / per); }

__device__ __forceinline__ double wsum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ double bsum256(double v, double* red) {
  v = wsum_d(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  const double t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
}

// Blocks 0..r-1: sign of column j of Ut (r x m, rows contiguous) so that its
// largest-|.| entry (lowest index on ties) is positive.  Blocks r .. r +
// FS_PARTS - 1: part[b] = sum of squares of rows [b m / FS_PARTS, (b + 1) m /
// FS_PARTS) of every column of S (m x ws, column-major, leading dimension lds).
constexpr int FS_PARTS = 64;
__global__ __launch_bounds__(256) void k_feature_stats(const float* __restrict__ S, int64_t lds, int64_t m, int ws,
                                                       const float* __restrict__ Ut, int r, float* __restrict__ sgn,
                                                       double* __restrict__ part) {
  __shared__ double red[4];
  __shared__ float bv[256];
  __shared__ int bi[256];
  const int tid = threadIdx.x;
  if ((int)blockIdx.x < r) {
    const float* u = Ut + (int64_t)blockIdx.x * m;
    float best = -1.f;
    int64_t idx = 0;
    for (int64_t i = tid; i < m; i += 256) {
      const float a = fabsf(u[i]);
      if (a > best) {
        best = a;
        idx = i;
      }
    }
    bv[tid] = best;
    bi[tid] = (int)idx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) {
        const float a = bv[tid], b = bv[tid + s];
        const int ia = bi[tid], ib = bi[tid + s];
        if (b > a || (b == a && ib < ia)) {
          bv[tid] = b;
          bi[tid] = ib;
        }
      }
      __syncthreads();
    }
    if (tid == 0) sgn[blockIdx.x] = u[bi[0]] < 0.f ? -1.f : 1.f;
  } else {
    const int b = (int)blockIdx.x - r;
    const int64_t lo = b * m / FS_PARTS, hi = (b + 1) * m / FS_PARTS;
    double ss = 0.0;
    for (int c = 0; c < ws; ++c)
      for (int64_t i = lo + tid; i < hi; i += 256) {
        const float v = S[(int64_t)c * lds + i];
        ss += (double)v * v;
      }
    const double tot = bsum256(ss, red);
    if (tid == 0) part[b] = tot;
  }
}

// X[i] = [S_i / c_S, sqrt(m) sgn_j Ut[j, i], 1, 0 ...] with c_S = sqrt(sum of
// the FS_PARTS partial sums of squares (fixed order) / (m ws)); block 0 also
// stores c_S in *cs.
__global__ __launch_bounds__(256) void k_features(const float* __restrict__ S, int64_t lds, int64_t m, int ws,
                                                  const float* __restrict__ Ut, int r, const float* __restrict__ sgn,
                                                  const double* __restrict__ part, float* __restrict__ cs,
                                                  float* __restrict__ X) {
  static_assert(FS_PARTS == 64, "one partial per lane");
  __shared__ float csl;
  if (threadIdx.x < 64) {
    const double tot = wsum_d(part[threadIdx.x]);
    if (threadIdx.x == 0) {
      csl = (float)sqrt(tot / ((double)m * ws));
      if (blockIdx.x == 0) *cs = csl;
    }
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  const float inv = csl > 0.f ? 1.f / csl : 0.f;
  const float sm = sqrtf((float)m);
  float* xi = X + i * XLD;
  for (int c = 0; c < ws; ++c) xi[c] = S[(int64_t)c * lds + i] * inv;
  for (int j = 0; j < r; ++j) xi[ws + j] = sm * sgn[j] * Ut[(int64_t)j * m + i];
  xi[ws + r] = 1.f;
  for (int c = ws + r + 1; c < XLD; ++c) xi[c] = 0.f;
}

// The hidden layer of a workgroup's rows: the units go over the lanes in
// chunks of NH_CHUNK (lane l: units h0 + 2 l and h0 + 2 l + 1), W1 of the
// chunk staged in LDS transposed (W1T[c][k]: a lane's two weights of input c
// are adjacent), b1 and w2 beside it; x_c reaches every lane as a uniform
// value read from lane c.  a_k = b1[k] + sum_c W1[k][c] x_c with the sum in
// input order, as one thread per row would form it.
constexpr int NH_CHUNK = 128;
struct HiddenLds {
  float W1T[(XLD - 1) * NH_CHUNK];
  float b1[NH_CHUNK];
  float w2[NH_CHUNK];
};

// Stage units [h0, h0 + NH_CHUNK) (zeros past hidden).  Ends with a barrier.
__device__ void stage_hidden(const float* __restrict__ prm, int in, int hidden, int h0, HiddenLds& L) {
  const float* W1 = prm;
  const float* b1 = prm + (int64_t)hidden * in;
  const float* w2 = b1 + hidden;
  const int hc = min(NH_CHUNK, hidden - h0);
  __syncthreads();   // the previous chunk's readers are done
  for (int e = threadIdx.x; e < NH_CHUNK * in; e += blockDim.x) {
    const int kk = e / in, c = e - kk * in;
    L.W1T[c * NH_CHUNK + kk] = kk < hc ? W1[(int64_t)(h0 + kk) * in + c] : 0.f;
  }
  for (int kk = threadIdx.x; kk < NH_CHUNK; kk += blockDim.x) {
    L.b1[kk] = kk < hc ? b1[h0 + kk] : 0.f;
    L.w2[kk] = kk < hc ? w2[h0 + kk] : 0.f;
  }
  __syncthreads();
}

// Pre-activations of this lane's two units of the staged chunk for one row
// (xv: this lane's entry of the row, lanes 0 .. in - 1 used).
__device__ __forceinline__ float2 preact(const HiddenLds& L, int in, float xv) {
  const int lane = threadIdx.x & 63;
  float a0 = L.b1[2 * lane], a1 = L.b1[2 * lane + 1];
  const int xi = __float_as_int(xv);
  for (int c = 0; c < in; ++c) {
    const float xc = __int_as_float(__builtin_amdgcn_readlane(xi, c));
    const float2 w = *reinterpret_cast<const float2*>(&L.W1T[c * NH_CHUNK + 2 * lane]);
    a0 = fmaf(w.x, xc, a0);
    a1 = fmaf(w.y, xc, a1);
  }
  return make_float2(a0, a1);
}

// z_i = w2 . relu(W1 x_i + b1) + b2 for FW_ROWS rows per workgroup, a wave
// per row; the hidden-layer sum over each lane's units, then across the wave
// (butterfly), then over the chunks; optionally H[i * hld + k] = relu(.)_k,
// H[i * hld + hidden] = 1 and zeros up to hld.
constexpr int FW_ROWS = 32;
__global__ __launch_bounds__(256) void k_mlp_fwd(const float* __restrict__ prm, int in, int hidden,
                                                 const float* __restrict__ X, int64_t m, float* __restrict__ z,
                                                 float* __restrict__ H, int hld) {
  __shared__ HiddenLds L;
  __shared__ float zacc[FW_ROWS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * FW_ROWS;
  const int nr = (int)min<int64_t>(FW_ROWS, m - r0);
  const float* w2g = prm + (int64_t)hidden * in + hidden;
  for (int h0 = 0; h0 < hidden; h0 += NH_CHUNK) {
    stage_hidden(prm, in, hidden, h0, L);
    for (int rr = wave; rr < nr; rr += 4) {
      const int64_t i = r0 + rr;
      const float2 a = preact(L, in, X[i * XLD + lane]);
      const float h0v = a.x > 0.f ? a.x : 0.f, h1v = a.y > 0.f ? a.y : 0.f;
      float s = fmaf(L.w2[2 * lane + 1], h1v, L.w2[2 * lane] * h0v);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) zacc[rr] = h0 == 0 ? s : zacc[rr] + s;
      if (H) {
        const int k = h0 + 2 * lane;
        if (k < hidden) H[i * hld + k] = h0v;
        if (k + 1 < hidden) H[i * hld + k + 1] = h1v;
      }
    }
  }
  for (int rr = wave; rr < nr; rr += 4) {
    const int64_t i = r0 + rr;
    if (lane == 0) z[i] = w2g[hidden] + zacc[rr];
    if (H)
      for (int k = hidden + lane; k < hld; k += 64) H[i * hld + k] = k == hidden ? 1.f : 0.f;
  }
}

// stats[j] = U_t[:, j] . z for j < r (Ut rows contiguous), stats[r] = ||z||^2.
__global__ __launch_bounds__(256) void k_loss_stats(const float* __restrict__ Ut, int r, const float* __restrict__ z,
                                                    int64_t m, double* __restrict__ stats) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  double s = 0.0;
  if (j < r) {
    const float* u = Ut + (int64_t)j * m;
    for (int64_t i = threadIdx.x; i < m; i += 256) s += (double)u[i] * z[i];
  } else {
    for (int64_t i = threadIdx.x; i < m; i += 256) s += (double)z[i] * z[i];
  }
  const double t = bsum256(s, red);
  if (threadIdx.x == 0) stats[j] = t;
}

// Loss kind 0 (energy outside the target subspace): L = 1 - cc / zz with
// c = U_t^T z, cc = c.c, zz = z.z; dz_i = (2 / zz) (-(U_t c)_i + (cc / zz) z_i).
// Loss kind 1 (mean log tan^2 of the angles between z and each target vector,
// regularised by delta): a_j = (1 + delta) zz - c_j^2, b_j = c_j^2 + delta zz,
// L = (1/r) sum_j log(a_j / b_j); dz_i = s1 z_i - sum_j U_t[i, j] v_j with
// s1 = (1/r) sum_j (2 (1 + delta) / a_j - 2 delta / b_j),
// v_j = (2/r) c_j (1 / a_j + 1 / b_j).
// DH[i + k m] = dz_i w2[k] [a_k > 0]; block 0 writes the loss.
constexpr double LOGTAN_DELTA = 1e-6;

// FW_ROWS rows per workgroup: threads 0 .. FW_ROWS - 1 form dL/dz of their
// row, then a wave per row forms the pre-activations of a chunk of units and
// DH[i + k m] = dz_i w2[k] [a_k > 0], staged in LDS and written a unit at a
// time over consecutive rows.
__global__ __launch_bounds__(256) void k_mlp_bwd_rows(const float* __restrict__ prm, int in, int hidden,
                                                      const float* __restrict__ X, int64_t m,
                                                      const float* __restrict__ z, const float* __restrict__ Ut, int r,
                                                      const double* __restrict__ stats, float* __restrict__ dz,
                                                      float* __restrict__ DH, double* __restrict__ loss, int kind) {
  __shared__ HiddenLds L;
  __shared__ float gzs[FW_ROWS];
  __shared__ float dhs[NH_CHUNK * FW_ROWS];   // [unit][row]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * FW_ROWS;
  const int nr = (int)min<int64_t>(FW_ROWS, m - r0);
  const double zz = stats[r];
  if (tid < FW_ROWS) {
    const int64_t i = r0 + tid;
    double g = 0.0;
    if (kind == 0) {
      double cc = 0.0;
      for (int j = 0; j < r; ++j) cc += stats[j] * stats[j];
      if (blockIdx.x == 0 && tid == 0) *loss = zz > 0 ? 1.0 - cc / zz : 1.0;
      if (i < m) {
        double pz = 0.0;
        for (int j = 0; j < r; ++j) pz += (double)Ut[(int64_t)j * m + i] * stats[j];
        g = zz > 0 ? (2.0 / zz) * (-pz + (cc / zz) * (double)z[i]) : 0.0;
      }
    } else {
      const double dl = LOGTAN_DELTA;
      double lsum = 0.0, s1 = 0.0, pv = 0.0;
      for (int j = 0; j < r; ++j) {
        const double c = stats[j];
        const double a = (1.0 + dl) * zz - c * c, b = c * c + dl * zz;
        lsum += log(a / b);
        s1 += 2.0 * (1.0 + dl) / a - 2.0 * dl / b;
        if (i < m) pv += (double)Ut[(int64_t)j * m + i] * (2.0 / r) * c * (1.0 / a + 1.0 / b);
      }
      if (blockIdx.x == 0 && tid == 0) *loss = zz > 0 ? lsum / r : 0.0;
      if (i < m) g = zz > 0 ? (s1 / r) * (double)z[i] - pv : 0.0;
    }
    gzs[tid] = (float)g;
    if (i < m) dz[i] = (float)g;
  }
  for (int h0 = 0; h0 < hidden; h0 += NH_CHUNK) {
    stage_hidden(prm, in, hidden, h0, L);   // (its first barrier also publishes gzs)
    for (int rr = wave; rr < nr; rr += 4) {
      const int64_t i = r0 + rr;
      const float2 a = preact(L, in, X[i * XLD + lane]);
      const float gz = gzs[rr];
      dhs[(2 * lane) * FW_ROWS + rr] = a.x > 0.f ? gz * L.w2[2 * lane] : 0.f;
      dhs[(2 * lane + 1) * FW_ROWS + rr] = a.y > 0.f ? gz * L.w2[2 * lane + 1] : 0.f;
    }
    __syncthreads();
    const int hc = min(NH_CHUNK, hidden - h0);
    for (int e = tid; e < hc * FW_ROWS; e += 256) {
      const int kk = e / FW_ROWS, rr = e - kk * FW_ROWS;
      if (rr < nr) DH[(r0 + rr) + (int64_t)(h0 + kk) * m] = dhs[e];
    }
  }
}

// grad = [dW1 (hidden x in) | db1 | dw2 | db2] from G1 (XLD x hidden, column-major:
// G1[c + XLD k] = sum_i X[i][c] DH[i][k]) and G2 (hld: G2[k] = sum_i H[i][k] dz_i).
__global__ __launch_bounds__(256) void k_pack_grad(const float* __restrict__ G1, const float* __restrict__ G2,
                                                   int in, int hidden, float* __restrict__ grad) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nW = (int64_t)hidden * in;
  if (e < nW) {
    const int k = (int)(e / in), c = (int)(e % in);
    grad[e] = G1[c + (int64_t)XLD * k];
  } else if (e < nW + hidden) {
    const int k = (int)(e - nW);
    grad[e] = G1[in + (int64_t)XLD * k];
  } else if (e < nW + 2 * hidden) {
    grad[e] = G2[e - nW - hidden];
  } else if (e == nW + 2 * hidden) {
    grad[e] = G2[hidden];
  }
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m1, float* __restrict__ m2, int64_t count, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= count) return;
  const float gi = g[e];
  const float a = b1 * m1[e] + (1.f - b1) * gi;
  const float b = b2 * m2[e] + (1.f - b2) * gi * gi;
  m1[e] = a;
  m2[e] = b;
  p[e] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

__global__ __launch_bounds__(256) void k_to_double(const float* __restrict__ z, int64_t m, double* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < m) q[i] = (double)z[i];
}

// workspace layout for loss_grad / start vector
struct MlpWs {
  size_t z, dz, DH, H, stats, G1, G2, Gpart, total;
  int hld;
};

MlpWs mlp_ws(int64_t m, int hidden, int r) {
  MlpWs w{};
  w.hld = (hidden + 1 + 15) / 16 * 16;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off += al256(b);
    return o;
  };
  w.z = take((size_t)m * 4);
  w.dz = take((size_t)m * 4);
  w.DH = take((size_t)m * hidden * 4);
  w.H = take((size_t)m * w.hld * 4);
  w.stats = take((size_t)(r + 1) * 8);
  w.G1 = take((size_t)XLD * hidden * 4);
  w.G2 = take((size_t)w.hld * 4);
  // split-K partial sums of the two gradient products (reused one after the other)
  const GemmSplit s1 = gemm_split(XLD, m, hidden), s2 = gemm_split(w.hld, m, 1);
  w.Gpart = take(std::max((size_t)s1.slices * XLD * hidden, (size_t)s2.slices * w.hld) * 4);
  w.total = off;
  return w;
}

size_t feature_ws_bytes(int r) { return (size_t)FS_PARTS * 8 + (size_t)(r + 1) * 4; }

thread_local std::string l_err;
gkb_status lfail(gkb_status s, const char* msg) {
  l_err = msg;
  return s;
}

#define L_HIP(call)                                  \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) {                          \
      l_err = hipGetErrorString(e_);                 \
      return GKB_ERR_HIP;                            \
    }                                                \
  } while (0)

bool shapes_ok(int in, int hidden) { return in >= 1 && in + 1 <= XLD && hidden >= 1 && hidden <= 1024; }

}  // namespace
}  // namespace gkb

using namespace gkb;

extern "C" {

const char* gkb_learned_last_error(void) { return l_err.c_str(); }

int64_t gkb_mlp_param_count(int in, int hidden) {
  if (!shapes_ok(in, hidden)) return 0;
  return (int64_t)hidden * in + 2 * (int64_t)hidden + 1;
}

int gkb_mlp_feature_stride(void) { return XLD; }

size_t gkb_mlp_workspace_size(int64_t m, int in, int hidden, int r) {
  if (m < 1 || !shapes_ok(in, hidden) || r < 0) return 0;
  return mlp_ws(m, hidden, r).total + al256(64 * 8);
}

gkb_status gkb_mlp_features(const float* S, int64_t lds, int64_t m, int ws, const float* Ut_prev, int r, float* X,
                            void* workspace, size_t ws_bytes, void* stream) {
  l_err.clear();
  if (!S || !X || m < 1 || ws < 0 || r < 0 || ws + r + 1 > XLD || lds < m || (r > 0 && !Ut_prev))
    return lfail(GKB_ERR_INVALID, "bad feature arguments");
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 7) || ws_bytes < feature_ws_bytes(r))
    return lfail(GKB_ERR_WORKSPACE, "workspace too small or misaligned");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  double* part = reinterpret_cast<double*>(workspace);
  float* sgn = reinterpret_cast<float*>(part + FS_PARTS);
  float* cs = sgn + r;
  hipLaunchKernelGGL(k_feature_stats, dim3(r + FS_PARTS), dim3(256), 0, st, S, lds, m, ws, Ut_prev, r, sgn, part);
  L_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_features, dim3(nblk(m, 256)), dim3(256), 0, st, S, lds, m, ws, Ut_prev, r, sgn, part, cs,
                     X);
  L_HIP(hipGetLastError());
  return GKB_OK;
}

gkb_status gkb_mlp_forward(const float* params, int in, int hidden, const float* X, int64_t m, float* z,
                           void* stream) {
  l_err.clear();
  if (!params || !X || !z || m < 1 || !shapes_ok(in, hidden)) return lfail(GKB_ERR_INVALID, "bad forward arguments");
  hipLaunchKernelGGL(k_mlp_fwd, dim3(nblk(m, FW_ROWS)), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), params,
                     in, hidden, X, m, z, nullptr, 0);
  L_HIP(hipGetLastError());
  return GKB_OK;
}

gkb_status gkb_mlp_loss_grad(const float* params, int in, int hidden, const float* X, int64_t m, const float* Ut,
                             int r, float* grad, double* loss, void* workspace, size_t ws_bytes, void* stream) {
  return gkb_mlp_loss_grad_kind(params, in, hidden, X, m, Ut, r, 0, grad, loss, workspace, ws_bytes, stream);
}

gkb_status gkb_mlp_loss_grad_kind(const float* params, int in, int hidden, const float* X, int64_t m,
                                  const float* Ut, int r, int kind, float* grad, double* loss, void* workspace,
                                  size_t ws_bytes, void* stream) {
  l_err.clear();
  if (!params || !X || !Ut || !grad || !loss || m < 1 || r < 1 || !shapes_ok(in, hidden))
    return lfail(GKB_ERR_INVALID, "bad loss/gradient arguments");
  if (kind != 0 && kind != 1) return lfail(GKB_ERR_INVALID, "loss kind must be 0 or 1");
  MlpWs w = mlp_ws(m, hidden, r);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) || ws_bytes < w.total)
    return lfail(GKB_ERR_WORKSPACE, "workspace too small or misaligned");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* b = reinterpret_cast<char*>(workspace);
  float* z = reinterpret_cast<float*>(b + w.z);
  float* dz = reinterpret_cast<float*>(b + w.dz);
  float* DH = reinterpret_cast<float*>(b + w.DH);
  float* H = reinterpret_cast<float*>(b + w.H);
  double* stats = reinterpret_cast<double*>(b + w.stats);
  float* G1 = reinterpret_cast<float*>(b + w.G1);
  float* G2 = reinterpret_cast<float*>(b + w.G2);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(nblk(m, FW_ROWS)), dim3(256), 0, st, params, in, hidden, X, m, z, H, w.hld);
  L_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_loss_stats, dim3(r + 1), dim3(256), 0, st, Ut, r, z, m, stats);
  L_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mlp_bwd_rows, dim3(nblk(m, FW_ROWS)), dim3(256), 0, st, params, in, hidden, X, m, z, Ut, r,
                     stats, dz, DH, loss, kind);
  L_HIP(hipGetLastError());
  // G1 = X^T DH (XLD x hidden), G2 = H^T dz (hld x 1): sums over the rows on MFMA, split over row ranges
  float* Gpart = reinterpret_cast<float*>(b + w.Gpart);
  L_HIP(launch_gemm_tall_splitk<float>(X, XLD, XLD, (int)m, DH, m, hidden, G1, XLD, Gpart, st));
  L_HIP(launch_gemm_tall_splitk<float>(H, w.hld, w.hld, (int)m, dz, m, 1, G2, w.hld, Gpart, st));
  const int64_t P = gkb_mlp_param_count(in, hidden);
  hipLaunchKernelGGL(k_pack_grad, dim3(nblk(P, 256)), dim3(256), 0, st, G1, G2, in, hidden, grad);
  L_HIP(hipGetLastError());
  return GKB_OK;
}

gkb_status gkb_adam_step(float* params, const float* grad, float* m1, float* m2, int64_t count, double lr,
                         double beta1, double beta2, double eps, int step, void* stream) {
  l_err.clear();
  if (!params || !grad || !m1 || !m2 || count < 1 || step < 1) return lfail(GKB_ERR_INVALID, "bad Adam arguments");
  const float c1 = (float)(1.0 - std::pow(beta1, step)), c2 = (float)(1.0 - std::pow(beta2, step));
  hipLaunchKernelGGL(k_adam, dim3(nblk(count, 256)), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), params,
                     grad, m1, m2, count, (float)lr, (float)beta1, (float)beta2, (float)eps, c1, c2);
  L_HIP(hipGetLastError());
  return GKB_OK;
}

gkb_status gkb_mlp_start_vector(const float* params, int in, int hidden, const float* X, int64_t m, double* q1,
                                void* workspace, size_t ws_bytes, void* stream) {
  l_err.clear();
  if (!q1 || ws_bytes < al256((size_t)m * 4) || !workspace) return lfail(GKB_ERR_INVALID, "bad start arguments");
  gkb_status rc = gkb_mlp_forward(params, in, hidden, X, m, reinterpret_cast<float*>(workspace), stream);
  if (rc != GKB_OK) return rc;
  hipLaunchKernelGGL(k_to_double, dim3(nblk(m, 256)), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                     reinterpret_cast<const float*>(workspace), m, q1);
  L_HIP(hipGetLastError());
  return GKB_OK;
}

}  // extern "C"
