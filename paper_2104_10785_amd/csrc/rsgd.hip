// Riemannian mini-batch gradient descent for similarity learning
// (Section 4, Algorithm 4): the projection products, the matrix
// Y = (1 - eta lambda) W + eta P_W(M) and the retraction (the batched partial
// SVD solver on Y), captured into one hipGraph per plan.
//
// With W = U diag(s) Vf^T and M = (1/b) X^T diag(y) V (X: b x d1, V: b x d2):
//   T = V Vf (b x r),  R = X U (b x r)
//   A1 = M Vf = (1/b) X^T (y * T)          (d1 x r)
//   B1 = U^T M = (1/b) (y * R)^T V         (r x d2)
//   C1 = U^T M Vf = (1/b) (y * R)^T T      (r x r)
//   P_W(M) = A1 Vf^T + U B1 - U C1 Vf^T
// so M is never formed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>

#include "../../include/gkb.h"
#include "../../include/gkb_batched.h"
#include "../../include/gkb_rsgd.h"

namespace {

constexpr int RMAX = 16;   // largest rank handled by the small kernels' registers
constexpr int BMAX = 4096; // largest batch

thread_local std::string r_err;
gkb_status rfail(gkb_status s, const std::string& m) {
  r_err = m;
  return s;
}

inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }
inline unsigned nblk(int64_t work, int64_t per) { return (unsigned)((work + per - 1) / per); }

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One block per batch row i: T[i][k] = V[i, :] . Vf[:, k], R[i][k] = X[i, :] . U[:, k],
// each scaled by y_i (the factor every later product needs).
__global__ __launch_bounds__(256) void k_rsgd_rows(const float* __restrict__ X, const float* __restrict__ V,
                                                    const float* __restrict__ y, const float* __restrict__ U,
                                                    const float* __restrict__ Vf, int d1, int d2, int r,
                                                    double* __restrict__ yT, double* __restrict__ yR) {
  __shared__ double red[4][2 * RMAX];
  const int i = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double t[RMAX], q[RMAX];
#pragma unroll
  for (int k = 0; k < RMAX; ++k) t[k] = q[k] = 0.0;
  for (int j = threadIdx.x; j < d2; j += 256) {
    const double v = V[(int64_t)i * d2 + j];
#pragma unroll
    for (int k = 0; k < RMAX; ++k)
      if (k < r) t[k] += v * (double)Vf[(int64_t)k * d2 + j];
  }
  for (int c = threadIdx.x; c < d1; c += 256) {
    const double x = X[(int64_t)i * d1 + c];
#pragma unroll
    for (int k = 0; k < RMAX; ++k)
      if (k < r) q[k] += x * (double)U[(int64_t)k * d1 + c];
  }
#pragma unroll
  for (int k = 0; k < RMAX; ++k) {
    if (k < r) {
      const double a = wsum(t[k]), b = wsum(q[k]);
      if (lane == 0) {
        red[wave][k] = a;
        red[wave][RMAX + k] = b;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < r) {
    const int k = threadIdx.x;
    const double yi = y[i];
    yT[(int64_t)i * RMAX + k] = yi * (red[0][k] + red[1][k] + red[2][k] + red[3][k]);
    yR[(int64_t)i * RMAX + k] = yi * (red[0][RMAX + k] + red[1][RMAX + k] + red[2][RMAX + k] + red[3][RMAX + k]);
  }
}

// A1[c][k] = (1/b) sum_i X[i][c] yT[i][k]   (c < d1; stored c * RMAX + k)
// B1[k][j] = (1/b) sum_i yR[i][k] V[i][j]   (j < d2; stored j * RMAX + k)
// C1[k][l] = (1/b) sum_i yR[i][k] T[i][l]   (one extra block; T = y * yT)
__global__ __launch_bounds__(256) void k_rsgd_proj(const float* __restrict__ X, const float* __restrict__ V,
                                                    const float* __restrict__ y, const double* __restrict__ yT,
                                                    const double* __restrict__ yR, int b, int d1, int d2, int r,
                                                    double* __restrict__ A1, double* __restrict__ B1,
                                                    double* __restrict__ C1) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const double inv = 1.0 / b;
  if (e < d1) {
    double a[RMAX];
#pragma unroll
    for (int k = 0; k < RMAX; ++k) a[k] = 0.0;
    for (int i = 0; i < b; ++i) {
      const double x = X[(int64_t)i * d1 + e];
#pragma unroll
      for (int k = 0; k < RMAX; ++k)
        if (k < r) a[k] += x * yT[(int64_t)i * RMAX + k];
    }
#pragma unroll
    for (int k = 0; k < RMAX; ++k)
      if (k < r) A1[e * RMAX + k] = a[k] * inv;
  } else if (e < d1 + d2) {
    const int64_t j = e - d1;
    double a[RMAX];
#pragma unroll
    for (int k = 0; k < RMAX; ++k) a[k] = 0.0;
    for (int i = 0; i < b; ++i) {
      const double v = V[(int64_t)i * d2 + j];
#pragma unroll
      for (int k = 0; k < RMAX; ++k)
        if (k < r) a[k] += yR[(int64_t)i * RMAX + k] * v;
    }
#pragma unroll
    for (int k = 0; k < RMAX; ++k)
      if (k < r) B1[j * RMAX + k] = a[k] * inv;
  } else if (e < d1 + d2 + (int64_t)r * r) {
    const int64_t kl = e - d1 - d2;
    const int k = (int)(kl / r), l = (int)(kl % r);
    double a = 0.0;
    for (int i = 0; i < b; ++i) a += yR[(int64_t)i * RMAX + k] * (y[i] * yT[(int64_t)i * RMAX + l]);
    C1[k * RMAX + l] = a * inv;
  }
}

// Y[c][j] = (1 - eta lambda) sum_k U[c][k] s_k Vf[j][k]
//         + eta (sum_k A1[c][k] Vf[j][k] + sum_k U[c][k] B1[k][j] - sum_{k,l} U[c][k] C1[k][l] Vf[j][l])
__global__ __launch_bounds__(256) void k_rsgd_form(const float* __restrict__ U, const double* __restrict__ s,
                                                    const float* __restrict__ Vf, const double* __restrict__ A1,
                                                    const double* __restrict__ B1, const double* __restrict__ C1,
                                                    int d1, int d2, int r, double keep, double eta,
                                                    float* __restrict__ Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)d1 * d2) return;
  const int64_t c = e / d2, j = e % d2;
  double uc[RMAX], vj[RMAX];
#pragma unroll
  for (int k = 0; k < RMAX; ++k) {
    uc[k] = k < r ? (double)U[(int64_t)k * d1 + c] : 0.0;
    vj[k] = k < r ? (double)Vf[(int64_t)k * d2 + j] : 0.0;
  }
  double w = 0.0, p = 0.0;
#pragma unroll
  for (int k = 0; k < RMAX; ++k) {
    if (k < r) {
      w += uc[k] * s[k] * vj[k];
      p += A1[c * RMAX + k] * vj[k] + uc[k] * B1[j * RMAX + k];
      double cv = 0.0;
#pragma unroll
      for (int l = 0; l < RMAX; ++l)
        if (l < r) cv += C1[k * RMAX + l] * vj[l];
      p -= uc[k] * cv;
    }
  }
  Y[c * ldy + j] = (float)(keep * w + eta * p);
}

__global__ __launch_bounds__(256) void k_rsgd_weights(const float* __restrict__ U, const double* __restrict__ s,
                                                       const float* __restrict__ Vf, int d1, int d2, int r,
                                                       float* __restrict__ W) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)d1 * d2) return;
  const int64_t c = e / d2, j = e % d2;
  double w = 0.0;
  for (int k = 0; k < r; ++k) w += (double)U[(int64_t)k * d1 + c] * s[k] * (double)Vf[(int64_t)k * d2 + j];
  W[e] = (float)w;
}

struct RsgdLayout {
  size_t yT = 0, yR = 0, A1 = 0, B1 = 0, C1 = 0, Y = 0, batch = 0, total = 0;
  int64_t ldy = 0;
};

RsgdLayout rsgd_layout(int d1, int d2, int r, int k, int b, size_t batch_ws) {
  RsgdLayout L;
  size_t off = 0;
  auto take = [&](size_t n) {
    size_t o = off;
    off += a256(n);
    return o;
  };
  L.ldy = (d2 + 3) & ~3;   // 16-byte rows: the batched solver reads Y without staging
  L.yT = take((size_t)b * RMAX * 8);
  L.yR = take((size_t)b * RMAX * 8);
  L.A1 = take((size_t)d1 * RMAX * 8);
  L.B1 = take((size_t)d2 * RMAX * 8);
  L.C1 = take((size_t)RMAX * RMAX * 8);
  L.Y = take((size_t)d1 * L.ldy * 4);
  L.batch = take(batch_ws);
  L.total = off;
  (void)k;
  (void)r;
  return L;
}

bool sizes_ok(int d1, int d2, int r, int k, int b) {
  return d1 >= 1 && d2 >= 1 && r >= 1 && r <= RMAX && r <= k && k <= std::min(d1, d2) && k <= 64 && b >= 1 &&
         b <= BMAX;
}

gkb_matrix y_matrix(int d1, int d2, int64_t ldy, const void* Y) {
  gkb_matrix A{};
  A.m = d1;
  A.n = d2;
  A.lda = ldy;
  A.dtype = GKB_F32;
  A.data = Y;
  return A;
}

}  // namespace

struct gkb_rsgd_plan_s {
  int d1 = 0, d2 = 0, r = 0, k = 0, b = 0;
  gkb_batch_plan solve = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;
};

extern "C" {

const char* gkb_rsgd_last_error(void) { return r_err.c_str(); }

size_t gkb_rsgd_workspace_size(int d1, int d2, int r, int k, int b) {
  if (!sizes_ok(d1, d2, r, k, b)) return 0;
  const int64_t ldy = (d2 + 3) & ~3;
  gkb_matrix A = y_matrix(d1, d2, ldy, nullptr);
  A.data = reinterpret_cast<const void*>(256);   // shape query only
  const size_t bw = gkb_batched_workspace_size(1, &A, &r, &k);
  if (bw == 0) return 0;
  return rsgd_layout(d1, d2, r, k, b, bw).total;
}

void gkb_rsgd_plan_destroy(gkb_rsgd_plan plan) {
  if (!plan) return;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  if (plan->capture) (void)hipStreamDestroy(plan->capture);
  if (plan->solve) gkb_batched_plan_destroy(plan->solve);
  delete plan;
}

gkb_status gkb_rsgd_plan_create(int d1, int d2, int r, int k, int b, double eta, double lambda, const float* X,
                                const float* V, const float* y, float* U, double* s, float* Vf, void* workspace,
                                size_t ws_bytes, void* stream, gkb_rsgd_plan* out) {
  r_err.clear();
  if (!out) return rfail(GKB_ERR_INVALID, "plan pointer is NULL");
  *out = nullptr;
  if (!sizes_ok(d1, d2, r, k, b))
    return rfail(GKB_ERR_INVALID, "need 1 <= r <= 16, r <= k <= min(d1, d2), k <= 64, 1 <= b <= 4096");
  if (!X || !V || !y || !U || !s || !Vf) return rfail(GKB_ERR_INVALID, "batch and state pointers must be non-NULL");
  if (!(eta > 0.0) || !(lambda >= 0.0)) return rfail(GKB_ERR_INVALID, "need eta > 0 and lambda >= 0");
  const size_t need = gkb_rsgd_workspace_size(d1, d2, r, k, b);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) || ws_bytes < need)
    return rfail(GKB_ERR_WORKSPACE, "workspace missing, misaligned or too small (need " + std::to_string(need) +
                                        " bytes)");
  const int64_t ldy = (d2 + 3) & ~3;
  gkb_matrix Aq = y_matrix(d1, d2, ldy, reinterpret_cast<const void*>(256));
  const size_t bw = gkb_batched_workspace_size(1, &Aq, &r, &k);
  RsgdLayout L = rsgd_layout(d1, d2, r, k, b, bw);
  char* ws = reinterpret_cast<char*>(workspace);
  double* yT = reinterpret_cast<double*>(ws + L.yT);
  double* yR = reinterpret_cast<double*>(ws + L.yR);
  double* A1 = reinterpret_cast<double*>(ws + L.A1);
  double* B1 = reinterpret_cast<double*>(ws + L.B1);
  double* C1 = reinterpret_cast<double*>(ws + L.C1);
  float* Y = reinterpret_cast<float*>(ws + L.Y);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  auto* plan = new gkb_rsgd_plan_s();
  plan->d1 = d1;
  plan->d2 = d2;
  plan->r = r;
  plan->k = k;
  plan->b = b;
  // the retraction: one problem, Krylov dimension k, no restart, outputs = the state
  gkb_matrix A = y_matrix(d1, d2, ldy, Y);
  gkb_batch_options bo;
  gkb_batch_default_options(&bo);
  bo.no_graph = 1;
  bo.seed = 0x5eed;
  bo.max_team = 1;   // a d1 x d2 of this size streams fastest from one workgroup, without team barriers
  gkb_status rc = gkb_batched_plan_create(1, &A, &r, &k, 0.0, 0, &bo, ws + L.batch, bw, s, U, Vf, stream,
                                          &plan->solve);
  if (rc != GKB_OK) {
    r_err = std::string("retraction plan: ") + gkb_batched_last_error();
    delete plan;
    return rc;
  }
  const double keep = 1.0 - eta * lambda;
  auto fail_hip = [&](const char* what) {
    gkb_rsgd_plan_destroy(plan);
    return rfail(GKB_ERR_HIP, what);
  };
  if (hipStreamCreateWithFlags(&plan->capture, hipStreamNonBlocking) != hipSuccess)
    return fail_hip("cannot create the capture stream");
  if (hipStreamBeginCapture(plan->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail_hip("cannot begin graph capture");
  hipLaunchKernelGGL(k_rsgd_rows, dim3(b), dim3(256), 0, plan->capture, X, V, y, U, Vf, d1, d2, r, yT, yR);
  hipError_t le = hipGetLastError();
  hipLaunchKernelGGL(k_rsgd_proj, dim3(nblk((int64_t)d1 + d2 + (int64_t)r * r, 256)), dim3(256), 0, plan->capture,
                     X, V, y, yT, yR, b, d1, d2, r, A1, B1, C1);
  if (le == hipSuccess) le = hipGetLastError();
  hipLaunchKernelGGL(k_rsgd_form, dim3(nblk((int64_t)d1 * d2, 256)), dim3(256), 0, plan->capture, U, s, Vf, A1,
                     B1, C1, d1, d2, r, keep, eta, Y, ldy);
  if (le == hipSuccess) le = hipGetLastError();
  gkb_status srun = gkb_batched_plan_run(plan->solve, plan->capture);
  hipError_t ee = hipStreamEndCapture(plan->capture, &plan->graph);
  if (le != hipSuccess || srun != GKB_OK || ee != hipSuccess) return fail_hip("graph capture failed");
  if (hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0) != hipSuccess)
    return fail_hip("graph instantiation failed");
  (void)st;
  *out = plan;
  return GKB_OK;
}

gkb_status gkb_rsgd_plan_step(gkb_rsgd_plan plan, void* stream) {
  r_err.clear();
  if (!plan || !plan->exec) return rfail(GKB_ERR_INVALID, "invalid plan");
  if (hipGraphLaunch(plan->exec, reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
    return rfail(GKB_ERR_HIP, "graph launch failed");
  return GKB_OK;
}

gkb_status gkb_rsgd_plan_info(gkb_rsgd_plan plan, int* info4, void* stream) {
  r_err.clear();
  if (!plan || !info4) return rfail(GKB_ERR_INVALID, "invalid plan or info pointer");
  gkb_status rc = gkb_batched_plan_info(plan->solve, info4, stream);
  if (rc != GKB_OK) return rfail(rc, gkb_batched_last_error());
  return GKB_OK;
}

gkb_status gkb_rsgd_weights(int d1, int d2, int r, const float* U, const double* s, const float* Vf, float* W,
                            void* stream) {
  r_err.clear();
  if (d1 < 1 || d2 < 1 || r < 1 || !U || !s || !Vf || !W) return rfail(GKB_ERR_INVALID, "bad arguments");
  hipLaunchKernelGGL(k_rsgd_weights, dim3(nblk((int64_t)d1 * d2, 256)), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), U, s, Vf, d1, d2, r, W);
  if (hipGetLastError() != hipSuccess) return rfail(GKB_ERR_HIP, "launch failed");
  return GKB_OK;
}

}  // extern "C"
