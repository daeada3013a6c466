// Host driver behind the C ABI (include/gkb.h): argument checks, workspace
// layout, the Golub-Kahan cycle loop, thick restart, convergence test and the
// final Ritz-vector GEMMs.  All device work is launched on the caller's stream;
// the host synchronises once per cycle to read the bidiagonal coefficients.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/gkb.h"
#include "../../include/gkb_kernels.h"
#include "gkb_internal.h"
#include "kernels.h"
#include "sparse.h"
#include "fused.h"
#include "reorth.h"

namespace {

thread_local std::string g_err;

gkb_status fail(gkb_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define GKB_HIP(call)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(GKB_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));       \
  } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
inline int64_t round64(int64_t x) { return (x + 63) / 64 * 64; }

int basis_bytes(gkb_dtype d) { return d == GKB_F64 ? 8 : 4; }
int elem_bytes(gkb_dtype d) { return d == GKB_F64 ? 8 : (d == GKB_F32 ? 4 : 2); }

// Device workspace layout.  Offsets are 256-byte aligned.
struct Layout {
  int64_t ldm = 0, ldn = 0, ldpart = 0;
  int ldh = 0, kcols = 0;
  size_t Q[2] = {0, 0}, P[2] = {0, 0};
  size_t w = 0, z = 0, part = 0, gsp = 0, normpart = 0;
  size_t qcoef = 0, pcoef = 0, sig = 0, flag = 0, Xs = 0, Ys = 0, rho = 0, q1 = 0;
  size_t Vd = 0, Wr = 0, Gpart = 0, G = 0;  // bfloat16 refinement
  size_t GQ[2] = {0, 0}, y = 0, ypart = 0, csum = 0, Uo = 0, Vo = 0, err[2] = {0, 0}, refresh = 0;  // one-pass
  size_t team = 0, team_bytes = 0;  // the team sweep's mailbox (rows longer than FUSED_NMAX)
  size_t total = 0;
};

Layout make_layout(int64_t m, int64_t n, gkb_dtype dt, int k, bool restart, bool small, bool refine = false,
                   bool dense = true, bool onepass = false) {
  Layout L;
  const size_t tb = onepass ? 8 : basis_bytes(dt);
  const size_t acc = dt == GKB_F64 ? 8 : 4;
  L.ldm = round64(m);
  L.ldn = round64(n);
  L.kcols = k + 1;
  L.ldh = (int)round64(L.kcols);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  L.Q[0] = take((size_t)L.kcols * L.ldm * tb);
  L.P[0] = take((size_t)L.kcols * L.ldn * tb);
  if (restart) {
    L.Q[1] = take((size_t)L.kcols * L.ldm * tb);
    L.P[1] = take((size_t)L.kcols * L.ldn * tb);
  } else {
    L.Q[1] = L.Q[0];
    L.P[1] = L.P[0];
  }
  L.w = take((size_t)L.ldm * 8);
  L.z = take((size_t)L.ldn * 8);
  // gemv_t partial sums: at most GEMV_T_MAX_BLOCKS row blocks, and no more
  // than one per 64 rows (the launch never uses more)
  const int64_t part_rows = dense && !onepass ? std::min<int64_t>(gkb::GEMV_T_MAX_BLOCKS, (m + 63) / 64) : 0;
  L.ldpart = L.ldn;
  L.part = take((size_t)part_rows * L.ldpart * acc);
  // Gram-Schmidt partial dots (two sets of one row per slice, or the column-spread
  // form's chunk partials) and the reduced coefficients
  const int64_t gsr = std::max(gkb::gs_partial_rows(m), gkb::gs_partial_rows(n));
  L.gsp = take((size_t)gsr * L.ldh * 8);
  L.normpart = take((size_t)std::max(gkb::update_blocks(m), gkb::update_blocks(n)) * 8);
  L.qcoef = take((size_t)(L.kcols + 1) * 8);
  L.pcoef = take((size_t)(L.kcols + 1) * 8);
  L.sig = take((size_t)(2 * L.kcols + 8) * 8);
  L.flag = take(4 * sizeof(int));
  if (small) {
    L.Xs = take((size_t)L.kcols * L.kcols * tb);
    L.Ys = take((size_t)L.kcols * L.kcols * tb);
    L.rho = take((size_t)L.ldh * 8);
  }
  L.q1 = take((size_t)L.ldm * 8);
  if (refine) {
    L.Vd = take((size_t)L.ldn * L.kcols * 4);
    L.Wr = take((size_t)L.ldm * L.kcols * 4);
    L.Gpart = take((size_t)gkb::gram_chunks(m) * L.kcols * L.kcols * 8);
    L.G = take((size_t)L.kcols * L.kcols * 8);
  }
  if (onepass) {
    // A^T Q (float64, n x (k + 1), one per Q buffer), A^T A p, its partial
    // sums, the step's coefficient sums, float64 Ritz vectors before narrowing
    L.GQ[0] = take((size_t)L.kcols * L.ldn * 8);
    L.GQ[1] = restart ? take((size_t)L.kcols * L.ldn * 8) : L.GQ[0];
    L.y = take((size_t)L.ldn * 8);
    L.ypart = take((size_t)gkb::fused_blocks(m, n, (int)dt) * L.ldn * 8);
    L.csum = take((size_t)L.ldh * 8);
    L.err[0] = take((size_t)L.ldh * 8);
    L.err[1] = take((size_t)L.ldh * 8);
    L.refresh = take(4 * sizeof(int));
    if (dt != GKB_F64) {   // float64 A: the Ritz vectors go straight to U, V
      L.Uo = take((size_t)L.ldm * L.kcols * 8);
      L.Vo = take((size_t)L.ldn * L.kcols * 8);
    }
    if (gkb::team_form(n, (int)dt)) {
      L.team_bytes = gkb::team_bytes(m, n, (int)dt);
      L.team = take(L.team_bytes);
    }
  }
  L.total = off;
  return L;
}

gkb_status check_matrix(const gkb_matrix* A) {
  if (A == nullptr) return fail(GKB_ERR_INVALID, "A is NULL");
  if (A->m < 1 || A->n < 1) return fail(GKB_ERR_INVALID, "need m >= 1 and n >= 1");
  if (A->lda < A->n) return fail(GKB_ERR_INVALID, "need lda >= n");
  if (A->dtype != GKB_F64 && A->dtype != GKB_F32 && A->dtype != GKB_BF16)
    return fail(GKB_ERR_INVALID, "unknown dtype");
  if (A->data == nullptr) return fail(GKB_ERR_INVALID, "A->data is NULL");
  if (A->m > (int64_t)1 << 31 || A->n > (int64_t)1 << 31)
    return fail(GKB_ERR_INVALID, "m and n must be below 2^31");
  return GKB_OK;
}

// The one-sweep step runs on dense A whose rows the sweep kernels take:
// float32 or bfloat16 rows of n <= 24576 in one workgroup's registers, longer
// ones up to 262144 by teams of workgroups, float64 rows up to 131072 by
// teams; n and lda multiples of the 16-byte group, A 16-byte aligned;
// elsewhere a one_pass request runs the two-product step.
bool one_pass_available(const gkb_matrix* A) {
  return gkb::fused_ok(A->m, A->n, A->lda, A->data, (int)A->dtype);
}

gkb_status check_workspace(void* ws, size_t bytes, size_t need) {
  if (ws == nullptr) return fail(GKB_ERR_WORKSPACE, "workspace is NULL");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
    return fail(GKB_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < need)
    return fail(GKB_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  return GKB_OK;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Device time per phase from HIP events recorded on the solver's stream at each
// phase boundary: the interval between two consecutive events belongs to the
// phase the first one opened.  Completed intervals are read after every host
// synchronisation and their events reused, so a solve holds a few dozen events.
enum Phase { PH_MATVEC = 0, PH_REORTH, PH_SYNC, PH_RITZ, PH_OTHER, PH_COUNT };

#define GKB_MARK_REORTH()                          \
  do {                                             \
    hipError_t m_ = mark(PH_REORTH);               \
    if (m_ != hipSuccess) return m_;               \
  } while (0)

struct PhaseTimer {
  bool on = false;
  std::vector<hipEvent_t> ev, spare;
  std::vector<int> ph;
  double ms[PH_COUNT] = {0, 0, 0, 0, 0};

  hipError_t mark(int phase, hipStream_t st) {
    if (!on || (!ph.empty() && ph.back() == phase)) return hipSuccess;
    hipEvent_t e;
    if (!spare.empty()) {
      e = spare.back();
      spare.pop_back();
    } else {
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
    }
    hipError_t r = hipEventRecord(e, st);
    if (r != hipSuccess) {
      spare.push_back(e);
      return r;
    }
    ev.push_back(e);
    ph.push_back(phase);
    return hipSuccess;
  }
  // Only after the stream has been synchronised: every recorded event is complete.
  hipError_t collect() {
    if (!on || ev.size() < 2) return hipSuccess;
    for (size_t i = 0; i + 1 < ev.size(); ++i) {
      float t = 0.0f;
      hipError_t r = hipEventElapsedTime(&t, ev[i], ev[i + 1]);
      if (r != hipSuccess) return r;
      ms[ph[i]] += t;
      spare.push_back(ev[i]);
    }
    ev.erase(ev.begin(), ev.end() - 1);
    ph.erase(ph.begin(), ph.end() - 1);
    return hipSuccess;
  }
  void fill(gkb_stats* stats) const {
    stats->ms_matvec = ms[PH_MATVEC];
    stats->ms_reorth = ms[PH_REORTH];
    stats->ms_sync = ms[PH_SYNC];
    stats->ms_ritz = ms[PH_RITZ];
    stats->ms_other = ms[PH_OTHER];
  }
  ~PhaseTimer() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : spare) (void)hipEventDestroy(e);
  }
};

// Projected matrix of one cycle, as read back from the device.
struct Proj {
  int nq = 0, np = 0;
  std::vector<double> H;  // nq x np row-major
  double alpha_res = 0.0;
  int breakdown = 0;      // 0 none, 1 beta, 2 alpha
  double sig_seen = 0.0;  // largest accepted coefficient of the cycle
  int64_t matvecs = 0;
};

template <typename TB>
struct Solver {
  gkb::MatrixRef A;
  const gkb::SparseRef* sp = nullptr;   // sparse A: products through the CSR kernels
  hipStream_t st;
  Layout L;
  char* ws;
  int cur = 0;
  double eps = 0.0;
  int relative = 1;
  int nsig = 0;

  TB* Q(int b) { return reinterpret_cast<TB*>(ws + L.Q[b]); }
  TB* P(int b) { return reinterpret_cast<TB*>(ws + L.P[b]); }
  TB* Qc(int j) { return Q(cur) + (int64_t)j * L.ldm; }
  TB* Pc(int j) { return P(cur) + (int64_t)j * L.ldn; }
  double* w() { return reinterpret_cast<double*>(ws + L.w); }
  double* z() { return reinterpret_cast<double*>(ws + L.z); }
  void* part() { return ws + L.part; }
  double* gsp() { return reinterpret_cast<double*>(ws + L.gsp); }
  double* normpart() { return reinterpret_cast<double*>(ws + L.normpart); }
  double* qcoef() { return reinterpret_cast<double*>(ws + L.qcoef); }
  double* pcoef() { return reinterpret_cast<double*>(ws + L.pcoef); }
  double* sig() { return reinterpret_cast<double*>(ws + L.sig); }
  int* flag() { return reinterpret_cast<int*>(ws + L.flag); }
  TB* Xs() { return reinterpret_cast<TB*>(ws + L.Xs); }
  TB* Ys() { return reinterpret_cast<TB*>(ws + L.Ys); }
  double* rho() { return reinterpret_cast<double*>(ws + L.rho); }
  double* q1buf() { return reinterpret_cast<double*>(ws + L.q1); }
  double* GQ(int b) { return reinterpret_cast<double*>(ws + L.GQ[b]); }
  double* ybuf() { return reinterpret_cast<double*>(ws + L.y); }
  double* ypart() { return reinterpret_cast<double*>(ws + L.ypart); }
  double* csum() { return reinterpret_cast<double*>(ws + L.csum); }
  double* err(int b) { return reinterpret_cast<double*>(ws + L.err[b]); }
  int* refresh() { return reinterpret_cast<int*>(ws + L.refresh); }
  void* team() { return L.team_bytes ? ws + L.team : nullptr; }
  double eps0() const { return std::ldexp(1.0, -52) * std::sqrt((double)(A.m + A.n)); }
  bool onepass = false;  // dense float32 A, float64 bases, one sweep of A per step
  PhaseTimer pt;         // per-phase device time (opt.phase_timing)
  int nparts = 1;        // norm partials left in normpart by the last cgs2
  int64_t a_passes = 0;  // full passes over A launched (a skipped direct sweep not counted)

  hipError_t mark(int phase) { return pt.mark(phase, st); }
  // algorithmic bytes of one pass over A: every element once (dense), every
  // stored value and its column index once (sparse)
  double bytes_per_pass() const {
    if (sp) return (double)sp->nnz * (sizeof(float) + sizeof(int32_t));
    return (double)A.m * (double)A.n * elem_bytes((gkb_dtype)A.dtype);
  }

  // w = A p - coef[cidx] qprev (dense or sparse A)
  hipError_t prod_n(const TB* p, const TB* qprev, const double* coef, int cidx, double* out) {
    if constexpr (std::is_same<TB, float>::value) {
      if (sp) return gkb::launch_spmv(sp->fwd, p, qprev, coef, cidx, out, flag(), st);
    }
    return gkb::launch_gemv_n<TB>(A, p, qprev, coef, cidx, out, flag(), st);
  }

  // Two classical Gram-Schmidt passes of x against V[:, 0..t), leaving the
  // partial sums of ||x||^2 in normpart (three launches, reorth.h).  If acc is
  // given, acc[0..t) receives the sum of the coefficients of both passes.
  hipError_t cgs2(const TB* V, int64_t ldv, int t, int64_t len, double* x, double* acc = nullptr,
                  int pre_kind = gkb::GS_PRE_NONE, const gkb::GsPreArgs& pre = gkb::GsPreArgs()) {
    return gkb::launch_gs2<TB>(V, ldv, t, len, x, gsp(), L.ldh, normpart(), acc, pre_kind, pre, flag(), st,
                               &nparts);
  }

  // z = A^T q - coef[cidx] pprev, then CGS2 of z against P[:, 0..t).  Dense A:
  // the row-block partial sums of A^T q are added by the first Gram-Schmidt
  // launch (no separate reduction launch).
  hipError_t prod_t_cgs2(const TB* q, const TB* pprev, const double* coef, int cidx, int t) {
    if constexpr (std::is_same<TB, float>::value) {
      if (sp) {
        hipError_t e = gkb::launch_spmv(sp->tr, q, pprev, coef, cidx, z(), flag(), st);
        if (e != hipSuccess) return e;
        GKB_MARK_REORTH();
        return cgs2(P(cur), L.ldn, t, A.n, z());
      }
    }
    hipError_t e = gkb::launch_gemv_t<TB>(A, q, nullptr, nullptr, 0, nullptr, part(), L.ldpart, flag(), st);
    if (e != hipSuccess) return e;
    GKB_MARK_REORTH();
    gkb::GsPreArgs pre;
    pre.part = part();
    pre.ldpart = L.ldpart;
    pre.nparts = gkb::gemv_t_shape(A.m, A.n, elem_bytes((gkb_dtype)A.dtype)).nb;
    pre.part_f64 = A.dtype == GKB_F64 ? 1 : 0;
    pre.prev = pprev;
    pre.coef = coef;
    pre.cidx = cidx;
    return cgs2(P(cur), L.ldn, t, A.n, z(), nullptr, gkb::GS_PRE_TSUM, pre);
  }

  // The first left vector after a thick restart: x -= Q~ rho (the kept Ritz
  // vectors' couplings, rho = alpha_res X[last, :l]), then CGS2 against
  // Q[:, 0..t); the rho update is the first Gram-Schmidt launch's pre-step.
  hipError_t cgs2_after_restart(int t, int l, int64_t len, double* x, double* acc) {
    gkb::GsPreArgs pre;
    pre.rho = rho();
    pre.l = l;
    return cgs2(Q(cur), L.ldm, t, len, x, acc, gkb::GS_PRE_RHO, pre);
  }

  hipError_t normalize(const double* x, int64_t len, TB* out, double* coef_out, int track, int code,
                       int index, bool test) {
    hipError_t e = gkb::launch_normalize<TB>(x, len, normpart(), nparts, out, coef_out,
                                             sig() + nsig, sig() + nsig + 1, test ? eps : 0.0, relative,
                                             track, flag(), code, index, st);
    ++nsig;
    return e;
  }

  // Read flag and coefficients after a cycle (one host synchronisation).
  gkb_status read_back(int ncoef, std::vector<double>& qc, std::vector<double>& pc, int* fl) {
    qc.assign(ncoef, 0.0);
    pc.assign(ncoef, 0.0);
    GKB_HIP(mark(PH_SYNC));
    GKB_HIP(hipMemcpyAsync(qc.data(), qcoef(), ncoef * sizeof(double), hipMemcpyDeviceToHost, st));
    GKB_HIP(hipMemcpyAsync(pc.data(), pcoef(), ncoef * sizeof(double), hipMemcpyDeviceToHost, st));
    GKB_HIP(hipMemcpyAsync(fl, flag(), 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    GKB_HIP(hipStreamSynchronize(st));
    GKB_HIP(pt.collect());
    return GKB_OK;
  }

  // Start: Q[:,0] = q/||q||, z = A^T q_1, P[:,0] = z/||z||.
  gkb_status start(const double* q1) {
    nsig = 0;
    GKB_HIP(mark(PH_OTHER));
    GKB_HIP(gkb::launch_init_cycle(flag(), sig(), 0.0, st));
    GKB_HIP(hipMemcpyAsync(w(), q1, (size_t)A.m * sizeof(double), hipMemcpyDeviceToDevice, st));
    GKB_HIP(cgs2(Q(cur), L.ldm, 0, A.m, w()));  // norm partials only
    GKB_HIP(normalize(w(), A.m, Qc(0), qcoef(), 0, 1, 0, false));
    GKB_HIP(mark(PH_MATVEC));
    ++a_passes;
    if (onepass) {
      // z = A^T q_1 with float64 sums, kept as the first column of A^T Q
      if constexpr (std::is_same<TB, double>::value) {
        // the team sweep's mailbox starts each solve zeroed
        if (team() != nullptr) GKB_HIP(gkb::launch_team_reset(team(), A.m, A.n, A.dtype, st));
        GKB_HIP(gkb::launch_gemv_fused<double>(fA(), A.dtype, A.lda, A.m, A.n, nullptr, Qc(0), nullptr, z(), ypart(), L.ldn,
                                               flag(), st, nullptr, nullptr, nullptr, team()));
        GKB_HIP(gkb::launch_copy_vec<double>(z(), A.n, GQ(cur), st));
        GKB_HIP(hipMemsetAsync(refresh(), 0, 4 * sizeof(int), st));
      }
      GKB_HIP(mark(PH_REORTH));
      GKB_HIP(cgs2(P(cur), L.ldn, 0, A.n, z()));
    } else {
      GKB_HIP(prod_t_cgs2(Qc(0), nullptr, nullptr, 0, 0));
    }
    GKB_HIP(mark(PH_REORTH));
    GKB_HIP(normalize(z(), A.n, Pc(0), pcoef(), 1, 2, 0, false));
    if (onepass) GKB_HIP(gkb::launch_err_set(err(cur), 0, sig() + nsig, eps0(), flag(), st));
    return GKB_OK;
  }

  // One Bidiag 1 step of the first cycle, s = 0-based step:
  //   w = A p_s - alpha_s q_s -> CGS2 vs Q[0..s] -> q_{s+1}, beta
  //   z = A^T q_{s+1} - beta p_s -> CGS2 vs P[0..s] -> p_{s+1}, alpha
  gkb_status first_step(int s) {
    GKB_HIP(mark(PH_MATVEC));
    GKB_HIP(prod_n(Pc(s), Qc(s), pcoef(), s, w()));
    GKB_HIP(mark(PH_REORTH));
    GKB_HIP(cgs2(Q(cur), L.ldm, s + 1, A.m, w()));
    GKB_HIP(normalize(w(), A.m, Qc(s + 1), qcoef() + s + 1, 1, 1, s + 1, true));
    GKB_HIP(mark(PH_MATVEC));
    GKB_HIP(prod_t_cgs2(Qc(s + 1), Pc(s), qcoef(), s + 1, s + 1));
    GKB_HIP(normalize(z(), A.n, Pc(s + 1), pcoef() + s + 1, 1, 2, s + 1, true));
    a_passes += 2;
    return GKB_OK;
  }

  // A restarted cycle's step j (two products): w = A p_j - (j == l ? Q~ rho :
  // alpha_j q_{j-1}), CGS2 vs Q[0..j), q_j; z = A^T q_j - beta p_j, CGS2 vs P[0..j], p_{j+1}.
  gkb_status restart_step(int j, int l) {
    GKB_HIP(mark(PH_MATVEC));
    GKB_HIP(prod_n(Pc(j), j == l ? nullptr : Qc(j - 1), pcoef(), j, w()));
    GKB_HIP(mark(PH_REORTH));
    GKB_HIP(cgs2_after_restart(j, l, A.m, w(), nullptr));
    GKB_HIP(normalize(w(), A.m, Qc(j), qcoef() + j, 1, 1, j, true));
    GKB_HIP(mark(PH_MATVEC));
    GKB_HIP(prod_t_cgs2(Qc(j), Pc(j), qcoef(), j, j + 1));
    GKB_HIP(normalize(z(), A.n, Pc(j + 1), pcoef() + j + 1, 1, 2, j + 1, true));
    a_passes += 2;
    return GKB_OK;
  }

  const void* fA() const { return A.data; }

  // The same step with one sweep of A (float32 A, float64 bases).  From
  // p = P[:, pi]: w = A p and y = A^T w in one pass; w loses the recurrence
  // term (alpha_pi q_qp, or Q[:, 0..nqc) rho after a restart) and two
  // Gram-Schmidt passes against Q[:, 0..nqc), which altogether subtract
  // Q[:, 0..nqc) c.  Then beta q_qn = w, and because every column of Q has
  // its A^T image in GQ, A^T q_qn = (y - GQ[:, 0..nqc) c) / beta (eq. (2.2)),
  // which becomes GQ[:, qn]; the p side then continues as in the two-pass step.
  // An error in a stored column reaches the next one multiplied by
  // alpha / beta, so each column carries an error bound; one whose bound
  // passes ONEPASS_TAU times the largest coefficient is recomputed by a
  // direct sweep A^T q_qn instead (skipped on the device otherwise).
  gkb_status onepass_step(int pi, int qp, int nqc, int qn, bool use_rho) {
    if constexpr (std::is_same<TB, double>::value) {
      const int nb = gkb::fused_blocks(A.m, A.n, A.dtype);
      // w = A p - alpha q_qp in the sweep itself (after a restart, Q~ rho by an update)
      GKB_HIP(mark(PH_MATVEC));
      GKB_HIP(gkb::launch_gemv_fused<double>(fA(), A.dtype, A.lda, A.m, A.n, Pc(pi), nullptr, w(), nullptr, ypart(),
                                             L.ldn, flag(), st, nullptr, use_rho ? nullptr : Qc(qp),
                                             use_rho ? nullptr : pcoef() + pi, team()));
      ++a_passes;
      GKB_HIP(mark(PH_REORTH));
      if (use_rho)
        GKB_HIP(cgs2_after_restart(nqc, nqc, A.m, w(), csum()));
      else
        GKB_HIP(cgs2(Q(cur), L.ldm, nqc, A.m, w(), csum()));
      // the normalisation of q_qn and the recovery of A^T q_qn in one launch
      GKB_HIP(mark(PH_MATVEC));
      gkb::NormArgs na;
      na.x = w();
      na.len = A.m;
      na.normpart = normpart();
      na.nparts = nparts;
      na.out = Qc(qn);
      na.coef_out = qcoef() + qn;
      na.sig_in = sig() + nsig;
      na.sig_out = sig() + nsig + 1;
      na.eps = eps;
      na.relative = relative;
      na.code = 1;
      na.index = qn;
      ++nsig;
      GKB_HIP(gkb::launch_onepass_recover(ypart(), nb, L.ldn, GQ(cur), L.ldn, nqc, csum(),
                                          use_rho ? rho() : pcoef() + pi, use_rho ? 0 : qp, use_rho ? nqc : 1,
                                          nullptr, qn, Pc(pi), z(), A.n, err(cur), nullptr, eps0(),
                                          gkb::ONEPASS_TAU, refresh(), flag(), st, &na));
      GKB_HIP(gkb::launch_gemv_fused<double>(fA(), A.dtype, A.lda, A.m, A.n, nullptr, Qc(qn), nullptr, nullptr, ypart(),
                                             L.ldn, flag(), st, refresh(), nullptr, nullptr, team()));
      // if the column was recomputed: A^T q_qn from the direct sweep's partial
      // sums replaces the recovered one (G[:, qn] and z), as the first
      // Gram-Schmidt launch's pre-step
      GKB_HIP(mark(PH_REORTH));
      gkb::GsPreArgs fix;
      fix.part = ypart();
      fix.ldpart = L.ldn;
      fix.nparts = nb;
      fix.part_f64 = 1;
      fix.prev = Pc(pi);
      fix.coef = qcoef() + qn;
      fix.cidx = 0;
      fix.run_if = refresh();
      fix.gcol = GQ(cur) + (int64_t)qn * L.ldn;
      GKB_HIP(cgs2(P(cur), L.ldn, pi + 1, A.n, z(), nullptr, gkb::GS_PRE_FIX, fix));
      GKB_HIP(normalize(z(), A.n, Pc(pi + 1), pcoef() + pi + 1, 1, 2, pi + 1, true));
      return GKB_OK;
    } else {
      return fail(GKB_ERR_INVALID, "the one-pass step runs on float64 bases");
    }
  }

};

struct Ritz {
  int kk = 0;
  std::vector<double> s, X, Y;  // X nq x kk, Y np x kk row-major
};

gkb_status host_svd(const Proj& pr, Ritz& rz) {
  rz.kk = std::min(pr.nq, pr.np);
  rz.s.assign(std::max(rz.kk, 1), 0.0);
  rz.X.assign((size_t)pr.nq * std::max(rz.kk, 1), 0.0);
  rz.Y.assign((size_t)std::max(pr.np, 1) * std::max(rz.kk, 1), 0.0);
  if (rz.kk == 0) return GKB_OK;
  if (!gkb::dense_svd(pr.nq, pr.np, pr.H.data(), rz.s.data(), rz.X.data(), rz.Y.data()))
    return fail(GKB_ERR_NUMERIC, "small SVD did not converge");
  return GKB_OK;
}

template <typename TB>
void to_colmajor(const std::vector<double>& M, int rows, int ldrow, int cols, std::vector<TB>& out) {
  out.assign((size_t)rows * std::max(cols, 1), TB(0));
  for (int c = 0; c < cols; ++c)
    for (int i = 0; i < rows; ++i) out[(size_t)c * rows + i] = (TB)M[(size_t)i * ldrow + c];
}

// Convergence test on a projected matrix (same rule as the oracle): the r
// largest Ritz values above the breakdown threshold must all satisfy
// alpha_res |X[last, i]| <= tol * sigma_1.
struct ConvTest {
  bool converged = false;
  int r_eff = 0, nconv = 0;
  std::vector<double> res;
};

void convergence(const Proj& pr, const Ritz& rz, int r, double tol, double thr, ConvTest& ct) {
  int avail = 0;
  for (int i = 0; i < rz.kk; ++i)
    if (rz.s[i] > thr) ++avail;
  ct.r_eff = std::min(r, avail);
  ct.res.assign(std::max(rz.kk, 1), 0.0);
  for (int i = 0; i < rz.kk; ++i) ct.res[i] = pr.alpha_res * std::fabs(rz.X[(size_t)(pr.nq - 1) * rz.kk + i]);
  ct.nconv = 0;
  const double s0 = rz.kk ? rz.s[0] : 0.0;
  for (int i = 0; i < ct.r_eff; ++i)
    if (ct.res[i] <= tol * s0) ++ct.nconv;
  ct.converged = ct.r_eff == r && ct.nconv == r;
}

// Screening of an in-cycle test on the first cycle's lower bidiagonal
// (diagonal pc[0..np), subdiagonal qc[1..np], residual coefficient pc[np]):
// true only if the test would clearly fail -- the r largest singular values
// above the breakdown threshold do not number r, or one of them has a
// residual estimate above 1.01 tol sigma_1 -- so that the dense SVD, which
// makes every accepting decision, would reject it as well.  Not used when two
// of the top r + 1 values are within 1e-8 of each other (the individual last
// components of a cluster are not unique).
bool screen_fails(int np, const std::vector<double>& pc, const std::vector<double>& qc, int r, double tol,
                  double thr_fixed, double sig_est, bool relative, double eps) {
  std::vector<double> alpha(pc.begin(), pc.begin() + np), beta(qc.begin() + 1, qc.begin() + np + 1);
  std::vector<double> sv(np), last(np);
  if (!gkb::bidiag_sv_lastrow(np, alpha.data(), beta.data(), sv.data(), last.data())) return false;
  double seen = sig_est;
  for (int j = 0; j < np; ++j) seen = std::max({seen, pc[j], qc[j + 1]});
  seen = std::max(seen, pc[np]);
  const double thr = relative ? eps * seen : thr_fixed;
  const int top = std::min(np, r + 1);
  for (int i = 0; i + 1 < top; ++i)
    if (sv[i] - sv[i + 1] <= 1e-8 * sv[0]) return false;
  int avail = 0;
  for (int i = 0; i < np; ++i)
    if (sv[i] > thr * (1.0 + 1e-9)) ++avail;
  int maybe = 0;
  for (int i = 0; i < np; ++i)
    if (sv[i] > thr * (1.0 - 1e-9)) ++maybe;
  if (maybe < r) return true;          // fewer than r values can pass the threshold
  if (avail < r) return false;         // a value at the threshold: let the dense SVD decide
  for (int i = 0; i < r; ++i)
    if (pc[np] * std::fabs(last[i]) > 1.01 * tol * sv[0]) return true;
  return false;
}

// Restart data carried into a restarted cycle.
struct RestartIn {
  int l = 0;
  std::vector<double> s, rho;
};

// Projected matrix after `np` right vectors of a cycle (no breakdown), or at a
// breakdown recorded in fl.  first: lower bidiagonal; else restarted form.
gkb_status assemble(bool first, int np_now, const RestartIn& rs, const std::vector<double>& qc,
                    const std::vector<double>& pc, const int* fl, Proj& pr) {
  const int code = fl[0], idx = fl[1];
  if (code == 3) return fail(GKB_ERR_NUMERIC, "NaN or Inf in a norm (non-finite input?)");
  if (code == 4)
    return fail(GKB_ERR_TIMEOUT, "one-sweep step: a workgroup of a team waited too long for the others "
                                 "(the device was not free for the whole grid)");
  if (first && code == 1 && idx == 0) return fail(GKB_ERR_INVALID, "start vector is zero");
  int nq, np;
  const int l = rs.l;
  if (first) {
    if (code == 0) {
      np = np_now;
      nq = np + 1;
      pr.matvecs = 1 + 2 * (int64_t)np;
    } else if (code == 1) {
      nq = np = idx;
      pr.matvecs = 2 * (int64_t)idx;
    } else {
      np = idx;
      nq = idx == 0 ? 1 : idx + 1;
      pr.matvecs = 1 + 2 * (int64_t)idx;
    }
  } else {
    if (code == 0) {
      nq = np = np_now;
      pr.matvecs = 2 * (int64_t)(np_now - l);
    } else if (code == 1) {
      nq = idx;
      np = idx + 1;
      pr.matvecs = 2 * (int64_t)(idx - l) + 1;
    } else {
      nq = np = idx;
      pr.matvecs = 2 * (int64_t)(idx - l);
    }
  }
  pr.nq = nq;
  pr.np = np;
  pr.breakdown = code;
  pr.H.assign((size_t)nq * std::max(np, 1), 0.0);
  double seen = 0.0;
  if (first) {
    for (int j = 0; j < np; ++j) {
      pr.H[(size_t)j * np + j] = pc[j];
      seen = std::max(seen, pc[j]);
      if (j + 1 < nq) {
        pr.H[(size_t)(j + 1) * np + j] = qc[j + 1];
        seen = std::max(seen, qc[j + 1]);
      }
    }
  } else {
    for (int i = 0; i < l && i < nq; ++i) {
      if (i < np) pr.H[(size_t)i * np + i] = rs.s[i];
      if (l < np) pr.H[(size_t)i * np + l] = rs.rho[i];
    }
    for (int j = l; j < nq; ++j) {
      pr.H[(size_t)j * np + j] = qc[j];
      seen = std::max(seen, qc[j]);
      if (j + 1 < np) {
        pr.H[(size_t)j * np + j + 1] = pc[j + 1];
        seen = std::max(seen, pc[j + 1]);
      }
    }
  }
  pr.alpha_res = code == 0 ? pc[np] : 0.0;
  if (code == 0) seen = std::max(seen, pc[np]);
  pr.sig_seen = seen;
  return GKB_OK;
}

// Cholesky G = R^T R (R upper, row-major d x d).  False if G is not
// numerically positive definite.
bool cholesky_upper(int d, const std::vector<double>& G, std::vector<double>& R) {
  R.assign((size_t)d * d, 0.0);
  for (int j = 0; j < d; ++j) {
    double s = G[(size_t)j * d + j];
    for (int k = 0; k < j; ++k) s -= R[(size_t)k * d + j] * R[(size_t)k * d + j];
    if (!(s > 0.0)) return false;
    const double rjj = std::sqrt(s);
    R[(size_t)j * d + j] = rjj;
    for (int i = j + 1; i < d; ++i) {
      double t = G[(size_t)j * d + i];
      for (int k = 0; k < j; ++k) t -= R[(size_t)k * d + j] * R[(size_t)k * d + i];
      R[(size_t)j * d + i] = t / rjj;
    }
  }
  return true;
}

// Rayleigh-Ritz refinement on the float32 matrix (eq. (5) for A^T A on the
// subspace of the top d Ritz vectors V_d found with the bfloat16 matrix):
//   W = A32 V_d,  W^T W = R^T R (Cholesky, float64),  R = Xr diag(s) Yr^T,
//   sigma = s,  V = V_d Yr,  U = W R^{-1} Xr (= A32 V / sigma).
template <typename TB>
gkb_status refine_bf16(Solver<TB>& S, const gkb_matrix* Am, const Proj& pr, const Ritz& rz, int r, int d,
                       double* sigma, float* U, float* V, int* refined) {
  hipStream_t st = S.st;
  float* Vd = reinterpret_cast<float*>(S.ws + S.L.Vd);
  float* W = reinterpret_cast<float*>(S.ws + S.L.Wr);
  double* Gpart = reinterpret_cast<double*>(S.ws + S.L.Gpart);
  double* Gd = reinterpret_cast<double*>(S.ws + S.L.G);
  const int64_t m = Am->m, n = Am->n;
  // V_d = P Y_d in the basis precision, then float32 for the refinement products
  std::vector<TB> Yh;
  to_colmajor<TB>(rz.Y, pr.np, rz.kk, d, Yh);
  GKB_HIP(hipMemcpyAsync(S.Ys(), Yh.data(), Yh.size() * sizeof(TB), hipMemcpyHostToDevice, st));
  if constexpr (std::is_same<TB, float>::value) {
    GKB_HIP(gkb::launch_gemm_tall<float>(S.P(S.cur), S.L.ldn, n, pr.np, S.Ys(), pr.np, d, Vd, S.L.ldn, st));
  } else {
    double* Vo = reinterpret_cast<double*>(S.ws + S.L.Vo);
    GKB_HIP(gkb::launch_gemm_tall<TB>(S.P(S.cur), S.L.ldn, n, pr.np, S.Ys(), pr.np, d, Vo, S.L.ldn, st));
    GKB_HIP(gkb::launch_narrow(Vo, S.L.ldn * d, Vd, st));   // rows n..ldn of each column are never read
  }
  GKB_HIP(gkb::launch_gemm_rm(Am->refine_f32, Am->lda_refine, m, n, Vd, S.L.ldn, d, W, S.L.ldm, st));
  GKB_HIP(gkb::launch_gram(W, S.L.ldm, m, d, Gpart, Gd, st));
  std::vector<double> G((size_t)d * d), R;
  GKB_HIP(hipMemcpyAsync(G.data(), Gd, G.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  GKB_HIP(hipStreamSynchronize(st));
  for (double g : G)
    if (!std::isfinite(g)) return fail(GKB_ERR_NUMERIC, "non-finite Gram matrix in the refinement");
  if (!cholesky_upper(d, G, R)) {
    *refined = -1;  // subspace numerically rank deficient: keep the unrefined triplets
    return GKB_OK;
  }
  std::vector<double> sr(d), Xr((size_t)d * d), Yr((size_t)d * d);
  if (!gkb::dense_svd(d, d, R.data(), sr.data(), Xr.data(), Yr.data()))
    return fail(GKB_ERR_NUMERIC, "refinement SVD did not converge");
  // Mr = R^{-1} Xr[:, :r] by back substitution (R upper triangular)
  std::vector<double> Mr((size_t)d * r);
  for (int c = 0; c < r; ++c)
    for (int i = d - 1; i >= 0; --i) {
      double t = Xr[(size_t)i * d + c];
      for (int k2 = i + 1; k2 < d; ++k2) t -= R[(size_t)i * d + k2] * Mr[(size_t)k2 * r + c];
      Mr[(size_t)i * r + c] = t / R[(size_t)i * d + i];
    }
  std::vector<float> Mh, Yrh;
  to_colmajor<float>(Mr, d, r, r, Mh);
  to_colmajor<float>(Yr, d, d, r, Yrh);
  GKB_HIP(hipMemcpyAsync(S.Xs(), Mh.data(), Mh.size() * sizeof(float), hipMemcpyHostToDevice, st));
  GKB_HIP(hipMemcpyAsync(S.Ys(), Yrh.data(), Yrh.size() * sizeof(float), hipMemcpyHostToDevice, st));
  GKB_HIP(gkb::launch_gemm_tall<float>(Vd, S.L.ldn, n, d, reinterpret_cast<const float*>(S.Ys()), d, r,
                                       V, n, st));
  GKB_HIP(gkb::launch_gemm_tall<float>(W, S.L.ldm, m, d, reinterpret_cast<const float*>(S.Xs()), d, r,
                                       U, m, st));
  GKB_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < r; ++i) sigma[i] = sr[i];
  *refined = 1;
  return GKB_OK;
}


// TO: type of U and V (TB, or float for the one-pass step on float64 bases)
// Device work between two host synchronisations of a solve -- the Golub-Kahan
// steps of one stretch of a cycle -- captured once as a HIP graph and replayed
// by later solves with the same matrix, workspace and options (a plan).  A
// stretch is keyed by (first cycle or not, first step, end step, current basis
// copy); replaying it advances the host-side counters the launches would have
// advanced.
struct SegmentGraphs {
  struct Seg {
    hipGraphExec_t exec = nullptr;
    int64_t passes = 0;
    int nsig = 0;
    int nparts = 1;
  };
  hipStream_t capture = nullptr;  // stream the stretches are captured on
  std::map<std::tuple<int, int, int, int>, Seg> segs;
  ~SegmentGraphs() {
    for (auto& kv : segs)
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (capture) (void)hipStreamDestroy(capture);
  }
};

// Launch steps [j0, j1) through the cache: replay the captured graph, or
// capture the launches on the cache's stream, instantiate, then replay.
template <typename TB, typename F>
gkb_status run_segment(Solver<TB>& S, SegmentGraphs& G, int first, int j0, int j1, F&& steps) {
  // the bases are double-buffered across restarts: the launches also depend on
  // which copy is current
  const auto key = std::make_tuple(first, j0, j1, S.cur);
  auto it = G.segs.find(key);
  if (it == G.segs.end()) {
    SegmentGraphs::Seg seg;
    const int64_t p0 = S.a_passes;
    const int n0 = S.nsig;
    hipStream_t user = S.st;
    S.st = G.capture;
    GKB_HIP(hipStreamBeginCapture(G.capture, hipStreamCaptureModeThreadLocal));
    const gkb_status rc = steps(j0, j1);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(G.capture, &graph);
    S.st = user;
    if (rc != GKB_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    GKB_HIP(e);
    const hipError_t ei = hipGraphInstantiate(&seg.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    GKB_HIP(ei);
    seg.passes = S.a_passes - p0;
    seg.nsig = S.nsig - n0;
    seg.nparts = S.nparts;
    S.a_passes = p0;
    S.nsig = n0;
    it = G.segs.emplace(key, seg).first;
  }
  GKB_HIP(hipGraphLaunch(it->second.exec, S.st));
  S.a_passes += it->second.passes;
  S.nsig += it->second.nsig;
  S.nparts = it->second.nparts;
  return GKB_OK;
}

// ONEPASS: the one-sweep step (float64 bases; U, V float32 for float32 and
// bfloat16 A, float64 for float64 A)
template <typename TB, typename TO = TB, bool ONEPASS = !std::is_same<TB, TO>::value>
gkb_status run_partial_svd(const gkb_matrix* Am, int r, int k, double tol, int max_restarts,
                           const gkb_options& opt, void* workspace, double* sigma, TO* U, TO* V,
                           gkb_stats* stats, hipStream_t st, const gkb::SparseRef* sp = nullptr,
                           SegmentGraphs* graphs = nullptr) {
  constexpr bool onepass = ONEPASS;
  const double t0 = now_ms();
  double ms_host = 0.0;
  Solver<TB> S;
  S.A = {Am->data, Am->m, Am->n, Am->lda, (int)Am->dtype};
  S.sp = sp;
  S.st = st;
  const int l = opt.keep ? opt.keep : std::min(r + (k - r) / 2, k - 1);
  if (k == r) max_restarts = 0;
  const int every = opt.check_every > 0 ? opt.check_every : 0;
  const bool refine = Am->dtype == GKB_BF16 && Am->refine_f32 != nullptr;
  S.L = make_layout(Am->m, Am->n, Am->dtype, k, k > r, true, refine, sp == nullptr, onepass);
  S.ws = reinterpret_cast<char*>(workspace);
  S.onepass = onepass;
  S.eps = opt.eps_break > 0 ? opt.eps_break : (Am->dtype == GKB_F64 ? 1e-12 : 1e-6);
  S.relative = opt.eps_relative ? 1 : 0;
  S.pt.on = opt.phase_timing != 0;
  const double* q1 = opt.q1;
  GKB_HIP(S.mark(PH_OTHER));
  if (q1 == nullptr) {
    GKB_HIP(gkb::launch_philox_start(S.q1buf(), Am->m, opt.seed, st));
    q1 = S.q1buf();
  }
  gkb_status rc = S.start(q1);
  if (rc != GKB_OK) return rc;

  double sig_est = 0.0;  // largest accepted coefficient / Ritz value so far
  int64_t matvecs = 0;
  int restarts = 0, checks = 0;
  Proj pr;
  Ritz rz;
  ConvTest ct;
  RestartIn rs;
  std::vector<double> qc, pc;
  int fl[2] = {0, 0};
  bool first = true;
  while (true) {
    // ---- one cycle: steps jstart..k-1, with optional in-cycle checks
    const int jstart = first ? 0 : l;
    bool early = false;
    // steps j0 .. j1-1 of this cycle (device work only)
    auto steps = [&](int j0, int j1) -> gkb_status {
      for (int j = j0; j < j1; ++j) {
        gkb_status e;
        if (onepass)
          e = first ? S.onepass_step(j, j, j + 1, j + 1, false) : S.onepass_step(j, j - 1, j, j, j == l);
        else if (first)
          e = S.first_step(j);
        else
          e = S.restart_step(j, l);
        if (e != GKB_OK) return e;
      }
      return GKB_OK;
    };
    for (int j = jstart; j < k;) {
      // the stretch up to the next in-cycle test (or the cycle end)
      int jend = k;
      if (every > 0)
        for (int np = j + 1; np < k; ++np)
          if (np >= r && np % every == 0) {
            jend = np;
            break;
          }
      rc = graphs ? run_segment(S, *graphs, first ? 1 : 0, j, jend, steps) : steps(j, jend);
      if (rc != GKB_OK) return rc;
      j = jend;
      const int np_now = j;
      if (every > 0 && np_now < k && np_now >= r && np_now % every == 0) {
        rc = S.read_back(k + 2, qc, pc, fl);
        if (rc != GKB_OK) return rc;
        if (fl[0] != 0) break;  // breakdown: assembled below
        if (first) {
          // screening: singular values and the last row of X alone (O(k^2));
          // a clearly failing test skips the dense SVD, which decides otherwise
          const double th0 = now_ms();
          const bool fails = screen_fails(np_now, pc, qc, r, tol, S.relative ? S.eps * sig_est : S.eps, sig_est,
                                          S.relative != 0, S.eps);
          ms_host += now_ms() - th0;
          if (fails) {
            ++checks;
            continue;
          }
        }
        Proj part;
        rc = assemble(first, np_now, rs, qc, pc, fl, part);
        if (rc != GKB_OK) return rc;
        const double th0 = now_ms();
        rc = host_svd(part, rz);
        ms_host += now_ms() - th0;
        if (rc != GKB_OK) return rc;
        ++checks;
        const double se = std::max(sig_est, part.sig_seen);
        convergence(part, rz, r, tol, S.relative ? S.eps * se : S.eps, ct);
        if (ct.converged) {
          pr = part;
          early = true;
          break;
        }
      }
    }
    if (!early) {
      rc = S.read_back(k + 2, qc, pc, fl);
      if (rc != GKB_OK) return rc;
      rc = assemble(first, k, rs, qc, pc, fl, pr);
      if (rc != GKB_OK) return rc;
      const double th0 = now_ms();
      rc = host_svd(pr, rz);
      ms_host += now_ms() - th0;
      if (rc != GKB_OK) return rc;
    }
    sig_est = std::max(sig_est, pr.sig_seen);
    matvecs += pr.matvecs;
    convergence(pr, rz, r, tol, S.relative ? S.eps * sig_est : S.eps, ct);
    const bool done = pr.breakdown != 0 || ct.converged;
    if (done || restarts >= max_restarts) break;
    // ---- thick restart: P~ = P Y_l, Q~ = Q X_l, p_{l+1} = p_res, rho = alpha_res X[last, :l]
    sig_est = std::max(sig_est, rz.s[0]);
    std::vector<TB> Xh, Yh;
    to_colmajor<TB>(rz.X, pr.nq, rz.kk, l, Xh);
    to_colmajor<TB>(rz.Y, pr.np, rz.kk, l, Yh);
    rs.l = l;
    rs.s.assign(rz.s.begin(), rz.s.begin() + l);
    rs.rho.assign(l, 0.0);
    for (int i = 0; i < l; ++i) rs.rho[i] = pr.alpha_res * rz.X[(size_t)(pr.nq - 1) * rz.kk + i];
    GKB_HIP(hipMemcpyAsync(S.Xs(), Xh.data(), Xh.size() * sizeof(TB), hipMemcpyHostToDevice, st));
    GKB_HIP(hipMemcpyAsync(S.Ys(), Yh.data(), Yh.size() * sizeof(TB), hipMemcpyHostToDevice, st));
    GKB_HIP(hipMemcpyAsync(S.rho(), rs.rho.data(), l * sizeof(double), hipMemcpyHostToDevice, st));
    GKB_HIP(S.mark(PH_RITZ));
    const int nb = 1 - S.cur;
    GKB_HIP(gkb::launch_gemm_tall<TB>(S.P(S.cur), S.L.ldn, Am->n, pr.np, S.Ys(), pr.np, l, S.P(nb), S.L.ldn,
                                      st));
    GKB_HIP(gkb::launch_gemm_tall<TB>(S.Q(S.cur), S.L.ldm, Am->m, pr.nq, S.Xs(), pr.nq, l, S.Q(nb), S.L.ldm,
                                      st));
    GKB_HIP(gkb::launch_copy_vec<TB>(S.P(S.cur) + (int64_t)pr.np * S.L.ldn, Am->n,
                                     S.P(nb) + (int64_t)l * S.L.ldn, st));
    if constexpr (onepass) {  // A^T Q~ = (A^T Q) X_l, with the error bounds of its columns
      GKB_HIP(gkb::launch_gemm_tall<TB>(S.GQ(S.cur), S.L.ldn, Am->n, pr.nq, S.Xs(), pr.nq, l, S.GQ(nb), S.L.ldn,
                                        st));
      GKB_HIP(gkb::launch_err_restart(S.err(S.cur), pr.nq, S.err(nb), l, st));
    }
    S.cur = nb;
    S.nsig = 0;
    GKB_HIP(S.mark(PH_OTHER));
    GKB_HIP(gkb::launch_init_cycle(S.flag(), S.sig(), sig_est, st));
    ++restarts;
    first = false;
  }
  // ---- Ritz vectors: V = P Y_r, U = Q X_r
  GKB_HIP(S.mark(PH_RITZ));
  const int r_eff = ct.r_eff;
  for (int i = 0; i < r; ++i) sigma[i] = i < r_eff ? rz.s[i] : 0.0;
  if (r_eff < r) {  // columns past the returned triplets are zero
    GKB_HIP(hipMemsetAsync(U + (size_t)r_eff * Am->m, 0, (size_t)(r - r_eff) * Am->m * sizeof(TO), st));
    GKB_HIP(hipMemsetAsync(V + (size_t)r_eff * Am->n, 0, (size_t)(r - r_eff) * Am->n * sizeof(TO), st));
    if (r_eff == 0) GKB_HIP(hipStreamSynchronize(st));
  }
  int refined = 0;
  double ms_refine = 0.0;
  if constexpr (std::is_same<TO, float>::value) {
    if (r_eff > 0 && refine) {
      const double tr0 = now_ms();
      int d = opt.refine_dim > 0 ? opt.refine_dim : 2 * r;
      d = std::max(r_eff, std::min(d, rz.kk));
      rc = refine_bf16<TB>(S, Am, pr, rz, r_eff, d, sigma, U, V, &refined);
      if (rc != GKB_OK) return rc;
      ms_refine = now_ms() - tr0;
    }
  }
  if (r_eff > 0 && !refined) {
    std::vector<TB> Xh, Yh;
    to_colmajor<TB>(rz.X, pr.nq, rz.kk, r_eff, Xh);
    to_colmajor<TB>(rz.Y, pr.np, rz.kk, r_eff, Yh);
    GKB_HIP(hipMemcpyAsync(S.Xs(), Xh.data(), Xh.size() * sizeof(TB), hipMemcpyHostToDevice, st));
    GKB_HIP(hipMemcpyAsync(S.Ys(), Yh.data(), Yh.size() * sizeof(TB), hipMemcpyHostToDevice, st));
    if constexpr (onepass && !std::is_same<TO, double>::value) {
      double* Vo = reinterpret_cast<double*>(S.ws + S.L.Vo);
      double* Uo = reinterpret_cast<double*>(S.ws + S.L.Uo);
      GKB_HIP(gkb::launch_gemm_tall<TB>(S.P(S.cur), S.L.ldn, Am->n, pr.np, S.Ys(), pr.np, r_eff, Vo, Am->n, st));
      GKB_HIP(gkb::launch_gemm_tall<TB>(S.Q(S.cur), S.L.ldm, Am->m, pr.nq, S.Xs(), pr.nq, r_eff, Uo, Am->m, st));
      GKB_HIP(gkb::launch_narrow(Vo, Am->n * r_eff, V, st));
      GKB_HIP(gkb::launch_narrow(Uo, Am->m * r_eff, U, st));
    } else {
      GKB_HIP(gkb::launch_gemm_tall<TB>(S.P(S.cur), S.L.ldn, Am->n, pr.np, S.Ys(), pr.np, r_eff, V, Am->n, st));
      GKB_HIP(gkb::launch_gemm_tall<TB>(S.Q(S.cur), S.L.ldm, Am->m, pr.nq, S.Xs(), pr.nq, r_eff, U, Am->m, st));
    }
    GKB_HIP(hipStreamSynchronize(st));
  }
  if (S.pt.on) {  // close the last interval
    GKB_HIP(S.mark(PH_OTHER));
    GKB_HIP(hipStreamSynchronize(st));
    GKB_HIP(S.pt.collect());
  }
  if (stats) {
    stats->nconv = ct.nconv;
    stats->restarts = restarts;
    stats->breakdown = pr.breakdown;
    stats->returned = r_eff;
    int refreshes = 0;
    if constexpr (onepass) {
      GKB_HIP(hipMemcpyAsync(&refreshes, S.refresh() + 1, sizeof(int), hipMemcpyDeviceToHost, st));
      GKB_HIP(hipStreamSynchronize(st));
    }
    stats->refreshes = refreshes;
    stats->matvecs = matvecs + refreshes;
    stats->bytes_A = (double)(S.a_passes + refreshes) * S.bytes_per_pass();
    double mr = 0.0;
    for (int i = 0; i < r_eff; ++i) mr = std::max(mr, ct.res[i]);
    stats->max_res_est = mr;
    stats->sigma1_est = rz.kk ? rz.s[0] : 0.0;
    stats->ms_total = now_ms() - t0;
    stats->ms_host = ms_host;
    stats->checks = checks;
    stats->krylov_dim = pr.np;
    stats->refined = refined;
    stats->ms_refine = ms_refine;
    stats->one_pass_used = onepass ? 1 : 0;
    S.pt.fill(stats);
  }
  if (r_eff < r) return GKB_RANK_DEFICIENT;
  return ct.nconv == r ? GKB_OK : GKB_NOT_CONVERGED;
}

template <typename TB>
gkb_status run_rank(const gkb_matrix* Am, double tau, int tau_relative, int k, const gkb_options& opt,
                    void* workspace, int64_t* rank, int64_t* rank_sturm, double* sigma_out, int* nsigma,
                    gkb_stats* stats, hipStream_t st, bool onepass = false) {
  const double t0 = now_ms();
  Solver<TB> S;
  S.A = {Am->data, Am->m, Am->n, Am->lda, (int)Am->dtype};
  S.st = st;
  S.L = make_layout(Am->m, Am->n, Am->dtype, k, false, false, false, true, onepass);
  S.ws = reinterpret_cast<char*>(workspace);
  S.onepass = onepass;
  S.eps = opt.eps_break > 0 ? opt.eps_break : (Am->dtype == GKB_F64 ? 1e-12 : 1e-6);
  S.relative = opt.eps_relative ? 1 : 0;
  S.pt.on = opt.phase_timing != 0;
  const double* q1 = opt.q1;
  GKB_HIP(S.mark(PH_OTHER));
  if (q1 == nullptr) {
    GKB_HIP(gkb::launch_philox_start(S.q1buf(), Am->m, opt.seed, st));
    q1 = S.q1buf();
  }
  gkb_status rc = S.start(q1);
  if (rc != GKB_OK) return rc;
  // launch in chunks; stop launching once a breakdown flag is seen
  const int chunk = 32;
  int fl[2] = {0, 0};
  for (int s0 = 0; s0 < k; s0 += chunk) {
    const int s1 = std::min(k, s0 + chunk);
    for (int s = s0; s < s1; ++s) {
      rc = onepass ? S.onepass_step(s, s, s + 1, s + 1, false) : S.first_step(s);
      if (rc != GKB_OK) return rc;
    }
    if (s1 < k) {
      GKB_HIP(hipMemcpyAsync(fl, S.flag(), 2 * sizeof(int), hipMemcpyDeviceToHost, st));
      GKB_HIP(hipStreamSynchronize(st));
      if (fl[0] != 0) break;
    }
  }
  std::vector<double> qc, pc;
  rc = S.read_back(k + 2, qc, pc, fl);
  if (rc != GKB_OK) return rc;
  Proj pr;
  RestartIn none;
  rc = assemble(true, k, none, qc, pc, fl, pr);
  if (rc != GKB_OK) return rc;
  const int np = pr.np, nq = pr.nq;
  std::vector<double> alpha(std::max(np, 1)), beta(std::max(nq, 1)), s(std::max(np, 1));
  for (int j = 0; j < np; ++j) alpha[j] = pc[j];
  for (int j = 0; j + 1 < nq; ++j) beta[j] = qc[j + 1];
  const double th = now_ms();
  if (np > 0 && !gkb::bidiag_singular_values(nq, np, alpha.data(), beta.data(), s.data()))
    return fail(GKB_ERR_NUMERIC, "bidiagonal SVD did not converge");
  const double ms_host = now_ms() - th;
  const double thr = np > 0 ? (tau_relative ? tau * s[0] : tau) : tau;
  int64_t cnt = 0;
  for (int j = 0; j < np; ++j)
    if (s[j] > thr) ++cnt;
  *rank = cnt;
  if (rank_sturm) *rank_sturm = np > 0 ? gkb::bidiag_count_above(nq, np, alpha.data(), beta.data(), thr) : 0;
  if (sigma_out)
    for (int j = 0; j < np; ++j) sigma_out[j] = s[j];
  if (nsigma) *nsigma = np;
  if (stats) {
    int refreshes = 0;
    if (onepass) {
      GKB_HIP(hipMemcpyAsync(&refreshes, S.refresh() + 1, sizeof(int), hipMemcpyDeviceToHost, st));
      GKB_HIP(hipStreamSynchronize(st));
    }
    std::memset(stats, 0, sizeof(*stats));
    stats->refreshes = refreshes;
    stats->breakdown = pr.breakdown;
    stats->returned = np;
    stats->matvecs = pr.matvecs + refreshes;
    stats->bytes_A = (double)(S.a_passes + refreshes) * S.bytes_per_pass();
    stats->sigma1_est = np > 0 ? s[0] : 0.0;
    stats->ms_total = now_ms() - t0;
    stats->ms_host = ms_host;
    stats->one_pass_used = onepass ? 1 : 0;
    S.pt.fill(stats);
  }
  return GKB_OK;
}

}  // namespace

// Argument checks of gkb_partial_svd (and of a plan); fills opt (defaults,
// one_pass dropped where the sweep is unavailable).
gkb_status validate_svd(const gkb_matrix* A, int r, int k, double tol, int max_restarts, const gkb_options* opt_in,
                        void* workspace, size_t ws_bytes, gkb_options& opt);

// The solve behind gkb_partial_svd and plans (arguments already checked).
gkb_status dispatch_svd(const gkb_matrix* A, int r, int k, double tol, int max_restarts, const gkb_options& opt,
                        void* workspace, double* sigma, void* U, void* V, gkb_stats* stats, hipStream_t st,
                        SegmentGraphs* graphs) {
  if (opt.one_pass && A->dtype == GKB_F64)
    return run_partial_svd<double, double, true>(A, r, k, tol, max_restarts, opt, workspace, sigma,
                                                 reinterpret_cast<double*>(U), reinterpret_cast<double*>(V), stats,
                                                 st, nullptr, graphs);
  if (opt.one_pass)
    return run_partial_svd<double, float>(A, r, k, tol, max_restarts, opt, workspace, sigma,
                                          reinterpret_cast<float*>(U), reinterpret_cast<float*>(V), stats, st,
                                          nullptr, graphs);
  if (A->dtype == GKB_F64)
    return run_partial_svd<double>(A, r, k, tol, max_restarts, opt, workspace, sigma,
                                   reinterpret_cast<double*>(U), reinterpret_cast<double*>(V), stats, st, nullptr,
                                   graphs);
  return run_partial_svd<float>(A, r, k, tol, max_restarts, opt, workspace, sigma, reinterpret_cast<float*>(U),
                                reinterpret_cast<float*>(V), stats, st, nullptr, graphs);
}

// ======================================================================= ABI
// ---- the entry point that allocates nothing: a fixed device array per GPU
static __device__ __align__(256) unsigned char scratch[GKB_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device
// (each GPU holds its own copy of the array at its own address).
gkb_status scratch_address(void** out) {
  int dev = 0;
  GKB_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(GKB_ERR_INVALID, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    GKB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) return fail(GKB_ERR_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GKB_OK;
}
}  // namespace

extern "C" {

void gkb_default_options(gkb_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->eps_relative = 1;
  opt->seed = 0;
}

size_t gkb_workspace_size(const gkb_matrix* A, int r, int k, const gkb_options* opt) {
  if (check_matrix(A) != GKB_OK) return 0;
  if (r < 1 || k < r || k > std::min(A->m, A->n)) return 0;
  const bool onepass = opt != nullptr && opt->one_pass != 0 && one_pass_available(A);
  return make_layout(A->m, A->n, A->dtype, k, k > r, true, A->dtype == GKB_BF16 && A->refine_f32 != nullptr,
                     true, onepass)
      .total;
}

}  // extern "C"

gkb_status validate_svd(const gkb_matrix* A, int r, int k, double tol, int max_restarts, const gkb_options* opt_in,
                        void* workspace, size_t ws_bytes, gkb_options& opt) {
  gkb_status rc = check_matrix(A);
  if (rc != GKB_OK) return rc;
  if (r < 1 || r > k) return fail(GKB_ERR_INVALID, "need 1 <= r <= k");
  if (k > std::min(A->m, A->n)) return fail(GKB_ERR_INVALID, "need k <= min(m, n)");
  if (!(tol >= 0.0)) return fail(GKB_ERR_INVALID, "need tol >= 0");
  if (max_restarts < 0) return fail(GKB_ERR_INVALID, "need max_restarts >= 0");
  gkb_default_options(&opt);
  if (opt_in) opt = *opt_in;
  if (opt.one_pass && !one_pass_available(A)) opt.one_pass = 0;  // the two-product step instead
  if (opt.keep != 0 && (opt.keep < r || opt.keep >= k))
    return fail(GKB_ERR_INVALID, "need r <= keep < k");
  if (opt.eps_break < 0) return fail(GKB_ERR_INVALID, "need eps_break >= 0");
  if (opt.check_every < 0) return fail(GKB_ERR_INVALID, "need check_every >= 0");
  if (opt.refine_dim < 0) return fail(GKB_ERR_INVALID, "need refine_dim >= 0");
  if (A->refine_f32 != nullptr) {
    if (A->dtype != GKB_BF16) return fail(GKB_ERR_INVALID, "refine_f32 is only used with GKB_BF16");
    if (A->lda_refine < A->n) return fail(GKB_ERR_INVALID, "need lda_refine >= n");
  }
  return check_workspace(workspace, ws_bytes, gkb_workspace_size(A, r, k, &opt));
}

extern "C" {

gkb_status gkb_partial_svd(const gkb_matrix* A, int r, int k, double tol, int max_restarts,
                           const gkb_options* opt_in, void* workspace, size_t ws_bytes, double* sigma,
                           void* U, void* V, gkb_stats* stats, void* stream) {
  g_err.clear();
  if (sigma == nullptr || U == nullptr || V == nullptr)
    return fail(GKB_ERR_INVALID, "sigma, U and V must be non-NULL");
  gkb_options opt;
  gkb_status rc = validate_svd(A, r, k, tol, max_restarts, opt_in, workspace, ws_bytes, opt);
  if (rc != GKB_OK) return rc;
  return dispatch_svd(A, r, k, tol, max_restarts, opt, workspace, sigma, U, V, stats,
                      reinterpret_cast<hipStream_t>(stream), nullptr);
}

// ---- plans: repeated solves of one matrix buffer with graph-captured stretches
struct gkb_svd_plan_s {
  gkb_matrix A;
  int r = 0, k = 0, max_restarts = 0;
  double tol = 0.0;
  gkb_options opt;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  SegmentGraphs graphs;
};

gkb_status gkb_svd_plan_create(const gkb_matrix* A, int r, int k, double tol, int max_restarts,
                               const gkb_options* opt_in, void* workspace, size_t ws_bytes, gkb_svd_plan* plan) {
  g_err.clear();
  if (plan == nullptr) return fail(GKB_ERR_INVALID, "plan must be non-NULL");
  *plan = nullptr;
  gkb_options opt;
  gkb_status rc = validate_svd(A, r, k, tol, max_restarts, opt_in, workspace, ws_bytes, opt);
  if (rc != GKB_OK) return rc;
  if (opt.phase_timing) return fail(GKB_ERR_INVALID, "phase_timing is not available with a plan");
  auto* p = new gkb_svd_plan_s();
  p->A = *A;
  p->r = r;
  p->k = k;
  p->tol = tol;
  p->max_restarts = max_restarts;
  p->opt = opt;
  p->ws = workspace;
  p->ws_bytes = ws_bytes;
  if (hipStreamCreateWithFlags(&p->graphs.capture, hipStreamNonBlocking) != hipSuccess) {
    delete p;
    return fail(GKB_ERR_HIP, "hipStreamCreateWithFlags failed");
  }
  *plan = p;
  return GKB_OK;
}

gkb_status gkb_svd_plan_run(gkb_svd_plan plan, const double* q1, double* sigma, void* U, void* V, gkb_stats* stats,
                            void* stream) {
  g_err.clear();
  if (plan == nullptr) return fail(GKB_ERR_INVALID, "plan is NULL");
  if (sigma == nullptr || U == nullptr || V == nullptr)
    return fail(GKB_ERR_INVALID, "sigma, U and V must be non-NULL");
  gkb_options opt = plan->opt;
  if (q1 != nullptr) opt.q1 = q1;
  return dispatch_svd(&plan->A, plan->r, plan->k, plan->tol, plan->max_restarts, opt, plan->ws, sigma, U, V, stats,
                      reinterpret_cast<hipStream_t>(stream), &plan->graphs);
}

void gkb_svd_plan_destroy(gkb_svd_plan plan) { delete plan; }

gkb_status gkb_partial_svd_noalloc(const gkb_matrix* A, int r, int k, double tol, int max_restarts,
                                   const gkb_options* opt, double* sigma, void* U, void* V, gkb_stats* stats,
                                   void* stream) {
  g_err.clear();
  gkb_status rc = check_matrix(A);
  if (rc != GKB_OK) return rc;
  if (opt != nullptr && opt->phase_timing != 0)
    return fail(GKB_ERR_INVALID, "phase_timing creates HIP events; not available without allocation");
  const size_t need = gkb_workspace_size(A, r, k, opt);
  if (need > GKB_NOALLOC_SCRATCH_BYTES)
    return fail(GKB_ERR_WORKSPACE, "problem needs " + std::to_string(need) + " bytes of workspace; the fixed " +
                                       "array holds " + std::to_string(GKB_NOALLOC_SCRATCH_BYTES) +
                                       " (use gkb_partial_svd with a caller workspace)");
  void* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc != GKB_OK) return rc;
  // need == 0 means invalid arguments: gkb_partial_svd reports which
  return gkb_partial_svd(A, r, k, tol, max_restarts, opt, ws, GKB_NOALLOC_SCRATCH_BYTES, sigma, U, V, stats,
                         stream);
}

size_t gkb_rank_workspace_size(const gkb_matrix* A, int k_max, const gkb_options* opt) {
  if (check_matrix(A) != GKB_OK) return 0;
  const int64_t kmin = std::min(A->m, A->n);
  const int64_t k = k_max ? k_max : kmin;
  if (k < 1 || k > kmin) return 0;
  const bool onepass = opt != nullptr && opt->one_pass != 0 && one_pass_available(A);
  return make_layout(A->m, A->n, A->dtype, (int)k, false, false, false, true, onepass).total;
}

gkb_status gkb_numerical_rank(const gkb_matrix* A, double tau, int tau_relative, int k_max,
                              const gkb_options* opt_in, void* workspace, size_t ws_bytes, int64_t* rank,
                              int64_t* rank_sturm, double* sigma_out, int* nsigma, gkb_stats* stats,
                              void* stream) {
  g_err.clear();
  gkb_status rc = check_matrix(A);
  if (rc != GKB_OK) return rc;
  if (!(tau > 0.0)) return fail(GKB_ERR_INVALID, "need tau > 0");
  const int64_t kmin = std::min(A->m, A->n);
  const int64_t k = k_max ? k_max : kmin;
  if (k < 1 || k > kmin) return fail(GKB_ERR_INVALID, "need 0 <= k_max <= min(m, n)");
  if (rank == nullptr) return fail(GKB_ERR_INVALID, "rank must be non-NULL");
  gkb_options opt;
  gkb_default_options(&opt);
  if (opt_in) opt = *opt_in;
  if (opt.eps_break < 0) return fail(GKB_ERR_INVALID, "need eps_break >= 0");
  if (opt.one_pass && !one_pass_available(A)) opt.one_pass = 0;  // the two-product step instead
  rc = check_workspace(workspace, ws_bytes, gkb_rank_workspace_size(A, (int)k, &opt));
  if (rc != GKB_OK) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (opt.one_pass)
    return run_rank<double>(A, tau, tau_relative, (int)k, opt, workspace, rank, rank_sturm, sigma_out, nsigma,
                            stats, st, true);
  if (A->dtype == GKB_F64)
    return run_rank<double>(A, tau, tau_relative, (int)k, opt, workspace, rank, rank_sturm, sigma_out, nsigma,
                            stats, st);
  return run_rank<float>(A, tau, tau_relative, (int)k, opt, workspace, rank, rank_sturm, sigma_out, nsigma,
                         stats, st);
}

size_t gkb_sparse_workspace_size(gkb_sparse_plan plan, int r, int k) {
  if (!plan) return 0;
  const gkb::SparseRef& R = plan->ref;
  if (r < 1 || k < r || k > std::min(R.m, R.n)) return 0;
  return make_layout(R.m, R.n, GKB_F32, k, k > r, true, false, false).total;
}

gkb_status gkb_partial_svd_sparse(gkb_sparse_plan plan, int r, int k, double tol, int max_restarts,
                                  const gkb_options* opt_in, void* workspace, size_t ws_bytes, double* sigma,
                                  float* U, float* V, gkb_stats* stats, void* stream) {
  g_err.clear();
  if (!plan) return fail(GKB_ERR_INVALID, "sparse plan is NULL");
  const gkb::SparseRef& R = plan->ref;
  if (r < 1 || k < r || k > std::min(R.m, R.n)) return fail(GKB_ERR_INVALID, "need 1 <= r <= k <= min(m, n)");
  if (!(tol >= 0.0) || max_restarts < 0) return fail(GKB_ERR_INVALID, "need tol >= 0 and max_restarts >= 0");
  if (!sigma || !U || !V) return fail(GKB_ERR_INVALID, "sigma, U and V must be non-NULL");
  gkb_options opt;
  gkb_default_options(&opt);
  if (opt_in) opt = *opt_in;
  if (opt.keep != 0 && (opt.keep < r || opt.keep >= k)) return fail(GKB_ERR_INVALID, "need r <= keep < k");
  if (opt.eps_break < 0) return fail(GKB_ERR_INVALID, "need eps_break >= 0");
  if (opt.check_every < 0) return fail(GKB_ERR_INVALID, "need check_every >= 0");
  opt.one_pass = 0;  // sparse A: always the two CSR products (stats.one_pass_used = 0)
  gkb_status rc = check_workspace(workspace, ws_bytes, gkb_sparse_workspace_size(plan, r, k));
  if (rc != GKB_OK) return rc;
  // the dense descriptor only carries the shape and the float32 basis type
  gkb_matrix Am{};
  Am.m = R.m;
  Am.n = R.n;
  Am.lda = R.n;
  Am.dtype = GKB_F32;
  return run_partial_svd<float>(&Am, r, k, tol, max_restarts, opt, workspace, sigma, U, V, stats,
                                reinterpret_cast<hipStream_t>(stream), &R);
}

const char* gkb_status_string(gkb_status s) {
  switch (s) {
    case GKB_OK: return "GKB_OK";
    case GKB_NOT_CONVERGED: return "GKB_NOT_CONVERGED";
    case GKB_RANK_DEFICIENT: return "GKB_RANK_DEFICIENT";
    case GKB_ERR_INVALID: return "GKB_ERR_INVALID";
    case GKB_ERR_HIP: return "GKB_ERR_HIP";
    case GKB_ERR_NUMERIC: return "GKB_ERR_NUMERIC";
    case GKB_ERR_WORKSPACE: return "GKB_ERR_WORKSPACE";
    case GKB_ERR_TIMEOUT: return "GKB_ERR_TIMEOUT";
  }
  return "unknown";
}

const char* gkb_last_error(void) { return g_err.c_str(); }

gkb_status gkb_host_dense_svd(int nq, int np, const double* H, double* s, double* X, double* Y) {
  g_err.clear();
  if (nq < 1 || np < 1 || !H || !s || !X || !Y) return fail(GKB_ERR_INVALID, "bad arguments");
  if (!gkb::dense_svd(nq, np, H, s, X, Y)) return fail(GKB_ERR_NUMERIC, "no convergence or non-finite input");
  return GKB_OK;
}

int64_t gkb_host_bidiag_count_above(int nq, int np, const double* alpha, const double* beta, double tau) {
  if (np < 1 || (nq != np && nq != np + 1) || !alpha || (nq > 1 && !beta) || !(tau > 0)) return -1;
  return gkb::bidiag_count_above(nq, np, alpha, beta, tau);
}

gkb_status gkb_host_bidiag_lastrow(int np, const double* alpha, const double* beta, double* s, double* last) {
  g_err.clear();
  if (np < 1 || !alpha || !beta || !s || !last) return fail(GKB_ERR_INVALID, "bad arguments");
  if (!gkb::bidiag_sv_lastrow(np, alpha, beta, s, last))
    return fail(GKB_ERR_NUMERIC, "no convergence or non-finite input");
  return GKB_OK;
}

// ------------------------------------------------------------ building blocks
size_t gkb_matvec_workspace_size(const gkb_matrix* A) {
  if (check_matrix(A) != GKB_OK) return 0;
  const int64_t part_rows = std::min<int64_t>(gkb::GEMV_T_MAX_BLOCKS, (A->m + 63) / 64);
  return align256((size_t)part_rows * round64(A->n) * (A->dtype == GKB_F64 ? 8 : 4));
}

size_t gkb_matvec_fused_workspace_size(const gkb_matrix* A) {
  if (check_matrix(A) != GKB_OK || A->dtype == GKB_F64 || !gkb::fused_ok(A->m, A->n, A->lda, A->data, (int)A->dtype))
    return 0;
  // partial sums, then the team sweep's mailbox for rows longer than FUSED_NMAX
  return align256((size_t)gkb::fused_blocks(A->m, A->n, (int)A->dtype) * round64(A->n) * 8) +
         (gkb::team_form(A->n, (int)A->dtype) ? align256(gkb::team_bytes(A->m, A->n, (int)A->dtype)) : 0);
}

gkb_status gkb_matvec_fused(const gkb_matrix* A, const float* p, double* w, double* y, void* workspace,
                            size_t ws_bytes, void* stream) {
  g_err.clear();
  gkb_status rc = check_matrix(A);
  if (rc != GKB_OK) return rc;
  if (A->dtype == GKB_F64 || !gkb::fused_ok(A->m, A->n, A->lda, A->data, (int)A->dtype))
    return fail(GKB_ERR_INVALID, "the fused sweep needs a float32 (bfloat16) A with lda and n multiples of 4 (8), "
                                 "n <= 262144, 16-byte aligned");
  if (!p || !w || !y) return fail(GKB_ERR_INVALID, "p, w and y must be non-NULL");
  rc = check_workspace(workspace, ws_bytes, gkb_matvec_fused_workspace_size(A));
  if (rc != GKB_OK) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  void* team = nullptr;
  if (gkb::team_form(A->n, (int)A->dtype)) {
    team = reinterpret_cast<char*>(workspace) +
           align256((size_t)gkb::fused_blocks(A->m, A->n, (int)A->dtype) * round64(A->n) * 8);
    GKB_HIP(gkb::launch_team_reset(team, A->m, A->n, (int)A->dtype, st));
  }
  GKB_HIP(gkb::launch_gemv_fused<float>(A->data, (int)A->dtype, A->lda, A->m, A->n, p, nullptr, w, y,
                                        reinterpret_cast<double*>(workspace), round64(A->n), nullptr, st, nullptr,
                                        nullptr, nullptr, team));
  return GKB_OK;
}

gkb_status gkb_matvec(const gkb_matrix* A, int trans, const void* x, double* y, void* workspace,
                      size_t ws_bytes, void* stream) {
  g_err.clear();
  gkb_status rc = check_matrix(A);
  if (rc != GKB_OK) return rc;
  if (!x || !y) return fail(GKB_ERR_INVALID, "x and y must be non-NULL");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  gkb::MatrixRef R{A->data, A->m, A->n, A->lda, (int)A->dtype};
  if (trans == 0) {
    if (A->dtype == GKB_F64)
      GKB_HIP(gkb::launch_gemv_n<double>(R, (const double*)x, nullptr, nullptr, 0, y, nullptr, st));
    else
      GKB_HIP(gkb::launch_gemv_n<float>(R, (const float*)x, nullptr, nullptr, 0, y, nullptr, st));
    return GKB_OK;
  }
  rc = check_workspace(workspace, ws_bytes, gkb_matvec_workspace_size(A));
  if (rc != GKB_OK) return rc;
  const int64_t ldpart = round64(A->n);
  if (A->dtype == GKB_F64)
    GKB_HIP(gkb::launch_gemv_t<double>(R, (const double*)x, nullptr, nullptr, 0, y, workspace, ldpart, nullptr,
                                       st));
  else
    GKB_HIP(gkb::launch_gemv_t<float>(R, (const float*)x, nullptr, nullptr, 0, y, workspace, ldpart, nullptr,
                                      st));
  return GKB_OK;
}

gkb_status gkb_gemm_tall(gkb_dtype dtype, const void* A, int64_t lda, int64_t M, int K, const void* B,
                         int64_t ldb, int N, void* C, int64_t ldc, void* stream) {
  g_err.clear();
  if (dtype != GKB_F64 && dtype != GKB_F32) return fail(GKB_ERR_INVALID, "dtype must be F64 or F32");
  if (M < 0 || K < 0 || N < 0 || lda < M || ldb < K || ldc < M)
    return fail(GKB_ERR_INVALID, "bad GEMM shape");
  if ((M > 0 && N > 0) && (!C || (K > 0 && (!A || !B)))) return fail(GKB_ERR_INVALID, "NULL operand");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (dtype == GKB_F64)
    GKB_HIP(gkb::launch_gemm_tall<double>((const double*)A, lda, M, K, (const double*)B, ldb, N, (double*)C, ldc,
                                          st));
  else
    GKB_HIP(gkb::launch_gemm_tall<float>((const float*)A, lda, M, K, (const float*)B, ldb, N, (float*)C, ldc,
                                         st));
  return GKB_OK;
}

gkb_status gkb_gemm_rowmajor(const float* A, int64_t lda, int64_t M, int64_t K, const float* B, int64_t ldb,
                             int N, float* C, int64_t ldc, void* stream) {
  g_err.clear();
  if (M < 0 || K < 0 || N < 0 || lda < K || ldb < K || ldc < M) return fail(GKB_ERR_INVALID, "bad GEMM shape");
  if ((M > 0 && N > 0) && (!A || !B || !C)) return fail(GKB_ERR_INVALID, "NULL operand");
  GKB_HIP(gkb::launch_gemm_rm(A, lda, M, K, B, ldb, N, C, ldc, reinterpret_cast<hipStream_t>(stream)));
  return GKB_OK;
}

size_t gkb_gram_workspace_size(int64_t m, int d) {
  if (m < 1 || d < 1) return 0;
  return align256((size_t)gkb::gram_chunks(m) * d * d * 8);
}

gkb_status gkb_gram(const float* W, int64_t ldw, int64_t m, int d, double* G, void* workspace, size_t ws_bytes,
                    void* stream) {
  g_err.clear();
  if (!W || !G || m < 1 || d < 1 || ldw < m) return fail(GKB_ERR_INVALID, "bad Gram arguments");
  gkb_status rc = check_workspace(workspace, ws_bytes, gkb_gram_workspace_size(m, d));
  if (rc != GKB_OK) return rc;
  GKB_HIP(gkb::launch_gram(W, ldw, m, d, reinterpret_cast<double*>(workspace), G,
                           reinterpret_cast<hipStream_t>(stream)));
  return GKB_OK;
}

gkb_status gkb_cast_bf16(const float* src, int64_t lds, int64_t m, int64_t n, uint16_t* dst, int64_t ldd,
                         void* stream) {
  g_err.clear();
  if (!src || !dst || m < 1 || n < 1 || lds < n || ldd < n) return fail(GKB_ERR_INVALID, "bad cast arguments");
  GKB_HIP(gkb::launch_cast_bf16(src, lds, m, n, dst, ldd, reinterpret_cast<hipStream_t>(stream)));
  return GKB_OK;
}

gkb_status gkb_start_vector(double* q, int64_t m, uint64_t seed, void* stream) {
  g_err.clear();
  if (!q || m < 1) return fail(GKB_ERR_INVALID, "bad start-vector arguments");
  GKB_HIP(gkb::launch_philox_start(q, m, seed, reinterpret_cast<hipStream_t>(stream)));
  return GKB_OK;
}

}  // extern "C"
