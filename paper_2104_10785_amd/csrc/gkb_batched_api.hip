// C ABI of the batched form: plan (problem table, largest-first order,
// hipGraph of [queue reset, staging copy of unaligned matrices, persistent
// solver]), run, results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/gkb.h"
#include "../../include/gkb_batched.h"
#include "batched.h"

namespace {

thread_local std::string b_err;

gkb_status bfail(gkb_status s, const std::string& m) {
  b_err = m;
  return s;
}

#define B_HIP(call)                                                                    \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return bfail(GKB_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int TEAM_MAX = 8;   // largest team of workgroups on one problem
constexpr double OUTLINE_MIN_BYTES = 2.0 * (1 << 20);   // average A bytes per problem for out-of-line products

struct Layout {
  size_t problems = 0, order = 0, member = 0, counter = 0, info = 0, ticks = 0, pool = 0, work = 0, stage_tab = 0,
         stage = 0,
         team_cnt = 0, team_buf = 0, total = 0;
  size_t pool_floats = 0, work_doubles = 0, stage_floats = 0, team_doubles = 0;
  int nstage = 0;
};

// Team buffers of one problem for a team of T: T x n partial products and two
// alternating T x (KMAX + 4) regions for the partial dots and norms.
inline size_t team_doubles(int T, int64_t n) { return (size_t)T * n + 2 * (size_t)T * (gkb::BATCH_KMAX + 4); }

inline int64_t round4(int64_t x) { return (x + 3) & ~int64_t(3); }

// The persistent kernel streams A with 16-byte loads; a matrix whose rows are
// not 16-byte aligned, or whose column count is not a multiple of 4, is first
// copied (inside the same graph) into zero-padded rows of round4(n) floats.
bool needs_stage(const gkb_matrix& A) {
  return (A.lda & 3) != 0 || (A.n & 3) != 0 || (reinterpret_cast<uintptr_t>(A.data) & 15) != 0;
}

gkb_status check_batch(int batch, const gkb_matrix* As, const int* r, const int* k) {
  if (batch < 1) return bfail(GKB_ERR_INVALID, "need batch >= 1");
  if (!As || !r || !k) return bfail(GKB_ERR_INVALID, "As, r and k must be non-NULL");
  for (int i = 0; i < batch; ++i) {
    const gkb_matrix& A = As[i];
    if (A.dtype != GKB_F32) return bfail(GKB_ERR_INVALID, "batched problems must be GKB_F32");
    if (!A.data || A.m < 1 || A.n < 1 || A.lda < A.n) return bfail(GKB_ERR_INVALID, "bad matrix in batch");
    if (A.m > (1 << 30) || A.n > (1 << 30)) return bfail(GKB_ERR_INVALID, "matrix too large for the batch");
    if (r[i] < 1 || r[i] > k[i] || k[i] > std::min(A.m, A.n))
      return bfail(GKB_ERR_INVALID, "need 1 <= r <= k <= min(m, n) for problem " + std::to_string(i));
    if (k[i] > gkb::BATCH_KMAX)
      return bfail(GKB_ERR_INVALID, "batched Krylov dimension above " + std::to_string(gkb::BATCH_KMAX));
  }
  return GKB_OK;
}

Layout layout(int batch, const gkb_matrix* As, const int* k) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off += a256(b);
    return o;
  };
  L.problems = take(sizeof(gkb::BatchProblem) * batch);
  L.order = take(sizeof(int) * batch * TEAM_MAX);
  L.member = take(sizeof(int) * batch * TEAM_MAX);
  L.counter = take(sizeof(int));
  L.info = take(sizeof(int) * 4 * batch);
  L.ticks = take(sizeof(unsigned long long) * batch);
  for (int i = 0; i < batch; ++i) {
    L.pool_floats += (size_t)2 * (k[i] + 1) * (round4(As[i].m) + round4(As[i].n));
    L.work_doubles += (size_t)(As[i].m + As[i].n);
    if (needs_stage(As[i])) {
      ++L.nstage;
      L.stage_floats += a256((size_t)As[i].m * round4(As[i].n) * sizeof(float)) / sizeof(float);
    }
    L.team_doubles += team_doubles(TEAM_MAX, As[i].n);   // room for the largest team
  }
  L.pool = take(L.pool_floats * sizeof(float));
  L.work = take(L.work_doubles * sizeof(double));
  L.stage_tab = take(sizeof(gkb::StageCopy) * std::max(L.nstage, 1));
  L.stage = take(L.stage_floats * sizeof(float));
  L.team_cnt = take(sizeof(int) * batch);
  L.team_buf = take(L.team_doubles * sizeof(double));
  L.total = off;
  return L;
}

}  // namespace

struct gkb_batch_plan_s {
  int batch = 0;
  int grid = 0;
  gkb::BatchParams prm{};
  std::vector<gkb::BatchProblem> table;
  std::vector<int> order;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;
  int* info_dev = nullptr;
  unsigned long long* ticks_dev = nullptr;
  double ticks_per_ms = 1e5;   // device wall clock (kHz)
  bool no_graph = false;
  int threads = 1024;
};

extern "C" {

const char* gkb_batched_last_error(void) { return b_err.c_str(); }

void gkb_batch_default_options(gkb_batch_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->eps_relative = 1;
}

size_t gkb_batched_workspace_size(int batch, const gkb_matrix* As, const int* r, const int* k) {
  if (check_batch(batch, As, r, k) != GKB_OK) return 0;
  return layout(batch, As, k).total;
}

gkb_status gkb_batched_plan_create(int batch, const gkb_matrix* As, const int* r, const int* k, double tol,
                                   int max_restarts, const gkb_batch_options* opt_in, void* workspace,
                                   size_t ws_bytes, double* sigma, float* U, float* V, void* stream,
                                   gkb_batch_plan* out) {
  b_err.clear();
  if (!out) return bfail(GKB_ERR_INVALID, "plan pointer is NULL");
  *out = nullptr;
  gkb_status rc = check_batch(batch, As, r, k);
  if (rc != GKB_OK) return rc;
  if (!(tol >= 0.0) || max_restarts < 0) return bfail(GKB_ERR_INVALID, "need tol >= 0 and max_restarts >= 0");
  if (!sigma || !U || !V) return bfail(GKB_ERR_INVALID, "sigma, U and V must be non-NULL");
  gkb_batch_options opt;
  gkb_batch_default_options(&opt);
  if (opt_in) opt = *opt_in;
  if (opt.check_every < 0 || opt.eps_break < 0 || opt.workgroups < 0)
    return bfail(GKB_ERR_INVALID, "bad batch options");
  if (opt.threads != 0 && opt.threads != 512 && opt.threads != 1024)
    return bfail(GKB_ERR_INVALID, "threads must be 0, 512 or 1024");
  if (opt.max_team < 0) return bfail(GKB_ERR_INVALID, "max_team must be >= 0");
  if (opt.form < 0 || opt.form > 2) return bfail(GKB_ERR_INVALID, "form must be 0, 1 or 2");
  int dev = 0, cus = 0, clock_khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
    return bfail(GKB_ERR_HIP, "cannot query the device");
  if (opt.cost_estimate)
    for (int i = 0; i < batch; ++i)
      if (!(opt.cost_estimate[i] >= 0.0) || !std::isfinite(opt.cost_estimate[i]))
        return bfail(GKB_ERR_INVALID, "cost estimates must be finite and >= 0");
  Layout L = layout(batch, As, k);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0 || ws_bytes < L.total)
    return bfail(GKB_ERR_WORKSPACE, "workspace missing, misaligned or too small (need " +
                                        std::to_string(L.total) + " bytes)");
  char* ws = reinterpret_cast<char*>(workspace);
  auto* plan = new gkb_batch_plan_s();
  plan->batch = batch;
  plan->table.resize(batch);
  int64_t offQ = 0, offW = 0, offU = 0, offV = 0, offS = 0, offQ1 = 0, offStage = 0, stage_rows = 0;
  std::vector<gkb::StageCopy> stage;
  float* stage_base = reinterpret_cast<float*>(ws + L.stage);
  for (int i = 0; i < batch; ++i) {
    gkb::BatchProblem& P = plan->table[i];
    P.A = reinterpret_cast<const float*>(As[i].data);
    P.lda = As[i].lda;
    P.m = (int)As[i].m;
    P.n = (int)As[i].n;
    P.padded = 0;
    if (needs_stage(As[i])) {
      gkb::StageCopy c;
      c.src = P.A;
      c.lds = P.lda;
      c.m = P.m;
      c.n = P.n;
      c.ldd = round4(P.n);
      c.dst = stage_base + offStage;
      c.row_start = stage_rows;
      stage.push_back(c);
      stage_rows += P.m;
      offStage += (int64_t)(a256((size_t)P.m * c.ldd * sizeof(float)) / sizeof(float));
      P.A = c.dst;
      P.lda = c.ldd;
      P.padded = 1;
    }
    P.r = r[i];
    P.k = k[i];
    P.l = std::min(r[i] + (k[i] - r[i]) / 2, k[i] - 1);
    P.index = i;
    P.ldq = (int)round4(P.m);
    P.ldp = (int)round4(P.n);
    P.offQ = offQ;
    P.offP = offQ + (int64_t)2 * (k[i] + 1) * P.ldq;
    offQ = P.offP + (int64_t)2 * (k[i] + 1) * P.ldp;
    P.offW = offW;
    offW += P.m + P.n;
    P.offU = offU;
    offU += (int64_t)P.m * r[i];
    P.offV = offV;
    offV += (int64_t)P.n * r[i];
    P.offS = offS;
    offS += r[i];
    P.offQ1 = offQ1;
    offQ1 += P.m;
  }
  // persistent grid: one workgroup per compute unit unless asked otherwise
  plan->threads = opt.threads ? opt.threads : 1024;
  plan->grid = opt.workgroups > 0 ? opt.workgroups : cus;
  // Teams: a problem whose estimated cost (m n k, or the caller's estimate) exceeds half of the average
  // per-workgroup share of the whole batch is split over
  // T = ceil(cost / (share / 2)) workgroups (at most max_team, the grid, m / 256
  // and n / 64), so that no single problem outlasts the rest of the batch.
  const int max_team = std::min(opt.max_team > 0 ? opt.max_team : TEAM_MAX, TEAM_MAX);
  std::vector<double> cost(batch);
  double total = 0.0;
  for (int i = 0; i < batch; ++i) {
    cost[i] = opt.cost_estimate ? std::max(opt.cost_estimate[i], 1e-30)
                                : (double)plan->table[i].m * plan->table[i].n * plan->table[i].k;
    total += cost[i];
  }
  const double half_share = 0.5 * total / plan->grid;
  int nteams = 0;
  int64_t offTeam = 0;
  int ntickets = 0;
  for (int i = 0; i < batch; ++i) {
    gkb::BatchProblem& P = plan->table[i];
    int T = (int)std::ceil(cost[i] / std::max(half_share, 1.0));
    T = std::min({T, max_team, plan->grid, std::max(1, P.m / 256), std::max(1, P.n / 64)});
    if (P.n > gkb::BATCH_TEAM_NMAX) T = 1;   // a team keeps p in LDS
    T = std::max(T, 1);
    P.team = T;
    P.team_id = T > 1 ? nteams++ : 0;
    P.offTeam = offTeam;
    offTeam += (int64_t)team_doubles(T, P.n);
    ntickets += T;
  }
  // tickets: largest per-member cost first, a team's members adjacent
  std::vector<int> byp(batch);
  std::iota(byp.begin(), byp.end(), 0);
  std::stable_sort(byp.begin(), byp.end(),
                   [&](int a, int b) { return cost[a] / plan->table[a].team > cost[b] / plan->table[b].team; });
  plan->order.clear();
  std::vector<int> members;
  for (int i : byp)
    for (int j = 0; j < plan->table[i].team; ++j) {
      plan->order.push_back(i);
      members.push_back(j);
    }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  gkb::BatchParams& prm = plan->prm;
  prm.problems = reinterpret_cast<const gkb::BatchProblem*>(ws + L.problems);
  prm.order = reinterpret_cast<const int*>(ws + L.order);
  prm.member = reinterpret_cast<const int*>(ws + L.member);
  prm.counter = reinterpret_cast<int*>(ws + L.counter);
  prm.batch = batch;
  prm.ntickets = ntickets;
  prm.team_cnt = reinterpret_cast<int*>(ws + L.team_cnt);
  prm.nteams = nteams;
  prm.team_buf = reinterpret_cast<double*>(ws + L.team_buf);
  // Out-of-line products pay a register save and restore per call, which the
  // streaming of long rows amortises: measured 124 -> 89.5 ms on the 512-problem
  // batch (10 MB of A per problem on average) and 0.86 -> 1.0 ms per step on the
  // single 784 x 256 retraction of the similarity-learning step (cache-resident).
  {
    double abytes = 0.0;
    for (int i = 0; i < batch; ++i) abytes += 4.0 * plan->table[i].m * plan->table[i].n;
    prm.outline = opt.form == 1 ? 0 : (opt.form == 2 ? 1 : (abytes / batch >= OUTLINE_MIN_BYTES ? 1 : 0));
  }
  prm.pool = reinterpret_cast<float*>(ws + L.pool);
  prm.work = reinterpret_cast<double*>(ws + L.work);
  prm.U = U;
  prm.V = V;
  prm.sigma = sigma;
  prm.info = reinterpret_cast<int*>(ws + L.info);
  prm.ticks = reinterpret_cast<unsigned long long*>(ws + L.ticks);
  prm.q1 = opt.q1_packed;
  prm.seed = opt.seed;
  prm.eps_break = opt.eps_break > 0 ? opt.eps_break : 1e-6;
  prm.tol = tol;
  prm.max_restarts = max_restarts;
  prm.check_every = opt.check_every;
  prm.relative = opt.eps_relative ? 1 : 0;
  prm.stage = reinterpret_cast<const gkb::StageCopy*>(ws + L.stage_tab);
  prm.nstage = (int)stage.size();
  prm.stage_rows = stage_rows;
  prm.spin_limit = gkb::BATCH_TEAM_SPIN_LIMIT;
  prm.barrier_skew = 0;
  if (const char* e = std::getenv("GKB_BATCH_STALL_POLLS")) {   // test of the timeout path
    const long polls = std::atol(e);
    if (polls > 0) {
      prm.spin_limit = polls;
      prm.barrier_skew = 1;
    }
  }
  plan->info_dev = prm.info;
  plan->ticks_dev = prm.ticks;
  plan->ticks_per_ms = clock_khz > 0 ? (double)clock_khz : 1e5;
  auto cleanup = [&](gkb_status s) {
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->capture) (void)hipStreamDestroy(plan->capture);
    delete plan;
    return s;
  };
  if (hipMemcpyAsync(ws + L.problems, plan->table.data(), sizeof(gkb::BatchProblem) * batch,
                     hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(ws + L.order, plan->order.data(), sizeof(int) * ntickets, hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(ws + L.member, members.data(), sizeof(int) * ntickets, hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      (!stage.empty() && hipMemcpyAsync(ws + L.stage_tab, stage.data(), sizeof(gkb::StageCopy) * stage.size(),
                                        hipMemcpyHostToDevice, st) != hipSuccess) ||
      hipStreamSynchronize(st) != hipSuccess)
    return cleanup(bfail(GKB_ERR_HIP, "uploading the problem table failed"));
  if (gkb::batched_setup() != hipSuccess) return cleanup(bfail(GKB_ERR_HIP, "cannot set the LDS size"));
  plan->grid = std::min(plan->grid, ntickets);
  plan->no_graph = opt.no_graph != 0;
  if (plan->no_graph) {
    *out = plan;
    return GKB_OK;
  }
  // capture [queue reset, persistent solver] once; replays reuse the graph
  if (hipStreamCreateWithFlags(&plan->capture, hipStreamNonBlocking) != hipSuccess)
    return cleanup(bfail(GKB_ERR_HIP, "cannot create the capture stream"));
  if (hipStreamBeginCapture(plan->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return cleanup(bfail(GKB_ERR_HIP, "cannot begin graph capture"));
  hipError_t le = gkb::launch_batched(prm, plan->grid, plan->threads, plan->capture);
  hipError_t ee = hipStreamEndCapture(plan->capture, &plan->graph);
  if (le != hipSuccess || ee != hipSuccess) return cleanup(bfail(GKB_ERR_HIP, "graph capture failed"));
  if (hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0) != hipSuccess)
    return cleanup(bfail(GKB_ERR_HIP, "graph instantiation failed"));
  *out = plan;
  return GKB_OK;
}

gkb_status gkb_batched_plan_run(gkb_batch_plan plan, void* stream) {
  b_err.clear();
  if (!plan) return bfail(GKB_ERR_INVALID, "invalid plan");
  if (plan->no_graph) {
    B_HIP(gkb::launch_batched(plan->prm, plan->grid, plan->threads, reinterpret_cast<hipStream_t>(stream)));
    return GKB_OK;
  }
  if (!plan->exec) return bfail(GKB_ERR_INVALID, "invalid plan");
  B_HIP(hipGraphLaunch(plan->exec, reinterpret_cast<hipStream_t>(stream)));
  return GKB_OK;
}

gkb_status gkb_batched_plan_info(gkb_batch_plan plan, int* info, void* stream) {
  b_err.clear();
  if (!plan || !info) return bfail(GKB_ERR_INVALID, "invalid plan or info pointer");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  B_HIP(hipMemcpyAsync(info, plan->info_dev, sizeof(int) * 4 * plan->batch, hipMemcpyDeviceToHost, st));
  B_HIP(hipStreamSynchronize(st));
  return GKB_OK;
}

gkb_status gkb_batched_plan_work(gkb_batch_plan plan, double* work_ms, void* stream) {
  b_err.clear();
  if (!plan || !work_ms) return bfail(GKB_ERR_INVALID, "invalid plan or output pointer");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::vector<unsigned long long> ticks((size_t)plan->batch);
  B_HIP(hipMemcpyAsync(ticks.data(), plan->ticks_dev, sizeof(unsigned long long) * plan->batch,
                       hipMemcpyDeviceToHost, st));
  B_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < plan->batch; ++i)
    work_ms[i] = (double)ticks[i] / plan->ticks_per_ms * plan->table[i].team;
  return GKB_OK;
}

int gkb_batched_plan_grid(gkb_batch_plan plan) { return plan ? plan->grid : 0; }

void gkb_batched_plan_destroy(gkb_batch_plan plan) {
  if (!plan) return;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  if (plan->capture) (void)hipStreamDestroy(plan->capture);
  delete plan;
}

gkb_status gkb_batched_autotune(int batch, const gkb_matrix* As, const int* r, const int* k, double tol,
                                int max_restarts, const gkb_batch_options* opt_in, void* workspace,
                                size_t ws_bytes, double* sigma, float* U, float* V, void* stream,
                                int* best_threads, int* best_workgroups, int* best_form, int* best_max_team,
                                double* times_ms, int* ncand) {
  b_err.clear();
  if (!best_threads || !best_workgroups) return bfail(GKB_ERR_INVALID, "output pointers are NULL");
  gkb_batch_options opt;
  gkb_batch_default_options(&opt);
  if (opt_in) opt = *opt_in;
  int dev = 0, cus = 0;
  B_HIP(hipGetDevice(&dev));
  B_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  size_t lds_max = 0;
  {
    int v = 0;
    B_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev));
    lds_max = (size_t)v;
  }
  const int cand_threads[3] = {1024, 512, 512};
  const int cand_per_cu[3] = {1, 1, 2};
  const int forms[2] = {1, 2}, teams[2] = {8, 4};
  const int nform = opt.form != 0 ? 1 : 2, nteam = opt.max_team != 0 ? 1 : 2;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  B_HIP(hipEventCreate(&e0));
  B_HIP(hipEventCreate(&e1));
  double best = 1e300;
  int n = 0;
  gkb_status rc = GKB_OK;
  for (int cf = 0; cf < 3 * nform * nteam && rc == GKB_OK; ++cf) {
    const int c = cf / (nform * nteam), f = (cf / nteam) % nform, tm = cf % nteam;
    double t = -1.0;
    if (gkb::batched_lds_bytes(cand_threads[c]) * cand_per_cu[c] <= lds_max) {
      gkb_batch_options o = opt;
      o.threads = cand_threads[c];
      o.workgroups = cus * cand_per_cu[c];
      o.no_graph = 1;
      if (opt.form == 0) o.form = forms[f];
      if (opt.max_team == 0) o.max_team = teams[tm];
      gkb_batch_plan plan = nullptr;
      rc = gkb_batched_plan_create(batch, As, r, k, tol, max_restarts, &o, workspace, ws_bytes, sigma, U, V,
                                   stream, &plan);
      if (rc != GKB_OK) break;
      rc = gkb_batched_plan_run(plan, stream);  // untimed
      if (rc == GKB_OK && hipEventRecord(e0, st) != hipSuccess) rc = bfail(GKB_ERR_HIP, "event record");
      if (rc == GKB_OK) rc = gkb_batched_plan_run(plan, stream);
      if (rc == GKB_OK && hipEventRecord(e1, st) != hipSuccess) rc = bfail(GKB_ERR_HIP, "event record");
      if (rc == GKB_OK && hipEventSynchronize(e1) != hipSuccess) rc = bfail(GKB_ERR_HIP, "event sync");
      float ms = 0.f;
      if (rc == GKB_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = bfail(GKB_ERR_HIP, "event time");
      gkb_batched_plan_destroy(plan);
      if (rc != GKB_OK) break;
      t = ms;
      if (t < best) {
        best = t;
        *best_threads = cand_threads[c];
        *best_workgroups = o.workgroups;
        if (best_form) *best_form = o.form;
        if (best_max_team) *best_max_team = o.max_team;
      }
    }
    if (times_ms) times_ms[n] = t;
    ++n;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (ncand) *ncand = n;
  return rc;
}

gkb_status gkb_partial_svd_batched(int batch, const gkb_matrix* As, const int* r, const int* k, double tol,
                                   int max_restarts, const gkb_batch_options* opt, void* workspace,
                                   size_t ws_bytes, double* sigma, float* U, float* V, int* info,
                                   void* stream) {
  gkb_batch_plan plan = nullptr;
  gkb_status rc = gkb_batched_plan_create(batch, As, r, k, tol, max_restarts, opt, workspace, ws_bytes, sigma, U,
                                          V, stream, &plan);
  if (rc != GKB_OK) return rc;
  rc = gkb_batched_plan_run(plan, stream);
  if (rc == GKB_OK && info) rc = gkb_batched_plan_info(plan, info, stream);
  if (rc == GKB_OK && !info) {
    if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
      rc = bfail(GKB_ERR_HIP, "stream synchronisation failed");
  }
  gkb_batched_plan_destroy(plan);
  return rc;
}

}  // extern "C"
