// Full reorthogonalisation of a new Golub-Kahan vector (Algorithm 1's
// projection steps, run twice: classical Gram-Schmidt with one repetition)
// in three launches, plus the norm partials that the normalisation reads.
// All launches go to the given stream; none allocates or synchronises.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gkb {

// Row split of a vector over the Gram-Schmidt workgroups: G workgroups, each
// owning `rows` consecutive entries (the last one fewer).  At most GS_MAX_G
// workgroups of at least 256 rows, unless that would exceed GS_MAX_ROWS rows
// each (the slice a workgroup keeps in LDS).
constexpr int GS_MAX_G = 256;
constexpr int GS_MAX_ROWS = 8192;
struct GsSplit {
  int G;
  int64_t rows;
};
GsSplit gs_split(int64_t len);
// Rows of ldh doubles launch_gs2 needs in gsp for a vector of length len:
// two sets of slice partials or the column-spread form's chunk partials,
// whichever is larger, plus one row for the reduced coefficients.
int64_t gs_partial_rows(int64_t len);

// What the first launch does before its dot products.
enum GsPre {
  GS_PRE_NONE = 0,  // x is given
  GS_PRE_RHO = 1,   // x -= V[:, 0..l) rho            (first step after a thick restart)
  GS_PRE_TSUM = 2,  // x = sum_p part[p][i] - coef[cidx] prev[i]   (A^T q from its row-block partials)
  GS_PRE_FIX = 3    // only if run_if[0] != 0: g = sum_p part[p][i] (double), gcol[i] = g,
                    // x = g - coef[cidx] prev[i]; else x is given (one sweep of A per step:
                    // a recovered A^T q column replaced by its direct recomputation)
};
struct GsPreArgs {
  const double* rho = nullptr;  // GS_PRE_RHO: l coefficients
  int l = 0;
  const void* part = nullptr;   // GS_PRE_TSUM: nparts x ldpart partial sums (float or double)
  int64_t ldpart = 0;
  int nparts = 0;
  int part_f64 = 0;             // 1: part is double, 0: float
  const void* prev = nullptr;   // GS_PRE_TSUM: previous basis vector (basis type) or NULL
  const double* coef = nullptr;
  int cidx = 0;
  const int* run_if = nullptr;  // GS_PRE_FIX
  double* gcol = nullptr;       // GS_PRE_FIX
};

// x (double, len) <- x - V h1 - V h2 with h1 = V^T x and h2 = V^T (x - V h1),
// V = the first t columns (basis type TB, column-major, leading dimension ldv).
//   first:  optional pre-step, then each workgroup's partial dots P1 of its slice
//   reduce: h1 = sum of P1 in a fixed order (a wave per coefficient)
//   mid:    slice -= V h1, then the partial dots P2 of the updated slice (the
//           basis slice staged in LDS when it fits: read once for both uses)
//   reduce: h2 = sum of P2
//   last:   slice -= V h2, npart[b] = sum of x^2 over workgroup b's slice
// acc (optional): acc[0..t) = h1 + h2.  gsp: gs_partial_rows(len) x ldh doubles
// (ldh >= t).  Every launch returns
// at once when flag[0] != 0.  t = 0: only the pre-step and the norm partials.
// *nparts (if given) receives the number of norm partials written to npart
// (what the normalisation must add up): gs_split(len).G, or update_blocks(len)
// when the passes spread the columns over workgroups (short vectors, see
// reorth.hip).  npart must hold max(G, update_blocks(len)) doubles.
template <typename TB>
hipError_t launch_gs2(const TB* V, int64_t ldv, int t, int64_t len, double* x, double* gsp, int ldh,
                      double* npart, double* acc, int pre_kind, const GsPreArgs& pre, const int* flag,
                      hipStream_t st, int* nparts = nullptr);

}  // namespace gkb
