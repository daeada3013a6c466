// Host float64 SVD of the small projected matrix and the inertia count used by
// the numerical-rank path.
//
// Dense SVD: Householder reduction to upper bidiagonal form, then implicit
// Wilkinson-shift QR sweeps on the bidiagonal (Golub and Kahan 1965, Golub and
// Reinsch 1970; the sweep is the "Golub-Kahan SVD step" of Golub and Van Loan,
// Matrix Computations, Section 8.6).  The projected matrix of the paper's
// Algorithm 2 is at most a few hundred on a side, so this is plain scalar
// code; rotations are applied to contiguous columns so the compiler
// vectorises them.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gkb_internal.h"

namespace gkb {
namespace {

// Householder vector: returns beta and overwrites x with v (v[0] adjusted) so
// that (I - beta v v^T) x_original = alpha e_1; *alpha_out gets alpha.
double householder(double* x, int len, double* alpha_out) {
  double sigma = 0.0;
  for (int i = 1; i < len; ++i) sigma += x[i] * x[i];
  double x0 = x[0];
  if (sigma == 0.0) {
    *alpha_out = x0;
    return 0.0;
  }
  double nrm = std::sqrt(x0 * x0 + sigma);
  double alpha = (x0 >= 0.0) ? -nrm : nrm;
  x[0] = x0 - alpha;
  double vtv = x[0] * x[0] + sigma;
  *alpha_out = alpha;
  return 2.0 / vtv;
}

inline void rot_cols(double* a, double* b, int len, double c, double s) {
  // a <- c a + s b ; b <- -s a + c b
  for (int i = 0; i < len; ++i) {
    double x = a[i], y = b[i];
    a[i] = c * x + s * y;
    b[i] = -s * x + c * y;
  }
}

inline void givens(double y, double z, double* c, double* s, double* r) {
  if (z == 0.0) {
    *c = 1.0;
    *s = 0.0;
    *r = y;
    return;
  }
  // sqrt(y^2 + z^2) where the squares cannot overflow (std::hypot, which
  // guards every input, costs tens of nanoseconds and the sweeps make two
  // rotations per step)
  const double big = std::max(std::fabs(y), std::fabs(z));
  const double h = (big < 1e150 && big > 1e-150) ? std::sqrt(y * y + z * z) : std::hypot(y, z);
  *c = y / h;
  *s = z / h;
  *r = h;
}

// Implicit-shift QR sweeps on the upper bidiagonal (d[0..N), e[0..N-1)).
// Rotations are accumulated into the rows of Ut (N x M) and Vt (N x N) when
// those are non-null (Ut may carry any M columns of the left factor, e.g. one
// row of the left singular vectors, with Vt null).  On return d holds the singular values, sorted
// descending and non-negative (rows of Ut/Vt permuted and signed to match).
bool bidiag_qr(int N, double* d, double* e, double* Ut, int M, double* Vt) {
  const bool vec = Ut != nullptr;
  if (N == 1) {
    if (d[0] < 0) {
      d[0] = -d[0];
      if (Vt) Vt[0] = -Vt[0];
    }
    return true;
  }
  const double eps = 2.220446049250313e-16;
  double anorm = 0.0;
  for (int i = 0; i < N; ++i)
    anorm = std::max(anorm, std::fabs(d[i]) + (i < N - 1 ? std::fabs(e[i]) : 0.0));
  const double dzero = eps * anorm;
  long iters = 0;
  const long max_iters = 75L * N * N + 100;
  int hi = N - 1;
  while (hi > 0) {
    if (++iters > max_iters) return false;
    // deflate converged superdiagonals at the bottom
    if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi])) ||
        std::fabs(e[hi - 1]) <= dzero * 1e-3) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0) {
      if (std::fabs(e[lo - 1]) <= eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo])) ||
          std::fabs(e[lo - 1]) <= dzero * 1e-3) {
        e[lo - 1] = 0.0;
        break;
      }
      --lo;
    }
    // a (numerically) zero diagonal entry splits the block
    int zi = -1;
    for (int i = lo; i <= hi; ++i)
      if (std::fabs(d[i]) <= dzero) {
        zi = i;
        break;
      }
    if (zi >= 0) {
      d[zi] = 0.0;
      if (zi < hi) {
        // zero row zi's superdiagonal by left rotations with rows zi+1..hi
        double xv = e[zi];
        e[zi] = 0.0;
        for (int j = zi + 1; j <= hi; ++j) {
          double c, s, r;
          givens(d[j], xv, &c, &s, &r);
          d[j] = r;
          if (vec) rot_cols(&Ut[(size_t)j * M], &Ut[(size_t)zi * M], M, c, s);
          if (j < hi) {
            xv = -s * e[j];
            e[j] = c * e[j];
          }
        }
      } else {
        // zero column hi's superdiagonal by right rotations with columns hi-1..lo
        double xv = e[hi - 1];
        e[hi - 1] = 0.0;
        for (int j = hi - 1; j >= lo; --j) {
          double c, s, r;
          givens(d[j], xv, &c, &s, &r);
          d[j] = r;
          if (Vt) rot_cols(&Vt[(size_t)j * N], &Vt[(size_t)hi * N], N, c, s);
          if (j > lo) {
            xv = -s * e[j - 1];
            e[j - 1] = c * e[j - 1];
          }
        }
      }
      continue;
    }
    // Wilkinson shift from the trailing 2x2 of B^T B on [lo, hi]
    double t11 = d[hi - 1] * d[hi - 1] + (hi - 1 > lo ? e[hi - 2] * e[hi - 2] : 0.0);
    double t12 = d[hi - 1] * e[hi - 1];
    double t22 = d[hi] * d[hi] + e[hi - 1] * e[hi - 1];
    double dl = 0.5 * (t11 - t22);
    double den = dl + (dl >= 0 ? 1.0 : -1.0) * std::hypot(dl, t12);
    double mu = (den != 0.0) ? t22 - t12 * t12 / den : t22;
    double y = d[lo] * d[lo] - mu;
    double z = d[lo] * e[lo];
    for (int kk = lo; kk < hi; ++kk) {
      double c, s, r;
      // right rotation on columns kk, kk+1
      givens(y, z, &c, &s, &r);
      if (kk > lo) e[kk - 1] = r;
      double dk = d[kk], ek = e[kk], dk1 = d[kk + 1];
      d[kk] = c * dk + s * ek;
      e[kk] = -s * dk + c * ek;
      double bulge = s * dk1;
      d[kk + 1] = c * dk1;
      if (Vt) rot_cols(&Vt[(size_t)kk * N], &Vt[(size_t)(kk + 1) * N], N, c, s);
      // left rotation on rows kk, kk+1
      givens(d[kk], bulge, &c, &s, &r);
      d[kk] = r;
      ek = e[kk];
      dk1 = d[kk + 1];
      e[kk] = c * ek + s * dk1;
      d[kk + 1] = -s * ek + c * dk1;
      if (vec) rot_cols(&Ut[(size_t)kk * M], &Ut[(size_t)(kk + 1) * M], M, c, s);
      if (kk + 1 < hi) {
        y = e[kk];
        z = s * e[kk + 1];
        e[kk + 1] = c * e[kk + 1];
      }
    }
  }
  // non-negative singular values, sorted descending
  for (int i = 0; i < N; ++i)
    if (d[i] < 0) {
      d[i] = -d[i];
      if (Vt)
        for (int t = 0; t < N; ++t) Vt[(size_t)i * N + t] = -Vt[(size_t)i * N + t];
    }
  for (int i = 0; i < N - 1; ++i) {
    int best = i;
    for (int j = i + 1; j < N; ++j)
      if (d[j] > d[best]) best = j;
    if (best != i) {
      std::swap(d[i], d[best]);
      if (vec) std::swap_ranges(&Ut[(size_t)i * M], &Ut[(size_t)i * M] + M, &Ut[(size_t)best * M]);
      if (Vt) std::swap_ranges(&Vt[(size_t)i * N], &Vt[(size_t)i * N] + N, &Vt[(size_t)best * N]);
    }
  }
  return true;
}

// SVD of a tall M x N (M >= N) row-major matrix W.  Outputs: d (N), Ut (N x M:
// row j is left vector j), Vt (N x N: row j is right vector j).
bool svd_tall(int M, int N, std::vector<double>& W, std::vector<double>& d,
              std::vector<double>& Ut, std::vector<double>& Vt) {
  std::vector<double> e(std::max(N - 1, 1), 0.0);
  d.assign(N, 0.0);
  std::vector<std::vector<double>> vl(N), vr(N);
  std::vector<double> bl(N, 0.0), br(N, 0.0);
  std::vector<double> x;
  // --- Householder bidiagonalisation: W = U B V^T, B upper bidiagonal.
  for (int j = 0; j < N; ++j) {
    int len = M - j;
    x.assign(len, 0.0);
    for (int i = 0; i < len; ++i) x[i] = W[(size_t)(j + i) * N + j];
    double alpha;
    double beta = householder(x.data(), len, &alpha);
    vl[j] = x;
    bl[j] = beta;
    if (beta != 0.0) {
      for (int c = j; c < N; ++c) {
        double dot = 0.0;
        for (int i = 0; i < len; ++i) dot += x[i] * W[(size_t)(j + i) * N + c];
        dot *= beta;
        for (int i = 0; i < len; ++i) W[(size_t)(j + i) * N + c] -= dot * x[i];
      }
    }
    d[j] = alpha;
    if (j < N - 1) {
      int lr = N - j - 1;
      x.assign(lr, 0.0);
      for (int i = 0; i < lr; ++i) x[i] = W[(size_t)j * N + j + 1 + i];
      double a2;
      double b2 = householder(x.data(), lr, &a2);
      vr[j] = x;
      br[j] = b2;
      if (b2 != 0.0) {
        for (int rrow = j; rrow < M; ++rrow) {
          double* row = &W[(size_t)rrow * N + j + 1];
          double dot = 0.0;
          for (int i = 0; i < lr; ++i) dot += row[i] * x[i];
          dot *= b2;
          for (int i = 0; i < lr; ++i) row[i] -= dot * x[i];
        }
      }
      e[j] = a2;
    }
  }
  // --- Accumulate U (stored transposed: Ut[c][i] = U[i][c]) and V.
  Ut.assign((size_t)N * M, 0.0);
  for (int c = 0; c < N; ++c) Ut[(size_t)c * M + c] = 1.0;
  for (int j = N - 1; j >= 0; --j) {
    if (bl[j] == 0.0) continue;
    const std::vector<double>& v = vl[j];
    int len = M - j;
    for (int c = 0; c < N; ++c) {
      double* col = &Ut[(size_t)c * M + j];
      double dot = 0.0;
      for (int i = 0; i < len; ++i) dot += v[i] * col[i];
      dot *= bl[j];
      for (int i = 0; i < len; ++i) col[i] -= dot * v[i];
    }
  }
  Vt.assign((size_t)N * N, 0.0);
  for (int c = 0; c < N; ++c) Vt[(size_t)c * N + c] = 1.0;
  for (int j = N - 2; j >= 0; --j) {
    if (br[j] == 0.0) continue;
    const std::vector<double>& v = vr[j];
    int len = N - j - 1;
    for (int c = 0; c < N; ++c) {
      double* col = &Vt[(size_t)c * N + j + 1];
      double dot = 0.0;
      for (int i = 0; i < len; ++i) dot += v[i] * col[i];
      dot *= br[j];
      for (int i = 0; i < len; ++i) col[i] -= dot * v[i];
    }
  }
  if (!bidiag_qr(N, d.data(), e.data(), Ut.data(), M, Vt.data())) return false;
  return true;
}

}  // namespace

bool dense_svd(int nq, int np, const double* H, double* s, double* X, double* Y) {
  const bool wide = nq < np;
  const int M = wide ? np : nq;
  const int N = wide ? nq : np;
  std::vector<double> W((size_t)M * N);
  for (int i = 0; i < nq; ++i)
    for (int j = 0; j < np; ++j) {
      double v = H[(size_t)i * np + j];
      if (!std::isfinite(v)) return false;
      if (wide)
        W[(size_t)j * N + i] = v;
      else
        W[(size_t)i * N + j] = v;
    }
  std::vector<double> d, Ut, Vt;
  if (!svd_tall(M, N, W, d, Ut, Vt)) return false;
  for (int c = 0; c < N; ++c) s[c] = d[c];
  // tall: H = U diag V^T -> X = U (nq x N), Y = V (np x N)
  // wide: H^T = U diag V^T -> X = V (nq x N), Y = U (np x N)
  const std::vector<double>& XL = wide ? Vt : Ut;
  const std::vector<double>& YL = wide ? Ut : Vt;
  const int xrows = nq, yrows = np;
  for (int c = 0; c < N; ++c) {
    for (int i = 0; i < xrows; ++i) X[(size_t)i * N + c] = XL[(size_t)c * xrows + i];
    for (int i = 0; i < yrows; ++i) Y[(size_t)i * N + c] = YL[(size_t)c * yrows + i];
  }
  return true;
}

bool bidiag_singular_values(int nq, int np, const double* alpha, const double* beta, double* s) {
  // Lower bidiagonal (nq x np, nq in {np, np+1}) -> upper bidiagonal by left
  // rotations of rows (j, j+1), then QR sweeps without vectors.
  if (np <= 0) return true;
  std::vector<double> d(alpha, alpha + np), e(std::max(np - 1, 1), 0.0);
  for (int j = 0; j < np; ++j) {
    if (!std::isfinite(d[j])) return false;
    if (j + 1 >= nq) break;
    double b = beta[j];
    if (!std::isfinite(b)) return false;
    double c, sn, r;
    givens(d[j], b, &c, &sn, &r);
    d[j] = r;
    if (j + 1 < np) {
      e[j] = sn * d[j + 1];
      d[j + 1] = c * d[j + 1];
    }
  }
  if (!bidiag_qr(np, d.data(), e.data(), nullptr, 0, nullptr)) return false;
  for (int j = 0; j < np; ++j) s[j] = d[j];
  return true;
}

bool bidiag_sv_lastrow(int np, const double* alpha, const double* beta, double* s, double* last) {
  // The (np + 1) x np lower bidiagonal B is G^T [B_up; 0] with G the row
  // rotations (j, j+1) that make it upper bidiagonal, so the last row of its
  // left singular vectors is (G e_last)^T [U_up; 0]: G e_last has entries only
  // at np - 1 (the last rotation's sine) and np.  That one row of left factor
  // is then carried through the QR sweeps as a single column.
  if (np <= 0) return true;
  std::vector<double> d(alpha, alpha + np), e(std::max(np - 1, 1), 0.0), u(np, 0.0);
  double sn_last = 0.0;
  for (int j = 0; j < np; ++j) {
    if (!std::isfinite(d[j]) || !std::isfinite(beta[j])) return false;
    double c, sn, r;
    givens(d[j], beta[j], &c, &sn, &r);
    d[j] = r;
    if (j + 1 < np) {
      e[j] = sn * d[j + 1];
      d[j + 1] = c * d[j + 1];
    } else {
      sn_last = sn;
    }
  }
  u[np - 1] = sn_last;
  if (!bidiag_qr(np, d.data(), e.data(), u.data(), 1, nullptr)) return false;
  for (int j = 0; j < np; ++j) {
    s[j] = d[j];
    last[j] = u[j];
  }
  return true;
}

int64_t bidiag_count_above(int nq, int np, const double* alpha, const double* beta, double tau) {
  // Off-diagonal of the zero-diagonal Golub-Kahan tridiagonal:
  // alpha_1, beta_2, alpha_2, beta_3, ...; its eigenvalues are +-sigma_i and
  // zeros, so the number above tau > 0 equals #{sigma_i > tau}.  Sylvester
  // inertia of T - tau I = L D L^T counts eigenvalues below tau.
  std::vector<double> off;
  off.reserve((size_t)nq + np);
  for (int j = 0; j < np; ++j) {
    off.push_back(alpha[j]);
    if (j + 1 < nq) off.push_back(beta[j]);
  }
  const int64_t order = (int64_t)off.size() + 1;
  const double tiny = 2.2250738585072014e-308;
  int64_t below = 0;
  double dd = -tau;
  if (dd < 0) ++below;
  for (double e : off) {
    if (dd == 0.0) dd = -tiny;
    dd = -tau - e * e / dd;
    if (dd < 0) ++below;
  }
  return order - below;
}

}  // namespace gkb
