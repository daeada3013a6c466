// Host-only exercise of the library's small float64 SVD code (dense SVD,
// bidiagonal values, last-row screening SVD, inertia count) for the
// sanitizer test: random and degenerate inputs of several shapes; exits
// non-zero when a factorisation does not reproduce its input.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "gkb_internal.h"

static int failures = 0;
static void check(bool ok, const char* what, int a, int b) {
  if (!ok) {
    std::fprintf(stderr, "FAIL %s (%d, %d)\n", what, a, b);
    ++failures;
  }
}

int main() {
  std::mt19937_64 rng(7);
  std::normal_distribution<double> nd(0.0, 1.0);
  const int shapes[][2] = {{1, 1}, {2, 1}, {1, 3}, {5, 4}, {31, 30}, {40, 55}, {71, 70}, {121, 120}};
  for (const auto& sh : shapes) {
    const int nq = sh[0], np = sh[1], kk = nq < np ? nq : np;
    for (int kind = 0; kind < 3; ++kind) {
      std::vector<double> H((size_t)nq * np, 0.0), s(kk), X((size_t)nq * kk), Y((size_t)np * kk);
      for (int i = 0; i < nq; ++i)
        for (int j = 0; j < np; ++j) {
          if (kind == 0) H[(size_t)i * np + j] = nd(rng);
          if (kind == 1 && (i == j || i == j + 1)) H[(size_t)i * np + j] = std::pow(0.9, j) * (1.0 + 0.1 * nd(rng));
          // kind 2: the zero matrix
        }
      const bool ok = gkb::dense_svd(nq, np, H.data(), s.data(), X.data(), Y.data());
      check(ok, "dense_svd converged", nq, np);
      double err = 0.0, scale = 1e-300;
      for (int c = 0; c < kk; ++c) scale = std::fmax(scale, s[c]);
      for (int i = 0; i < nq; ++i)
        for (int j = 0; j < np; ++j) {
          double v = 0.0;
          for (int c = 0; c < kk; ++c) v += X[(size_t)i * kk + c] * s[c] * Y[(size_t)j * kk + c];
          err = std::fmax(err, std::fabs(v - H[(size_t)i * np + j]));
        }
      check(kind == 2 ? err == 0.0 : err <= 1e-12 * scale, "dense_svd reproduces H", nq, np);
    }
  }
  for (int np : {1, 2, 7, 50, 70, 120}) {
    std::vector<double> a(np), b(np), s(np), last(np), s2(np);
    for (int j = 0; j < np; ++j) {
      a[j] = std::pow(0.95, j) * (1.0 + 0.1 * std::fabs(nd(rng)));
      b[j] = 0.3 * std::fabs(nd(rng));
    }
    check(gkb::bidiag_sv_lastrow(np, a.data(), b.data(), s.data(), last.data()), "lastrow", np, 0);
    check(gkb::bidiag_singular_values(np + 1, np, a.data(), b.data(), s2.data()), "bidiag values", np, 0);
    for (int j = 0; j < np; ++j) check(std::fabs(s[j] - s2[j]) <= 1e-13 * s2[0], "lastrow values", np, j);
    const int64_t cnt = gkb::bidiag_count_above(np + 1, np, a.data(), b.data(), 0.5 * s2[0]);
    int64_t want = 0;
    for (int j = 0; j < np; ++j) want += s2[j] > 0.5 * s2[0];
    check(cnt == want, "inertia count", np, (int)cnt);
  }
  std::vector<double> Hn = {1.0, NAN, 0.5, 2.0}, s(2), X(4), Y(4);
  check(!gkb::dense_svd(2, 2, Hn.data(), s.data(), X.data(), Y.data()), "NaN rejected", 2, 2);
  std::printf("host svd harness: %d failures\n", failures);
  return failures == 0 ? 0 : 1;
}
