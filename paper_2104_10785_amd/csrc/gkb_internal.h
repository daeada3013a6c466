// Internal declarations shared by the host driver, the host SVD and the
// kernel launchers.  Not part of the public ABI.
#pragma once

#include <cstddef>
#include <cstdint>

namespace gkb {

// Dense float64 SVD H = X diag(s) Y^T of an nq x np row-major matrix;
// X is nq x min(nq,np), Y is np x min(nq,np), both row-major.  False on
// non-finite input or no convergence.
bool dense_svd(int nq, int np, const double* H, double* s, double* X, double* Y);

// Singular values (descending) of the lower bidiagonal with diagonal
// alpha[0..np) and subdiagonal beta[0..nq-1), nq in {np, np+1}; O(np^2).
bool bidiag_singular_values(int nq, int np, const double* alpha, const double* beta, double* s);

// Singular values s (descending) of the (np + 1) x np lower bidiagonal with
// diagonal alpha[0..np) and subdiagonal beta[0..np), and last[i] = the last
// entry of the i-th left singular vector (up to the common sign of the pair);
// O(np^2).
bool bidiag_sv_lastrow(int np, const double* alpha, const double* beta, double* s, double* last);

// #{sigma_i > tau} of the lower bidiagonal (alpha diagonal, beta subdiagonal)
// by Sylvester inertia of its Golub-Kahan tridiagonal.
int64_t bidiag_count_above(int nq, int np, const double* alpha, const double* beta, double tau);

}  // namespace gkb
