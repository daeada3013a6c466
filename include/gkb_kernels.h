/*
 * gkb_kernels.h -- building blocks of the Golub-Kahan path, exposed on their
 * own so each can be checked and timed in isolation.  Same conventions as
 * gkb.h: device pointers unless stated, caller-owned memory, all work on
 * `stream`, validation before any device work.
 */
#ifndef GKB_KERNELS_H
#define GKB_KERNELS_H

#include "gkb.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Workspace bytes for gkb_matvec with trans = 1 (0 if A is invalid). */
size_t gkb_matvec_workspace_size(const gkb_matrix* A);

/*
 * The two products of Bidiag 1 (eq. (2.2); Algorithm 1's A p and A^T q):
 *   trans = 0:  y (m doubles) = A x,   x: n elements
 *   trans = 1:  y (n doubles) = A^T x, x: m elements, through the workspace
 *               (deterministic two-phase reduction over row blocks).
 * x is double for GKB_F64 and float for GKB_F32 / GKB_BF16; products
 * accumulate in the matrix's precision class (double for GKB_F64, float
 * otherwise) and the final sums are converted to double.
 */
gkb_status gkb_matvec(const gkb_matrix* A, int trans, const void* x, double* y, void* workspace,
                      size_t ws_bytes, void* stream);

/*
 * Both products of a Golub-Kahan step in one sweep of A: w = A p (m doubles)
 * and y = A^T w (n doubles), every sum in float64 (A float32 or bfloat16,
 * row-major, lda and n multiples of 4 (float32) or 8 (bfloat16), A 16-byte
 * aligned, n <= 262144; p float32, n entries).  A workgroup streams a range
 * of rows once, reducing each row's dot product before adding the row, scaled
 * by it, into its partial of A^T w; rows longer than 24576 are split into
 * slices of at most 8192 (float32) or 16384 (bfloat16) columns, one per
 * workgroup of a team, whose members exchange their parts of each row's dot
 * product through the workspace.  float64 A is rejected here (p is float32);
 * the solvers' one_pass option takes it.  The
 * partials (in gkb_matvec_fused_workspace_size bytes, with the teams'
 * exchange area, which each call zeroes first) are added in a fixed order, so
 * results are reproducible.  A^T q of the next Lanczos vector then follows
 * from y and the recurrence (eq. (2.2)).  A team's members must all be
 * resident at once (one workgroup per compute unit at most); if the device is
 * not free for the whole grid, a member stops waiting after about a second
 * and its outputs are NaN.  Returns GKB_ERR_INVALID for other shapes.
 */
size_t gkb_matvec_fused_workspace_size(const gkb_matrix* A);
gkb_status gkb_matvec_fused(const gkb_matrix* A, const float* p, double* w, double* y, void* workspace,
                            size_t ws_bytes, void* stream);

/*
 * C (M x N) = A (M x K) B (K x N), all column-major with leading dimensions
 * lda >= M, ldb >= K, ldc >= M, on the 16x16x4 MFMA (float64 or float32).
 * This is the Ritz-vector product V = P Y, U = Q X of Algorithm 2 (and the
 * restart products).  dtype is GKB_F64 or GKB_F32.  All pointers are device
 * pointers owned by the caller; A and B may be NULL when K = 0 (C is then
 * zero-filled).  Columns whose start is 16-byte aligned (lda, ldc multiples
 * of 16 bytes and aligned base pointers) are moved with 16-byte accesses.
 * Returns GKB_ERR_INVALID for negative sizes or too-small leading dimensions.
 */
gkb_status gkb_gemm_tall(gkb_dtype dtype, const void* A, int64_t lda, int64_t M, int K, const void* B,
                         int64_t ldb, int N, void* C, int64_t ldc, void* stream);

/*
 * C (M x N, column-major, ldc >= M) = A (M x K, row-major, lda >= K) *
 * B (K x N, column-major, ldb >= K), float32 on the 16x16x4 MFMA with the
 * A and B tiles staged in LDS (the next K chunk loading during the MFMAs).
 * The block product of the Rayleigh-Ritz refinement (W = A V, eq. (5)) and
 * of the sketch A Omega.  C is overwritten and must not overlap A or B.  For
 * N <= 32 the two halves of the K range are added into C (zeroed first) by
 * float atomics; with two addends on zero the sum does not depend on their
 * order, so results are reproducible.  Device pointers owned by the caller.
 */
gkb_status gkb_gemm_rowmajor(const float* A, int64_t lda, int64_t M, int64_t K, const float* B, int64_t ldb,
                             int N, float* C, int64_t ldc, void* stream);

/* Workspace bytes (float64 partial sums) for gkb_gram. */
size_t gkb_gram_workspace_size(int64_t m, int d);

/*
 * G (d x d, row-major float64) = W^T W for a column-major float32 W (m x d,
 * ldw >= m); float64 products and sums on the MFMA, deterministic order.
 */
gkb_status gkb_gram(const float* W, int64_t ldw, int64_t m, int d, double* G, void* workspace, size_t ws_bytes,
                    void* stream);

/*
 * bfloat16 storage of a float32 matrix: dst = RNE(src), row-major m x n
 * (leading dimensions lds, ldd >= n).  NaN stays NaN (quiet).
 */
gkb_status gkb_cast_bf16(const float* src, int64_t lds, int64_t m, int64_t n, uint16_t* dst, int64_t ldd,
                         void* stream);

/*
 * The random start of Algorithm 1, q ~ N(2, 1)^m, drawn on the device:
 * Philox4x32-10 (Salmon et al., SC 2011) with counter (i, 0, 0, 0) and key
 * (seed low, seed high) gives 32-bit words x0, x1; u_j = (x_j + 1) 2^-32;
 * q_i = 2 + sqrt(-2 ln u0) cos(2 pi u1).  This is what gkb_partial_svd and
 * gkb_numerical_rank use when opt->q1 is NULL.
 */
gkb_status gkb_start_vector(double* q, int64_t m, uint64_t seed, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* GKB_KERNELS_H */
