/*
 * gkb_sparse.h -- the partial SVD of a sparse matrix.
 *
 * The method needs A only through the two products A p and A^T q of the
 * bidiagonalization recurrences (eq. (2.1)-(2.2)); the paper states its cost
 * for a sparse or dense A (Section 3, complexity).  Here A is float32 in
 * compressed sparse row form, given twice by the caller: the CSR arrays of A
 * and the CSR arrays of A^T (= CSC of A), so that both products read their
 * matrix row by row with contiguous loads and no atomics.  Everything after
 * the products (two Gram-Schmidt passes, small SVDs, thick restart, Ritz
 * vectors, the convergence rule, statuses and statistics) is the float32
 * path of gkb_partial_svd (gkb.h).
 *
 * A plan bins the rows of A and of A^T by length (<= 32, <= 256, <= 2048,
 * longer) so that each bin runs with a matching number of lanes per row
 * (4, 16, 64 or a 256-thread workgroup); the bins keep row order.  Every row
 * sum has a fixed order, so results are bitwise reproducible.
 *
 * Pointers in gkb_csr are device pointers owned by the caller and must stay
 * valid while a plan that refers to them is used.  Column (row) indices must
 * lie in [0, n) ([0, m)); duplicate entries are summed.  The plan keeps the
 * caller's plan workspace (bins) and must be destroyed before it is freed.
 */
#ifndef GKB_SPARSE_H
#define GKB_SPARSE_H

#include "gkb.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int64_t m, n, nnz;
  const int64_t* row_ptr;   /* m + 1 offsets of the rows of A                 */
  const int32_t* col_idx;   /* nnz column indices                             */
  const float* val;         /* nnz values                                      */
  const int64_t* col_ptr;   /* n + 1 offsets of the rows of A^T                */
  const int32_t* row_idx;   /* nnz row indices (of A)                          */
  const float* val_t;       /* nnz values, in A^T row order                    */
} gkb_csr;

typedef struct gkb_sparse_plan_s* gkb_sparse_plan;

/* Device bytes the plan needs for its row bins (0 if A is invalid). */
size_t gkb_sparse_plan_workspace_size(const gkb_csr* A);

/* Device bytes of a plan that also keeps A and A^T in column panels (0 if A
   is invalid): the columns cut into panels of 28672, each panel stored as the
   CSR matrix of its columns with 16-bit panel-relative indices (6 bytes per
   entry), its row offsets (4 bytes per row and panel) and per-panel row sums
   (4 bytes per row and panel).  A workgroup holds one panel of the input
   vector in LDS while it streams that panel's entries, so the products read
   the input vector from LDS instead of gathering it from memory.  A
   direction is kept in panels when it has one panel or at most 4 row
   segments per entry (rows x panels <= 4 nnz), and nnz < 2^31 - 1; otherwise
   it keeps the CSR products. */
size_t gkb_sparse_panel_workspace_size(const gkb_csr* A);

/* Validate A, bin the rows of A and A^T on the device (row_ptr, col_ptr must
   be non-decreasing from 0 to nnz), and read the bin sizes back (one
   synchronisation of `stream`).  ws must be 256-byte aligned.  With at least
   gkb_sparse_panel_workspace_size(A) bytes the plan also builds the column
   panels on the host from copies of the arrays (one more synchronisation per
   direction) and the products of those directions run through them (their
   CSR arrays are not read again).  The panel products add each row's
   entries of a panel in their CSR order and the panel sums in panel order:
   a different, equally fixed order than the CSR products (results differ
   from theirs by rounding only). */
gkb_status gkb_sparse_plan_create(const gkb_csr* A, void* ws, size_t ws_bytes, void* stream,
                                  gkb_sparse_plan* plan);
void gkb_sparse_plan_destroy(gkb_sparse_plan plan);

/* Which products run through column panels: bit 0 A p, bit 1 A^T q. */
int gkb_sparse_plan_panels(gkb_sparse_plan plan);

/* y = A x (trans = 0; x length n, y length m) or y = A^T x (trans = 1):
   x float32, y float64, both device; float32 products summed per row in a
   fixed order, the sum converted to double. */
gkb_status gkb_sparse_matvec(gkb_sparse_plan plan, int trans, const float* x, double* y, void* stream);

/* Workspace of gkb_partial_svd_sparse (0 if the sizes are invalid). */
size_t gkb_sparse_workspace_size(gkb_sparse_plan plan, int r, int k);

/* Top-r singular triplets of the sparse A, exactly as gkb_partial_svd with a
   GKB_F32 matrix: U device float32 m x r, V device float32 n x r (column-major),
   sigma host doubles.  Same statuses, options and statistics. */
gkb_status gkb_partial_svd_sparse(gkb_sparse_plan plan, int r, int k, double tol, int max_restarts,
                                  const gkb_options* opt, void* workspace, size_t ws_bytes, double* sigma,
                                  float* U, float* V, gkb_stats* stats, void* stream);

const char* gkb_sparse_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
