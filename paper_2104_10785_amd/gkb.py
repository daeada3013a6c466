"""Python binding of libgkb.so (ctypes): argument marshalling only.

Every step of the computation runs in the HIP library; PyTorch supplies device
memory (tensors) and the stream.  If the library is not built, every call
raises: there is no fallback.

Function names follow the C ABI in include/gkb.h and include/gkb_kernels.h.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgkb.so")

GKB_F64, GKB_F32, GKB_BF16 = 0, 1, 2
STATUS = {0: "GKB_OK", 1: "GKB_NOT_CONVERGED", 2: "GKB_RANK_DEFICIENT", -1: "GKB_ERR_INVALID",
          -2: "GKB_ERR_HIP", -3: "GKB_ERR_NUMERIC", -4: "GKB_ERR_WORKSPACE", -5: "GKB_ERR_TIMEOUT"}


class GkbError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class GkbMatrix(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("lda", C.c_int64), ("dtype", C.c_int),
                ("data", C.c_void_p), ("refine_f32", C.c_void_p), ("lda_refine", C.c_int64)]


class GkbOptions(C.Structure):
    _fields_ = [("keep", C.c_int), ("eps_relative", C.c_int), ("eps_break", C.c_double),
                ("q1", C.c_void_p), ("seed", C.c_uint64), ("refine_dim", C.c_int), ("check_every", C.c_int),
                ("one_pass", C.c_int), ("phase_timing", C.c_int)]


class GkbBatchOptions(C.Structure):
    _fields_ = [("check_every", C.c_int), ("eps_relative", C.c_int), ("eps_break", C.c_double),
                ("seed", C.c_uint64), ("q1_packed", C.c_void_p), ("workgroups", C.c_int), ("no_graph", C.c_int),
                ("threads", C.c_int), ("max_team", C.c_int), ("form", C.c_int),
                ("cost_estimate", C.c_void_p)]


class GkbCsr(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("val", C.c_void_p), ("col_ptr", C.c_void_p), ("row_idx", C.c_void_p),
                ("val_t", C.c_void_p)]


class GkbStats(C.Structure):
    _fields_ = [("nconv", C.c_int), ("restarts", C.c_int), ("breakdown", C.c_int), ("returned", C.c_int),
                ("matvecs", C.c_int64), ("max_res_est", C.c_double), ("sigma1_est", C.c_double),
                ("ms_total", C.c_double), ("ms_host", C.c_double), ("checks", C.c_int),
                ("krylov_dim", C.c_int), ("refined", C.c_int), ("ms_refine", C.c_double),
                ("refreshes", C.c_int), ("ms_matvec", C.c_double), ("ms_reorth", C.c_double),
                ("ms_sync", C.c_double), ("ms_ritz", C.c_double), ("ms_other", C.c_double),
                ("bytes_A", C.c_double), ("one_pass_used", C.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None

EXPORTS = ["gkb_default_options", "gkb_workspace_size", "gkb_partial_svd", "gkb_rank_workspace_size",
           "gkb_numerical_rank", "gkb_status_string", "gkb_last_error", "gkb_host_dense_svd",
           "gkb_host_bidiag_count_above", "gkb_host_bidiag_lastrow", "gkb_matvec_workspace_size", "gkb_matvec", "gkb_gemm_tall",
           "gkb_cast_bf16", "gkb_start_vector", "gkb_gemm_rowmajor", "gkb_gram_workspace_size", "gkb_gram",
           "gkb_batch_default_options", "gkb_batched_workspace_size", "gkb_batched_plan_create",
           "gkb_batched_plan_run", "gkb_batched_plan_info", "gkb_batched_plan_grid", "gkb_batched_plan_destroy",
           "gkb_partial_svd_batched", "gkb_batched_last_error", "gkb_batched_autotune", "gkb_batched_plan_work",
           "gkb_mlp_param_count", "gkb_mlp_feature_stride", "gkb_mlp_workspace_size", "gkb_mlp_features",
           "gkb_mlp_forward", "gkb_mlp_loss_grad", "gkb_adam_step", "gkb_mlp_start_vector",
           "gkb_learned_last_error", "gkb_sparse_plan_workspace_size", "gkb_sparse_panel_workspace_size",
           "gkb_sparse_plan_create", "gkb_sparse_plan_destroy", "gkb_sparse_plan_panels", "gkb_sparse_matvec", "gkb_sparse_workspace_size", "gkb_partial_svd_sparse",
           "gkb_sparse_last_error", "gkb_rsgd_workspace_size", "gkb_rsgd_plan_create", "gkb_rsgd_plan_step",
           "gkb_rsgd_plan_info", "gkb_rsgd_plan_destroy", "gkb_rsgd_weights", "gkb_rsgd_last_error",
           "gkb_matvec_fused_workspace_size", "gkb_matvec_fused", "gkb_mlp_loss_grad_kind", "gkb_partial_svd_noalloc",
           "gkb_svd_plan_create", "gkb_svd_plan_run", "gkb_svd_plan_destroy"]

NOALLOC_SCRATCH_BYTES = 32 << 20


def lib():
    """Load libgkb.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(python -m paper_2104_10785_amd.build)")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    L.gkb_default_options.argtypes = [P(GkbOptions)]
    L.gkb_default_options.restype = None
    L.gkb_workspace_size.argtypes = [P(GkbMatrix), C.c_int, C.c_int, P(GkbOptions)]
    L.gkb_workspace_size.restype = C.c_size_t
    L.gkb_partial_svd.argtypes = [P(GkbMatrix), C.c_int, C.c_int, C.c_double, C.c_int, P(GkbOptions),
                                  C.c_void_p, C.c_size_t, P(C.c_double), C.c_void_p, C.c_void_p,
                                  P(GkbStats), C.c_void_p]
    L.gkb_partial_svd.restype = C.c_int
    L.gkb_partial_svd_noalloc.argtypes = [P(GkbMatrix), C.c_int, C.c_int, C.c_double, C.c_int, P(GkbOptions),
                                          P(C.c_double), C.c_void_p, C.c_void_p, P(GkbStats), C.c_void_p]
    L.gkb_partial_svd_noalloc.restype = C.c_int
    L.gkb_svd_plan_create.argtypes = [P(GkbMatrix), C.c_int, C.c_int, C.c_double, C.c_int, P(GkbOptions),
                                      C.c_void_p, C.c_size_t, P(C.c_void_p)]
    L.gkb_svd_plan_create.restype = C.c_int
    L.gkb_svd_plan_run.argtypes = [C.c_void_p, C.c_void_p, P(C.c_double), C.c_void_p, C.c_void_p, P(GkbStats),
                                   C.c_void_p]
    L.gkb_svd_plan_run.restype = C.c_int
    L.gkb_svd_plan_destroy.argtypes = [C.c_void_p]
    L.gkb_svd_plan_destroy.restype = None
    L.gkb_rank_workspace_size.argtypes = [P(GkbMatrix), C.c_int, P(GkbOptions)]
    L.gkb_rank_workspace_size.restype = C.c_size_t
    L.gkb_numerical_rank.argtypes = [P(GkbMatrix), C.c_double, C.c_int, C.c_int, P(GkbOptions), C.c_void_p,
                                     C.c_size_t, P(C.c_int64), P(C.c_int64), P(C.c_double), P(C.c_int),
                                     P(GkbStats), C.c_void_p]
    L.gkb_numerical_rank.restype = C.c_int
    L.gkb_status_string.argtypes = [C.c_int]
    L.gkb_status_string.restype = C.c_char_p
    L.gkb_last_error.argtypes = []
    L.gkb_last_error.restype = C.c_char_p
    L.gkb_host_dense_svd.argtypes = [C.c_int, C.c_int, P(C.c_double), P(C.c_double), P(C.c_double),
                                     P(C.c_double)]
    L.gkb_host_dense_svd.restype = C.c_int
    L.gkb_host_bidiag_count_above.argtypes = [C.c_int, C.c_int, P(C.c_double), P(C.c_double), C.c_double]
    L.gkb_host_bidiag_count_above.restype = C.c_int64
    L.gkb_host_bidiag_lastrow.argtypes = [C.c_int, P(C.c_double), P(C.c_double), P(C.c_double), P(C.c_double)]
    L.gkb_host_bidiag_lastrow.restype = C.c_int
    L.gkb_matvec_workspace_size.argtypes = [P(GkbMatrix)]
    L.gkb_matvec_workspace_size.restype = C.c_size_t
    L.gkb_matvec.argtypes = [P(GkbMatrix), C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
    L.gkb_matvec.restype = C.c_int
    L.gkb_gemm_tall.argtypes = [C.c_int, C.c_void_p, C.c_int64, C.c_int64, C.c_int, C.c_void_p, C.c_int64,
                                C.c_int, C.c_void_p, C.c_int64, C.c_void_p]
    L.gkb_gemm_tall.restype = C.c_int
    L.gkb_cast_bf16.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_void_p, C.c_int64,
                                C.c_void_p]
    L.gkb_cast_bf16.restype = C.c_int
    L.gkb_start_vector.argtypes = [C.c_void_p, C.c_int64, C.c_uint64, C.c_void_p]
    L.gkb_start_vector.restype = C.c_int
    L.gkb_gemm_rowmajor.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_void_p, C.c_int64, C.c_int,
                                    C.c_void_p, C.c_int64, C.c_void_p]
    L.gkb_gemm_rowmajor.restype = C.c_int
    L.gkb_gram_workspace_size.argtypes = [C.c_int64, C.c_int]
    L.gkb_gram_workspace_size.restype = C.c_size_t
    L.gkb_gram.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int, C.c_void_p, C.c_void_p, C.c_size_t,
                           C.c_void_p]
    L.gkb_gram.restype = C.c_int
    L.gkb_batch_default_options.argtypes = [P(GkbBatchOptions)]
    L.gkb_batch_default_options.restype = None
    L.gkb_batched_workspace_size.argtypes = [C.c_int, P(GkbMatrix), P(C.c_int), P(C.c_int)]
    L.gkb_batched_workspace_size.restype = C.c_size_t
    L.gkb_batched_plan_create.argtypes = [C.c_int, P(GkbMatrix), P(C.c_int), P(C.c_int), C.c_double, C.c_int,
                                          P(GkbBatchOptions), C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_void_p, P(C.c_void_p)]
    L.gkb_batched_plan_create.restype = C.c_int
    L.gkb_batched_plan_run.argtypes = [C.c_void_p, C.c_void_p]
    L.gkb_batched_plan_run.restype = C.c_int
    L.gkb_batched_plan_info.argtypes = [C.c_void_p, P(C.c_int), C.c_void_p]
    L.gkb_batched_plan_info.restype = C.c_int
    L.gkb_batched_plan_grid.argtypes = [C.c_void_p]
    L.gkb_batched_plan_grid.restype = C.c_int
    L.gkb_batched_plan_destroy.argtypes = [C.c_void_p]
    L.gkb_batched_plan_destroy.restype = None
    L.gkb_partial_svd_batched.argtypes = [C.c_int, P(GkbMatrix), P(C.c_int), P(C.c_int), C.c_double, C.c_int,
                                          P(GkbBatchOptions), C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                          C.c_void_p, P(C.c_int), C.c_void_p]
    L.gkb_partial_svd_batched.restype = C.c_int
    L.gkb_batched_plan_work.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.gkb_batched_plan_work.restype = C.c_int
    L.gkb_batched_autotune.argtypes = [C.c_int, P(GkbMatrix), P(C.c_int), P(C.c_int), C.c_double, C.c_int,
                                       P(GkbBatchOptions), C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, P(C.c_int), P(C.c_int), P(C.c_int), P(C.c_int),
                                       P(C.c_double), P(C.c_int)]
    L.gkb_batched_autotune.restype = C.c_int
    L.gkb_batched_last_error.argtypes = []
    L.gkb_batched_last_error.restype = C.c_char_p
    L.gkb_mlp_param_count.argtypes = [C.c_int, C.c_int]
    L.gkb_mlp_param_count.restype = C.c_int64
    L.gkb_mlp_feature_stride.argtypes = []
    L.gkb_mlp_feature_stride.restype = C.c_int
    L.gkb_mlp_workspace_size.argtypes = [C.c_int64, C.c_int, C.c_int, C.c_int]
    L.gkb_mlp_workspace_size.restype = C.c_size_t
    L.gkb_mlp_features.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int, C.c_void_p, C.c_int, C.c_void_p,
                                   C.c_void_p, C.c_size_t, C.c_void_p]
    L.gkb_mlp_features.restype = C.c_int
    L.gkb_mlp_forward.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
    L.gkb_mlp_forward.restype = C.c_int
    L.gkb_mlp_loss_grad.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int64, C.c_void_p, C.c_int,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
    L.gkb_mlp_loss_grad.restype = C.c_int
    L.gkb_adam_step.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_double,
                                C.c_double, C.c_double, C.c_int, C.c_void_p]
    L.gkb_adam_step.restype = C.c_int
    L.gkb_mlp_start_vector.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                       C.c_size_t, C.c_void_p]
    L.gkb_mlp_start_vector.restype = C.c_int
    L.gkb_learned_last_error.argtypes = []
    L.gkb_learned_last_error.restype = C.c_char_p
    L.gkb_sparse_plan_workspace_size.argtypes = [P(GkbCsr)]
    L.gkb_sparse_plan_workspace_size.restype = C.c_size_t
    L.gkb_sparse_panel_workspace_size.argtypes = [P(GkbCsr)]
    L.gkb_sparse_panel_workspace_size.restype = C.c_size_t
    L.gkb_sparse_plan_panels.argtypes = [C.c_void_p]
    L.gkb_sparse_plan_panels.restype = C.c_int
    L.gkb_sparse_plan_create.argtypes = [P(GkbCsr), C.c_void_p, C.c_size_t, C.c_void_p, P(C.c_void_p)]
    L.gkb_sparse_plan_create.restype = C.c_int
    L.gkb_sparse_plan_destroy.argtypes = [C.c_void_p]
    L.gkb_sparse_plan_destroy.restype = None
    L.gkb_sparse_matvec.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
    L.gkb_sparse_matvec.restype = C.c_int
    L.gkb_sparse_workspace_size.argtypes = [C.c_void_p, C.c_int, C.c_int]
    L.gkb_sparse_workspace_size.restype = C.c_size_t
    L.gkb_partial_svd_sparse.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_int, P(GkbOptions),
                                         C.c_void_p, C.c_size_t, P(C.c_double), C.c_void_p, C.c_void_p,
                                         P(GkbStats), C.c_void_p]
    L.gkb_partial_svd_sparse.restype = C.c_int
    L.gkb_sparse_last_error.argtypes = []
    L.gkb_sparse_last_error.restype = C.c_char_p
    L.gkb_rsgd_workspace_size.argtypes = [C.c_int] * 5
    L.gkb_rsgd_workspace_size.restype = C.c_size_t
    L.gkb_rsgd_plan_create.argtypes = [C.c_int] * 5 + [C.c_double, C.c_double] + [C.c_void_p] * 6 + \
        [C.c_void_p, C.c_size_t, C.c_void_p, P(C.c_void_p)]
    L.gkb_rsgd_plan_create.restype = C.c_int
    L.gkb_rsgd_plan_step.argtypes = [C.c_void_p, C.c_void_p]
    L.gkb_rsgd_plan_step.restype = C.c_int
    L.gkb_rsgd_plan_info.argtypes = [C.c_void_p, P(C.c_int), C.c_void_p]
    L.gkb_rsgd_plan_info.restype = C.c_int
    L.gkb_rsgd_plan_destroy.argtypes = [C.c_void_p]
    L.gkb_rsgd_plan_destroy.restype = None
    L.gkb_rsgd_weights.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p]
    L.gkb_rsgd_weights.restype = C.c_int
    L.gkb_rsgd_last_error.argtypes = []
    L.gkb_rsgd_last_error.restype = C.c_char_p
    L.gkb_matvec_fused_workspace_size.argtypes = [P(GkbMatrix)]
    L.gkb_matvec_fused_workspace_size.restype = C.c_size_t
    L.gkb_matvec_fused.argtypes = [P(GkbMatrix), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                   C.c_void_p]
    L.gkb_matvec_fused.restype = C.c_int
    L.gkb_mlp_loss_grad_kind.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int64, C.c_void_p, C.c_int,
                                         C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
    L.gkb_mlp_loss_grad_kind.restype = C.c_int
    _lib = L
    return L


def last_error() -> str:
    return lib().gkb_last_error().decode()


def _check(status: int, allow_positive: bool = True) -> int:
    if status < 0 or (status > 0 and not allow_positive):
        raise GkbError(status, last_error())
    return status


# ------------------------------------------------------------------ helpers
def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return GKB_F64
    if t.dtype == torch.float32:
        return GKB_F32
    if t.dtype == torch.bfloat16:
        return GKB_BF16
    raise TypeError(f"unsupported matrix dtype {t.dtype}")


def basis_dtype(code: int):
    torch = _torch()
    return torch.float64 if code == GKB_F64 else torch.float32


def make_matrix(A, refine=None) -> GkbMatrix:
    """Describe a 2-D device tensor (row-major, unit column stride)."""
    if A.dim() != 2 or A.stride(1) != 1 or not A.is_cuda:
        raise ValueError("A must be a 2-D device tensor with unit column stride")
    mat = GkbMatrix(A.shape[0], A.shape[1], max(A.stride(0), A.shape[1]), _dtype_code(A), A.data_ptr(), None, 0)
    if refine is not None:
        if refine.dtype != _torch().float32 or refine.shape != A.shape or refine.stride(1) != 1:
            raise ValueError("refine must be a float32 device tensor shaped like A")
        mat.refine_f32 = refine.data_ptr()
        mat.lda_refine = max(refine.stride(0), refine.shape[1])
    return mat


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def make_options(q1=None, seed=0, keep=0, eps_break=0.0, eps_relative=True, refine_dim=0,
                 check_every=0, one_pass=False, phase_timing=False) -> GkbOptions:
    o = GkbOptions()
    lib().gkb_default_options(C.byref(o))
    o.keep = keep
    o.eps_relative = 1 if eps_relative else 0
    o.eps_break = eps_break
    o.seed = seed
    o.refine_dim = refine_dim
    o.check_every = check_every
    o.one_pass = 1 if one_pass else 0
    o.phase_timing = 1 if phase_timing else 0
    if q1 is not None:
        if q1.dtype != _torch().float64 or not q1.is_cuda or not q1.is_contiguous():
            raise ValueError("q1 must be a contiguous float64 device tensor")
        o.q1 = q1.data_ptr()
    return o


def _workspace(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# ------------------------------------------------------------------ ABI calls
def gkb_workspace_size(A, r, k, refine=None, **opts) -> int:
    mat = make_matrix(A, refine)
    o = make_options(**opts)
    return int(lib().gkb_workspace_size(C.byref(mat), r, k, C.byref(o)))


def gkb_partial_svd(A, r, k, tol, max_restarts, refine=None, workspace=None, stream=None, **opts):
    """Top-r singular triplets of the device matrix A.

    Returns (sigma, Ut, Vt, status, stats): sigma a numpy array (r, descending),
    Ut (r x m) and Vt (r x n) device tensors whose rows are the singular
    vectors (float64 for a float64 A, float32 otherwise).
    """
    torch = _torch()
    mat = make_matrix(A, refine)
    o = make_options(**opts)
    L = lib()
    need = L.gkb_workspace_size(C.byref(mat), r, k, C.byref(o))
    if need == 0:
        _check(L.gkb_partial_svd(C.byref(mat), r, k, tol, max_restarts, C.byref(o), None, 0,
                                 (C.c_double * max(r, 1))(), None, None, None, None), False)
    if workspace is None:
        workspace = _workspace(need, A.device)
    bt = basis_dtype(mat.dtype)
    Ut = torch.empty((r, A.shape[0]), dtype=bt, device=A.device)
    Vt = torch.empty((r, A.shape[1]), dtype=bt, device=A.device)
    sig = (C.c_double * r)()
    st = GkbStats()
    status = L.gkb_partial_svd(C.byref(mat), r, k, float(tol), int(max_restarts), C.byref(o),
                               C.c_void_p(workspace.data_ptr()), workspace.numel(), sig,
                               C.c_void_p(Ut.data_ptr()), C.c_void_p(Vt.data_ptr()), C.byref(st),
                               _stream(stream))
    _check(status)
    return np.array(sig[:], dtype=np.float64), Ut, Vt, status, st.as_dict()


def gkb_partial_svd_noalloc(A, r, k, tol, max_restarts, refine=None, stream=None, U=None, V=None, **opts):
    """gkb_partial_svd with the library's fixed device array as workspace (no
    workspace argument; nothing allocated by the library).  U, V: optional
    preallocated output tensors (r x m and r x n rows = singular vectors).
    Returns (sigma, Ut, Vt, status, stats) as gkb_partial_svd."""
    torch = _torch()
    mat = make_matrix(A, refine)
    o = make_options(**opts)
    bt = basis_dtype(mat.dtype)
    Ut = U if U is not None else torch.empty((r, A.shape[0]), dtype=bt, device=A.device)
    Vt = V if V is not None else torch.empty((r, A.shape[1]), dtype=bt, device=A.device)
    sig = (C.c_double * max(r, 1))()
    st = GkbStats()
    status = lib().gkb_partial_svd_noalloc(C.byref(mat), r, k, float(tol), int(max_restarts), C.byref(o), sig,
                                           C.c_void_p(Ut.data_ptr()), C.c_void_p(Vt.data_ptr()), C.byref(st),
                                           _stream(stream))
    _check(status)
    return np.array(sig[:r], dtype=np.float64), Ut, Vt, status, st.as_dict()


class SvdPlan:
    """Repeated partial SVDs of one device matrix buffer (gkb_svd_plan_*): the
    stretches of device work between host synchronisations are captured as
    HIP graphs on the first solve that reaches them and replayed afterwards.
    A may be modified in place between solves; results equal gkb_partial_svd's."""

    def __init__(self, A, r, k, tol, max_restarts, refine=None, workspace=None, **opts):
        torch = _torch()
        self.A, self.r, self.refine = A, r, refine
        self.mat = make_matrix(A, refine)
        self.opts = make_options(**opts)
        L = lib()
        need = L.gkb_workspace_size(C.byref(self.mat), r, k, C.byref(self.opts))
        self.ws = workspace if workspace is not None else _workspace(max(need, 256), A.device)
        plan = C.c_void_p()
        _check(L.gkb_svd_plan_create(C.byref(self.mat), r, k, float(tol), int(max_restarts), C.byref(self.opts),
                                     C.c_void_p(self.ws.data_ptr()), self.ws.numel(), C.byref(plan)), False)
        self.plan = plan
        bt = basis_dtype(self.mat.dtype)
        self.Ut = torch.empty((r, A.shape[0]), dtype=bt, device=A.device)
        self.Vt = torch.empty((r, A.shape[1]), dtype=bt, device=A.device)

    def run(self, q1=None, stream=None):
        """One solve; returns (sigma, Ut, Vt, status, stats) like gkb_partial_svd
        (Ut, Vt are the plan's output tensors, overwritten by the next run)."""
        if q1 is not None and (q1.dtype != _torch().float64 or not q1.is_cuda or not q1.is_contiguous()):
            raise ValueError("q1 must be a contiguous float64 device tensor")
        sig = (C.c_double * self.r)()
        st = GkbStats()
        status = lib().gkb_svd_plan_run(self.plan, C.c_void_p(q1.data_ptr()) if q1 is not None else None, sig,
                                        C.c_void_p(self.Ut.data_ptr()), C.c_void_p(self.Vt.data_ptr()),
                                        C.byref(st), _stream(stream))
        _check(status)
        return np.array(sig[:], dtype=np.float64), self.Ut, self.Vt, status, st.as_dict()

    def close(self):
        if self.plan:
            lib().gkb_svd_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gkb_rank_workspace_size(A, k_max=0, **opts) -> int:
    mat = make_matrix(A)
    o = make_options(**opts)
    return int(lib().gkb_rank_workspace_size(C.byref(mat), k_max, C.byref(o)))


def gkb_numerical_rank(A, tau, tau_relative=True, k_max=0, workspace=None, stream=None, **opts):
    """Numerical rank of the device matrix A.

    Returns (rank, rank_sturm, sigma (numpy, singular values of B), status, stats).
    """
    mat = make_matrix(A)
    o = make_options(**opts)
    L = lib()
    kk = k_max if k_max else min(A.shape)
    need = L.gkb_rank_workspace_size(C.byref(mat), k_max, C.byref(o))
    if workspace is None:
        workspace = _workspace(need, A.device)
    rank = C.c_int64()
    rank_s = C.c_int64()
    sig = (C.c_double * max(kk, 1))()
    ns = C.c_int()
    st = GkbStats()
    status = L.gkb_numerical_rank(C.byref(mat), float(tau), 1 if tau_relative else 0, int(k_max), C.byref(o),
                                  C.c_void_p(workspace.data_ptr()), workspace.numel(), C.byref(rank),
                                  C.byref(rank_s), sig, C.byref(ns), C.byref(st), _stream(stream))
    _check(status)
    return rank.value, rank_s.value, np.array(sig[: ns.value]), status, st.as_dict()


def gkb_matvec(A, x, trans, y=None, workspace=None, stream=None):
    """y = A x (trans=0) or A^T x (trans=1) with the library's streaming kernels (y float64)."""
    torch = _torch()
    mat = make_matrix(A)
    L = lib()
    out_len = A.shape[1] if trans else A.shape[0]
    if y is None:
        y = torch.empty(out_len, dtype=torch.float64, device=A.device)
    if workspace is None and trans:
        workspace = _workspace(L.gkb_matvec_workspace_size(C.byref(mat)), A.device)
    wsp = C.c_void_p(workspace.data_ptr()) if workspace is not None else None
    wsz = workspace.numel() if workspace is not None else 0
    _check(L.gkb_matvec(C.byref(mat), int(trans), C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), wsp, wsz,
                        _stream(stream)), False)
    return y


def gkb_gemm_tall(A, B, C_out=None, stream=None):
    """C = A B on MFMA for column-major operands given as transposed tensors:
    A as (K, M) row-major (= M x K column-major), B as (N, K), result (N, M)."""
    torch = _torch()
    K, M = A.shape
    N, K2 = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    code = GKB_F64 if A.dtype == torch.float64 else GKB_F32
    if C_out is None:
        C_out = torch.empty((N, M), dtype=A.dtype, device=A.device)
    _check(lib().gkb_gemm_tall(code, C.c_void_p(A.data_ptr()), A.stride(0), M, K, C.c_void_p(B.data_ptr()),
                               B.stride(0), N, C.c_void_p(C_out.data_ptr()), C_out.stride(0), _stream(stream)),
           False)
    return C_out


def gkb_matvec_fused(A, p, w=None, y=None, workspace=None, stream=None):
    """(w, y) = (A p, A^T A p) in one sweep of the float32 or bfloat16 device matrix A."""
    torch = _torch()
    mat = make_matrix(A)
    L = lib()
    need = L.gkb_matvec_fused_workspace_size(C.byref(mat))
    if w is None:
        w = torch.empty(A.shape[0], dtype=torch.float64, device=A.device)
    if y is None:
        y = torch.empty(A.shape[1], dtype=torch.float64, device=A.device)
    if workspace is None:
        workspace = _workspace(need, A.device)
    _check(L.gkb_matvec_fused(C.byref(mat), C.c_void_p(p.data_ptr()), C.c_void_p(w.data_ptr()),
                              C.c_void_p(y.data_ptr()), C.c_void_p(workspace.data_ptr()), workspace.numel(),
                              _stream(stream)), False)
    return w, y


def gkb_cast_bf16(src, dst=None, stream=None):
    """Round a float32 device matrix to bfloat16 (nearest even)."""
    torch = _torch()
    m, n = src.shape
    if dst is None:
        dst = torch.empty((m, n), dtype=torch.bfloat16, device=src.device)
    _check(lib().gkb_cast_bf16(C.c_void_p(src.data_ptr()), src.stride(0), m, n, C.c_void_p(dst.data_ptr()),
                               dst.stride(0), _stream(stream)), False)
    return dst


def gkb_start_vector(m, seed, device="cuda", stream=None):
    """q ~ N(2, 1)^m from the device Philox generator (float64)."""
    torch = _torch()
    q = torch.empty(m, dtype=torch.float64, device=device)
    _check(lib().gkb_start_vector(C.c_void_p(q.data_ptr()), m, seed, _stream(stream)), False)
    return q


def gkb_host_dense_svd(H: np.ndarray):
    """Host float64 SVD used per cycle (no device work)."""
    H = np.ascontiguousarray(H, dtype=np.float64)
    nq, np_ = H.shape
    kk = min(nq, np_)
    s = np.zeros(kk)
    X = np.zeros((nq, kk))
    Y = np.zeros((np_, kk))
    dp = C.POINTER(C.c_double)
    _check(lib().gkb_host_dense_svd(nq, np_, H.ctypes.data_as(dp), s.ctypes.data_as(dp), X.ctypes.data_as(dp),
                                    Y.ctypes.data_as(dp)), False)
    return X, s, Y


def gkb_host_bidiag_lastrow(alpha, beta):
    """Singular values and the last row of the left singular vectors of the
    (n + 1) x n lower bidiagonal with diagonal alpha and subdiagonal beta."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    assert a.shape == b.shape
    s = np.zeros(a.size)
    last = np.zeros(a.size)
    dp = C.POINTER(C.c_double)
    _check(lib().gkb_host_bidiag_lastrow(a.size, a.ctypes.data_as(dp), b.ctypes.data_as(dp), s.ctypes.data_as(dp),
                                         last.ctypes.data_as(dp)), False)
    return s, last


def gkb_host_bidiag_count_above(alpha, beta, nq, tau) -> int:
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta if len(beta) else [0.0], dtype=np.float64)
    dp = C.POINTER(C.c_double)
    return int(lib().gkb_host_bidiag_count_above(nq, a.size, a.ctypes.data_as(dp), b.ctypes.data_as(dp), tau))


def gkb_matvec_workspace_size(A) -> int:
    mat = make_matrix(A)
    return int(lib().gkb_matvec_workspace_size(C.byref(mat)))


def gkb_gemm_rowmajor(A, Bt, C_out=None, stream=None):
    """C = A B with A a row-major float32 (M, K) device tensor and B given as
    Bt (N, K) (= K x N column-major).  Returns Ct (N, M) (= M x N column-major)."""
    torch = _torch()
    M, K = A.shape
    N, K2 = Bt.shape
    if K != K2 or A.dtype != torch.float32 or Bt.dtype != torch.float32:
        raise ValueError("need float32 operands with matching inner dimension")
    if C_out is None:
        C_out = torch.empty((N, M), dtype=torch.float32, device=A.device)
    _check(lib().gkb_gemm_rowmajor(C.c_void_p(A.data_ptr()), A.stride(0), M, K, C.c_void_p(Bt.data_ptr()),
                                   Bt.stride(0), N, C.c_void_p(C_out.data_ptr()), C_out.stride(0),
                                   _stream(stream)), False)
    return C_out


def gkb_gram(Wt, stream=None):
    """G = W^T W (float64, d x d) for W given as Wt (d, m) float32 (= m x d column-major)."""
    torch = _torch()
    d, m = Wt.shape
    G = torch.empty((d, d), dtype=torch.float64, device=Wt.device)
    ws = _workspace(lib().gkb_gram_workspace_size(m, d), Wt.device)
    _check(lib().gkb_gram(C.c_void_p(Wt.data_ptr()), Wt.stride(0), m, d, C.c_void_p(G.data_ptr()),
                          C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)), False)
    return G


class BatchPlan:
    """A captured batched solve (gkb_batched_plan_*): build once, run many times.

    As: list of float32 device matrices (2-D, unit column stride); r, k: ints
    per problem.  Outputs (sigma, U, V) are packed device tensors owned by the
    plan; `results()` unpacks them per problem.
    """

    def __init__(self, As, r, k, tol, max_restarts, check_every=0, seed=0, q1=None, workgroups=0,
                 no_graph=False, eps_break=0.0, threads=0, stream=None, tune=False, tune_cache=None, max_team=0,
                 form=0, cost_estimate=None):
        torch = _torch()
        L = lib()
        self.batch = len(As)
        self.As = As
        self.r = [int(x) for x in r]
        self.k = [int(x) for x in k]
        self.mats = (GkbMatrix * self.batch)(*[make_matrix(A) for A in As])
        self.r_arr = (C.c_int * self.batch)(*self.r)
        self.k_arr = (C.c_int * self.batch)(*self.k)
        dev = As[0].device
        need = L.gkb_batched_workspace_size(self.batch, self.mats, self.r_arr, self.k_arr)
        if need == 0:
            raise GkbError(-1, "invalid batch")
        self.ws = _workspace(need, dev)
        self.sigma = torch.zeros(sum(self.r), dtype=torch.float64, device=dev)
        self.U = torch.zeros(sum(A.shape[0] * rr for A, rr in zip(As, self.r)), dtype=torch.float32, device=dev)
        self.V = torch.zeros(sum(A.shape[1] * rr for A, rr in zip(As, self.r)), dtype=torch.float32, device=dev)
        o = GkbBatchOptions()
        L.gkb_batch_default_options(C.byref(o))
        o.check_every = check_every
        o.seed = seed
        o.workgroups = workgroups
        o.no_graph = 1 if no_graph else 0
        o.eps_break = eps_break
        o.threads = threads
        o.max_team = max_team
        o.form = form
        self.q1 = q1
        if q1 is not None:
            o.q1_packed = q1.data_ptr()
        self.opts = o
        self.tuning = None
        self.plan = None
        if tune and cost_estimate is None:
            # calibration: one run with the default schedule measures what
            # each problem costs on one workgroup; that weighs the schedule
            self._create(tol, max_restarts, stream)
            self.run(stream)
            cost_estimate = self.work(stream)
            self.close()
        self.cost_estimate = None
        if cost_estimate is not None:
            if len(cost_estimate) != self.batch:
                raise ValueError("cost_estimate needs one value per problem")
            self.cost_estimate = (C.c_double * self.batch)(*[float(x) for x in cost_estimate])
            o.cost_estimate = C.cast(self.cost_estimate, C.c_void_p)
        if tune:
            self.tuning = self._autotune(tol, max_restarts, stream, tune_cache)
            o.threads, o.workgroups = self.tuning["threads"], self.tuning["workgroups"]
            o.form, o.max_team = self.tuning["form"], self.tuning["max_team"]
            self.tuning["measured_costs"] = self.cost_estimate is not None
        self._create(tol, max_restarts, stream)

    def _create(self, tol, max_restarts, stream):
        L = lib()
        o = self.opts
        plan = C.c_void_p()
        st = L.gkb_batched_plan_create(self.batch, self.mats, self.r_arr, self.k_arr, float(tol), int(max_restarts),
                                       C.byref(o), C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                       C.c_void_p(self.sigma.data_ptr()), C.c_void_p(self.U.data_ptr()),
                                       C.c_void_p(self.V.data_ptr()), _stream(stream), C.byref(plan))
        if st != 0:
            raise GkbError(st, L.gkb_batched_last_error().decode())
        self.plan = plan

    def signature(self):
        """Cache key: device name and the sorted problem shapes."""
        torch = _torch()
        shapes = sorted((int(A.shape[0]), int(A.shape[1]), rr, kk) for A, rr, kk in zip(self.As, self.r, self.k))
        import hashlib
        h = hashlib.sha1(repr(shapes).encode()).hexdigest()[:16]
        return f"{torch.cuda.get_device_properties(self.As[0].device).gcnArchName}:{len(shapes)}:{h}"

    def _autotune(self, tol, max_restarts, stream, cache_path):
        import json
        key = self.signature()
        cache = {}
        if cache_path and os.path.exists(cache_path):
            try:
                cache = json.load(open(cache_path))
            except (OSError, ValueError):
                cache = {}
        if key in cache and "form" in cache[key]:
            return dict(cache[key], cached=True)
        L = lib()
        bt, bw, bf, bm, n = C.c_int(), C.c_int(), C.c_int(), C.c_int(), C.c_int()
        times = (C.c_double * 12)()
        st = L.gkb_batched_autotune(self.batch, self.mats, self.r_arr, self.k_arr, float(tol), int(max_restarts),
                                    C.byref(self.opts), C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                    C.c_void_p(self.sigma.data_ptr()), C.c_void_p(self.U.data_ptr()),
                                    C.c_void_p(self.V.data_ptr()), _stream(stream), C.byref(bt), C.byref(bw),
                                    C.byref(bf), C.byref(bm), times, C.byref(n))
        if st != 0:
            raise GkbError(st, L.gkb_batched_last_error().decode())
        res = {"threads": bt.value, "workgroups": bw.value, "form": bf.value, "max_team": bm.value,
               "times_ms": list(times[: n.value])}
        if cache_path:
            cache[key] = res
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1)
            os.replace(tmp, cache_path)
        return dict(res, cached=False)

    @property
    def grid(self):
        return lib().gkb_batched_plan_grid(self.plan)

    def run(self, stream=None):
        st = lib().gkb_batched_plan_run(self.plan, _stream(stream))
        if st != 0:
            raise GkbError(st, lib().gkb_batched_last_error().decode())

    def info(self, stream=None):
        arr = (C.c_int * (4 * self.batch))()
        st = lib().gkb_batched_plan_info(self.plan, arr, _stream(stream))
        if st != 0:
            raise GkbError(st, lib().gkb_batched_last_error().decode())
        return np.array(arr[:], dtype=np.int64).reshape(self.batch, 4)

    def results(self):
        """Per problem: (sigma (numpy), Ut (r x m tensor), Vt (r x n tensor))."""
        out = []
        os_ = ou = ov = 0
        for A, rr in zip(self.As, self.r):
            m, n = A.shape
            out.append((self.sigma[os_:os_ + rr].cpu().numpy(), self.U[ou:ou + m * rr].view(rr, m),
                        self.V[ov:ov + n * rr].view(rr, n)))
            os_ += rr
            ou += m * rr
            ov += n * rr
        return out

    def work(self, stream=None):
        """Per problem: ms its first workgroup spent on it in the last run, times
        its team size (gkb_batched_plan_work)."""
        out = np.zeros(self.batch, dtype=np.float64)
        st = lib().gkb_batched_plan_work(self.plan, out.ctypes.data_as(C.c_void_p), _stream(stream))
        if st != 0:
            raise GkbError(st, lib().gkb_batched_last_error().decode())
        return out

    def close(self):
        if self.plan:
            lib().gkb_batched_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ learned start
def _lcheck(status):
    if status != 0:
        raise GkbError(status, lib().gkb_learned_last_error().decode())


def gkb_mlp_param_count(n_in, hidden) -> int:
    return int(lib().gkb_mlp_param_count(n_in, hidden))


def gkb_mlp_features(St, Ut_prev, stream=None):
    """Features X (m x stride) from the sketch St (ws x m, i.e. m x ws column-major)
    and the previous left vectors Ut_prev (r x m)."""
    torch = _torch()
    ws, m = St.shape
    r = Ut_prev.shape[0] if Ut_prev is not None else 0
    X = torch.empty((m, lib().gkb_mlp_feature_stride()), dtype=torch.float32, device=St.device)
    wk = _workspace(64 * 8 + 4 * (r + 1) + 256, St.device)
    _lcheck(lib().gkb_mlp_features(C.c_void_p(St.data_ptr()), St.stride(0), m, ws,
                                   C.c_void_p(Ut_prev.data_ptr()) if r else None, r, C.c_void_p(X.data_ptr()),
                                   C.c_void_p(wk.data_ptr()), wk.numel(), _stream(stream)))
    return X


def gkb_mlp_forward(params, n_in, hidden, X, stream=None):
    torch = _torch()
    z = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _lcheck(lib().gkb_mlp_forward(C.c_void_p(params.data_ptr()), n_in, hidden, C.c_void_p(X.data_ptr()),
                                  X.shape[0], C.c_void_p(z.data_ptr()), _stream(stream)))
    return z


def gkb_mlp_loss_grad(params, n_in, hidden, X, Ut, grad=None, loss=None, workspace=None, stream=None, kind=0):
    """(grad, loss) device tensors for the target left vectors Ut (r x m); kind 0:
    energy outside the target subspace, kind 1: mean log tan^2 of the angles."""
    torch = _torch()
    m = X.shape[0]
    r = Ut.shape[0]
    if grad is None:
        grad = torch.empty(gkb_mlp_param_count(n_in, hidden), dtype=torch.float32, device=X.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=X.device)
    if workspace is None:
        workspace = _workspace(lib().gkb_mlp_workspace_size(m, n_in, hidden, r), X.device)
    _lcheck(lib().gkb_mlp_loss_grad_kind(C.c_void_p(params.data_ptr()), n_in, hidden, C.c_void_p(X.data_ptr()), m,
                                         C.c_void_p(Ut.data_ptr()), r, int(kind), C.c_void_p(grad.data_ptr()),
                                         C.c_void_p(loss.data_ptr()), C.c_void_p(workspace.data_ptr()),
                                         workspace.numel(), _stream(stream)))
    return grad, loss


def gkb_adam_step(params, grad, m1, m2, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _lcheck(lib().gkb_adam_step(C.c_void_p(params.data_ptr()), C.c_void_p(grad.data_ptr()),
                                C.c_void_p(m1.data_ptr()), C.c_void_p(m2.data_ptr()), params.numel(), lr, beta1,
                                beta2, eps, step, _stream(stream)))


def gkb_mlp_start_vector(params, n_in, hidden, X, stream=None):
    torch = _torch()
    m = X.shape[0]
    q = torch.empty(m, dtype=torch.float64, device=X.device)
    wk = _workspace(4 * m + 256, X.device)
    _lcheck(lib().gkb_mlp_start_vector(C.c_void_p(params.data_ptr()), n_in, hidden, C.c_void_p(X.data_ptr()), m,
                                       C.c_void_p(q.data_ptr()), C.c_void_p(wk.data_ptr()), wk.numel(),
                                       _stream(stream)))
    return q


class SparsePlan:
    """A sparse float32 matrix on the device (CSR of A and of A^T) with its row
    bins (gkb_sparse_plan_*).  `arrays` holds row_ptr (int64), col_idx (int32),
    val (float32), col_ptr, row_idx, val_t as numpy arrays or device tensors.
    panels=True gives the plan the workspace of the column-panel layout
    (gkb_sparse_panel_workspace_size); `self.panels` says which products use
    it (bit 0: A p, bit 1: A^T q)."""

    def __init__(self, m, n, arrays, device="cuda:0", stream=None, panels=True):
        torch = _torch()
        self.m, self.n = int(m), int(n)
        self.t = {}
        for key, dt in (("row_ptr", torch.int64), ("col_idx", torch.int32), ("val", torch.float32),
                        ("col_ptr", torch.int64), ("row_idx", torch.int32), ("val_t", torch.float32)):
            a = arrays[key]
            if not torch.is_tensor(a):
                a = torch.from_numpy(np.ascontiguousarray(a))
            self.t[key] = a.to(device=device, dtype=dt).contiguous()
        self.nnz = int(self.t["val"].numel())
        self.csr = GkbCsr(self.m, self.n, self.nnz, *[C.c_void_p(self.t[k].data_ptr()) for k in
                                                       ("row_ptr", "col_idx", "val", "col_ptr", "row_idx", "val_t")])
        self.device = torch.device(device)
        L = lib()
        need = (L.gkb_sparse_panel_workspace_size if panels else L.gkb_sparse_plan_workspace_size)(C.byref(self.csr))
        if need == 0:
            raise GkbError(-1, "invalid sparse matrix")
        self.ws = _workspace(need, self.device)
        plan = C.c_void_p()
        st = L.gkb_sparse_plan_create(C.byref(self.csr), C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                      _stream(stream), C.byref(plan))
        if st != 0:
            raise GkbError(st, L.gkb_sparse_last_error().decode())
        self.plan = plan
        self.panels = int(L.gkb_sparse_plan_panels(plan))

    def matvec(self, x, trans=0, y=None, stream=None):
        """y = A x (trans 0) or A^T x (trans 1); x float32, y float64 device tensors."""
        torch = _torch()
        if y is None:
            y = torch.empty(self.n if trans else self.m, dtype=torch.float64, device=self.device)
        st = lib().gkb_sparse_matvec(self.plan, int(trans), C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                     _stream(stream))
        if st != 0:
            raise GkbError(st, lib().gkb_sparse_last_error().decode())
        return y

    def workspace_size(self, r, k):
        return int(lib().gkb_sparse_workspace_size(self.plan, r, k))

    def partial_svd(self, r, k, tol, max_restarts, workspace=None, stream=None, **opts):
        """As gkb_partial_svd: (sigma, Ut, Vt, status, stats)."""
        torch = _torch()
        L = lib()
        o = make_options(**opts)
        need = self.workspace_size(r, k)
        if workspace is None:
            workspace = _workspace(need, self.device)
        Ut = torch.empty((r, self.m), dtype=torch.float32, device=self.device)
        Vt = torch.empty((r, self.n), dtype=torch.float32, device=self.device)
        sig = (C.c_double * r)()
        st = GkbStats()
        status = L.gkb_partial_svd_sparse(self.plan, int(r), int(k), float(tol), int(max_restarts), C.byref(o),
                                          C.c_void_p(workspace.data_ptr()), workspace.numel(), sig,
                                          C.c_void_p(Ut.data_ptr()), C.c_void_p(Vt.data_ptr()), C.byref(st),
                                          _stream(stream))
        _check(status)
        return np.array(sig[:], dtype=np.float64), Ut, Vt, status, st.as_dict()

    def close(self):
        if getattr(self, "plan", None):
            lib().gkb_sparse_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RsgdPlan:
    """Riemannian mini-batch gradient descent on rank-r matrices (gkb_rsgd_*).

    State (device): U (r x d1 float32, rows = the columns of the d1 x r factor),
    s (r float64), Vt (r x d2 float32): W = U^T diag(s) Vt.  Batch buffers X
    (b x d1), V (b x d2), y (b) are owned by the plan; `step(X, V, y)` copies a
    batch in and replays the captured step."""

    def __init__(self, d1, d2, r, k, b, eta, lam, U0, s0, V0, device="cuda:0", stream=None):
        torch = _torch()
        self.d1, self.d2, self.r, self.k, self.b = int(d1), int(d2), int(r), int(k), int(b)
        dev = torch.device(device)
        self.device = dev
        self.X = torch.zeros((b, d1), dtype=torch.float32, device=dev)
        self.V = torch.zeros((b, d2), dtype=torch.float32, device=dev)
        self.y = torch.zeros(b, dtype=torch.float32, device=dev)
        self.U = torch.as_tensor(np.ascontiguousarray(np.asarray(U0).T), dtype=torch.float32).to(dev).contiguous()
        self.s = torch.as_tensor(np.asarray(s0, dtype=np.float64)).to(dev).contiguous()
        self.Vt = torch.as_tensor(np.ascontiguousarray(np.asarray(V0).T), dtype=torch.float32).to(dev).contiguous()
        L = lib()
        need = L.gkb_rsgd_workspace_size(d1, d2, r, k, b)
        if need == 0:
            raise GkbError(-1, "invalid RSGD sizes")
        self.ws = _workspace(need, dev)
        plan = C.c_void_p()
        st = L.gkb_rsgd_plan_create(d1, d2, r, k, b, float(eta), float(lam), C.c_void_p(self.X.data_ptr()),
                                    C.c_void_p(self.V.data_ptr()), C.c_void_p(self.y.data_ptr()),
                                    C.c_void_p(self.U.data_ptr()), C.c_void_p(self.s.data_ptr()),
                                    C.c_void_p(self.Vt.data_ptr()), C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                    _stream(stream), C.byref(plan))
        if st != 0:
            raise GkbError(st, L.gkb_rsgd_last_error().decode())
        self.plan = plan

    def load(self, X, V, y):
        self.X.copy_(X, non_blocking=True)
        self.V.copy_(V, non_blocking=True)
        self.y.copy_(y, non_blocking=True)

    def step(self, X=None, V=None, y=None, stream=None):
        if X is not None:
            self.load(X, V, y)
        st = lib().gkb_rsgd_plan_step(self.plan, _stream(stream))
        if st != 0:
            raise GkbError(st, lib().gkb_rsgd_last_error().decode())

    def info(self, stream=None):
        out = (C.c_int * 4)()
        st = lib().gkb_rsgd_plan_info(self.plan, out, _stream(stream))
        if st != 0:
            raise GkbError(st, lib().gkb_rsgd_last_error().decode())
        return list(out)

    def weights(self, stream=None):
        torch = _torch()
        W = torch.empty((self.d1, self.d2), dtype=torch.float32, device=self.device)
        st = lib().gkb_rsgd_weights(self.d1, self.d2, self.r, C.c_void_p(self.U.data_ptr()),
                                    C.c_void_p(self.s.data_ptr()), C.c_void_p(self.Vt.data_ptr()),
                                    C.c_void_p(W.data_ptr()), _stream(stream))
        if st != 0:
            raise GkbError(st, lib().gkb_rsgd_last_error().decode())
        return W

    def close(self):
        if getattr(self, "plan", None):
            lib().gkb_rsgd_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
