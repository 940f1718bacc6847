"""ctypes binding of libpaqif_ehl.so (argument marshalling only).

Every numerical step runs in the HIP library; this module only converts
torch tensors on the GPU into the raw pointers and sizes of the C ABI
declared in ``include/paqif_ehl.h`` and raises on call-level errors.  There
is no CPU fallback: if the library is missing the import of a function
fails loudly.
"""
import ctypes
import os

from . import build as _build

_LIB = None

PAQIF_OK, PAQIF_EINVAL, PAQIF_EWORKSPACE, PAQIF_EHIP = 0, -1, -2, -3
SYS_OK, SYS_ZERO_PIVOT, SYS_NONFINITE, SYS_LCP_NOT_CONVERGED = 0, 1, 2, 3
SYS_REFINE_STALLED, SYS_NEGATIVE_FILM, SYS_NEWTON_NOT_CONVERGED = 4, 5, 6
SYS_ADJOINT_NOT_CONVERGED = 7
PREC_FP64, PREC_FP32_IR, PREC_SPLIT_BF16, PREC_FP32 = 0, 1, 2, 3
LCP_LINEAR, LCP_CLIP, LCP_EXACT, LCP_EXACT_FROM_U = 0, 1, 2, 3


class PaqifBatch(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("q", ctypes.c_int32),
                ("offsets", ctypes.c_void_p), ("max_n", ctypes.c_int64),
                ("total_rows", ctypes.c_int64), ("order", ctypes.c_void_p)]


class PaqifLcpCall(ctypes.Structure):
    _fields_ = [("batch", ctypes.POINTER(PaqifBatch)), ("band", ctypes.c_void_p),
                ("b", ctypes.c_void_p), ("bounded", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("active_out", ctypes.c_void_p),
                ("sys_status", ctypes.c_void_p), ("sys_iters", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p)]


MAX_LCP_CALLS = 8


class EhlGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("x0", ctypes.c_double),
                ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double)]


class EhlParams(ctypes.Structure):
    _fields_ = [("M", ctypes.c_double), ("L", ctypes.c_double)]


class EhlOpts(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("c_h0", ctypes.c_double),
                ("switch_ratio", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_newton", ctypes.c_int32), ("kernel_terms", ctypes.c_int32),
                ("lcp_max_iter", ctypes.c_int32), ("deform_prec", ctypes.c_int32),
                ("lcp_prec", ctypes.c_int32), ("steps_per_graph", ctypes.c_int32),
                ("start_rule", ctypes.c_int32), ("limiter_jacobian", ctypes.c_int32),
                ("stall_steps", ctypes.c_int32), ("convection", ctypes.c_int32),
                ("kappa", ctypes.c_double), ("lcp_fail_steps", ctypes.c_int32),
                ("splitting", ctypes.c_int32)]


class LibraryMissing(RuntimeError):
    pass


def library_path():
    return _build.LIB


def lib():
    """Load the HIP library; raise LibraryMissing if it was not built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise LibraryMissing(
            f"{path} not found: build it with paper_2008_03276_amd.build.build() "
            "(there is no CPU fallback)")
    L = ctypes.CDLL(path)
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    bp = ctypes.POINTER(PaqifBatch)
    sig = {
        "paqif_create": ([ctypes.POINTER(vp)], ctypes.c_int),
        "paqif_destroy": ([vp], ctypes.c_int),
        "paqif_status_str": ([ctypes.c_int], ctypes.c_char_p),
        "paqif_workspace_bytes": ([vp, bp, ctypes.c_int, ctypes.c_int], ctypes.c_size_t),
        "paqif_factor": ([vp, bp, vp, vp, ctypes.c_int, vp, vp, vp], ctypes.c_int),
        "paqif_solve_factored": ([vp, bp, vp, ctypes.c_int, vp, vp, vp, vp], ctypes.c_int),
        "paqif_solve_lcp": ([vp, bp, vp, vp, vp, ctypes.c_int, ctypes.c_int, d, ctypes.c_int,
                             vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "paqif_solve_lcp_noalloc": ([vp, bp, vp, vp, vp, ctypes.c_int, ctypes.c_int, d,
                                     ctypes.c_int, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "paqif_layout_count": ([ctypes.c_int], ctypes.c_int),
        "paqif_set_layout": ([vp, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "paqif_get_layout": ([vp, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "paqif_set_start_sweeps": ([vp, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "paqif_get_start_sweeps": ([vp, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "paqif_start_sweeps": ([vp, bp, vp, vp, vp, ctypes.c_int, vp, vp, vp], ctypes.c_int),
        "paqif_solve_lcp_many": ([vp, ctypes.c_int, ctypes.POINTER(PaqifLcpCall), ctypes.c_int,
                                  ctypes.c_int, d, ctypes.c_int, vp], ctypes.c_int),
        "paqif_autotune": ([vp, bp, vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp,
                            vp, vp, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
        "ehl_deformation_workspace_bytes": ([ctypes.POINTER(EhlGrid), ctypes.c_int],
                                            ctypes.c_size_t),
        "ehl_deformation": ([vp, ctypes.POINTER(EhlGrid), vp, ctypes.c_int, ctypes.c_int, vp, vp,
                             vp], ctypes.c_int),
        "ehl_jacobian_assemble": ([vp, ctypes.POINTER(EhlGrid), vp, ctypes.c_int,
                                   ctypes.POINTER(EhlOpts), vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                   vp], ctypes.c_int),
        "ehl_newton_workspace_bytes": ([vp, ctypes.POINTER(EhlGrid), ctypes.c_int,
                                        ctypes.POINTER(EhlOpts)], ctypes.c_size_t),
        "ehl_newton_tvd": ([vp, ctypes.POINTER(EhlGrid), vp, ctypes.c_int, ctypes.POINTER(EhlOpts),
                            vp, vp, vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "ehl_point_assemble_workspace_bytes": ([ctypes.POINTER(EhlGrid), ctypes.c_int],
                                               ctypes.c_size_t),
        "ehl_point_sweep_assemble": ([vp, ctypes.POINTER(EhlGrid), vp, ctypes.c_int,
                                      ctypes.POINTER(EhlOpts), ctypes.c_int, ctypes.c_int, vp, vp,
                                      vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "ehl_adjoint_workspace_bytes": ([vp, ctypes.POINTER(EhlGrid), ctypes.c_int],
                                        ctypes.c_size_t),
        "ehl_adjoint_solve": ([vp, ctypes.POINTER(EhlGrid), vp, ctypes.c_int,
                               ctypes.POINTER(EhlOpts), vp, vp, vp, vp, vp, vp, d, ctypes.c_int,
                               vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "paqif_partitioned_workspace_bytes": ([i64, ctypes.c_int, i32], ctypes.c_size_t),
        "paqif_solve_partitioned": ([vp, i64, ctypes.c_int, i32, vp, vp, vp, ctypes.c_int,
                                     ctypes.c_int, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "cd_workspace_bytes": ([ctypes.c_int], ctypes.c_size_t),
        "cd_ls3_workspace_bytes": ([ctypes.c_int], ctypes.c_size_t),
        "cd_distributive_relax": ([vp, ctypes.c_int, d, d, d, d, d, d, ctypes.c_int, vp, vp,
                                   ctypes.POINTER(i32), ctypes.POINTER(d), vp, vp], ctypes.c_int),
        "cd_example": ([ctypes.c_int, d, d, d, vp, vp, vp], ctypes.c_int),
        "cd_line_relax": ([vp, ctypes.c_int, d, d, d, d, d, d, ctypes.c_int, vp, vp,
                           ctypes.POINTER(i32), ctypes.POINTER(d), vp, vp], ctypes.c_int),
        "cd_split_relax": ([vp, ctypes.c_int, ctypes.c_int, d, d, d, d, d, d, ctypes.c_int, vp,
                            vp, ctypes.POINTER(i32), ctypes.POINTER(d), vp, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _LIB = L
    return L


def check(code, what):
    if code != PAQIF_OK:
        msg = lib().paqif_status_str(code).decode()
        raise RuntimeError(f"{what} failed: {msg} ({code})")
