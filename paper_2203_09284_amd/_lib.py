"""ctypes declarations of the C ABI in include/fusedpr.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfusedpr.so")

PR_OK, PR_NOT_CONVERGED, PR_EINVAL, PR_ENOMEM, PR_EDEVICE = 0, 1, -1, -2, -3
PR_JACOBI, PR_FUSED, PR_EDGE_LIST, PR_INPLACE, PR_FUSED_EDGE_LIST = 0, 1, 2, 3, 4
PR_FP64, PR_FP32 = 0, 1
PR_DANGLING_UNIFORM, PR_DANGLING_LEAK = 0, 1
PR_NORM_L1, PR_NORM_LINF = 0, 1

c_i32p = ctypes.POINTER(ctypes.c_int32)
c_i64p = ctypes.POINTER(ctypes.c_int64)
c_f64p = ctypes.POINTER(ctypes.c_double)
vp = ctypes.c_void_p


class PrCsr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64),
                ("in_ptr", c_i64p), ("in_src", c_i32p), ("in_w", c_f64p),
                ("out_ptr", c_i64p), ("out_dst", c_i32p), ("out_w", c_f64p),
                ("out_to_in", c_i64p), ("out_deg", c_i32p), ("in_deg", c_i32p),
                ("m_input", ctypes.c_int64), ("edge_map", c_i64p)]


class PrPlanOpts(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int), ("tile_max_row", ctypes.c_int), ("tile_rows", ctypes.c_int),
                ("steps", ctypes.c_int), ("hot_slots", ctypes.c_int),
                ("gather_layout", ctypes.c_int), ("with_adjoint", ctypes.c_int), ("gs_blocks", ctypes.c_int),
                ("with_cl", ctypes.c_int), ("with_inplace", ctypes.c_int)]


class PrGraphStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64),
                ("n_light", ctypes.c_int64), ("n_medium", ctypes.c_int64), ("n_heavy", ctypes.c_int64),
                ("e_light", ctypes.c_int64), ("e_medium", ctypes.c_int64), ("e_heavy", ctypes.c_int64),
                ("n_items", ctypes.c_int64), ("n_dangling", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("grid", ctypes.c_int), ("gs_blocks", ctypes.c_int),
                ("chunk", ctypes.c_int), ("graph_captures", ctypes.c_int64), ("signature", ctypes.c_uint64),
                ("local_share", ctypes.c_double), ("gather_layout", ctypes.c_int)]


class PrBatchShape(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int), ("items_per_grab", ctypes.c_int), ("wg_per_cu", ctypes.c_int)]


class PrOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("precision", ctypes.c_int), ("dangling", ctypes.c_int),
                ("norm", ctypes.c_int), ("warm_start", ctypes.c_int), ("fused_scaled", ctypes.c_int),
                ("sweeps_per_poll", ctypes.c_int), ("use_hip_graph", ctypes.c_int),
                ("refine_tol", ctypes.c_double), ("fp32_tol", ctypes.c_double),
                ("trace", c_f64p)]


# name -> (restype, argtypes); the symbols every include/fusedpr.h declaration exports
SIGNATURES = {
    "pr_last_error": (ctypes.c_char_p, []),
    "pr_build_csr": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, vp, vp, vp, ctypes.POINTER(PrCsr)]),
    "pr_csr_free": (None, [ctypes.POINTER(PrCsr)]),
    "pr_plan_opts_default": (None, [ctypes.POINTER(PrPlanOpts)]),
    "pr_graph_create": (ctypes.c_int, [ctypes.POINTER(PrCsr), ctypes.POINTER(PrPlanOpts), ctypes.POINTER(vp)]),
    "pr_graph_destroy": (None, [vp]),
    "pr_graph_device_bytes": (ctypes.c_int, [ctypes.POINTER(PrCsr), ctypes.POINTER(PrPlanOpts),
                                             ctypes.POINTER(ctypes.c_size_t)]),
    "pr_graph_bind": (ctypes.c_int, [ctypes.POINTER(PrCsr), ctypes.POINTER(PrPlanOpts), vp, ctypes.c_size_t,
                                     ctypes.POINTER(vp)]),
    "pr_graph_free": (None, [vp]),
    "pr_workspace_bytes": (ctypes.c_int, [vp, ctypes.c_double, ctypes.POINTER(PrOpts),
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "pr_solve_ws": (ctypes.c_int, [vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.POINTER(PrOpts), vp,
                                   vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int), c_f64p, vp]),
    "pr_graph_stats_get": (ctypes.c_int, [vp, ctypes.POINTER(PrGraphStats)]),
    "pr_opts_default": (None, [ctypes.POINTER(PrOpts)]),
    "pr_solve": (ctypes.c_int, [vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.POINTER(PrOpts),
                                vp, vp, ctypes.POINTER(ctypes.c_int), c_f64p, vp]),
    "pr_solve_noalloc": (ctypes.c_int, [vp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                        ctypes.POINTER(PrOpts), vp, vp, ctypes.POINTER(ctypes.c_int), c_f64p, vp]),
    "pr_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "pr_iterate": (ctypes.c_int, [vp, ctypes.c_double, ctypes.POINTER(PrOpts), vp, vp, ctypes.c_int, c_f64p,
                                  c_f64p, vp]),
    "pr_certificate": (ctypes.c_int, [vp, ctypes.c_double, vp, vp, c_f64p, vp]),
    "pr_profile_sweeps": (ctypes.c_int, [vp, ctypes.c_double, ctypes.POINTER(PrOpts), vp, ctypes.c_int, c_f64p,
                                         c_f64p, vp]),
    "pr_probe_gathers": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, c_f64p, c_f64p, vp]),
    "pr_batch_shape_default": (None, [ctypes.POINTER(PrBatchShape)]),
    "pr_solve_batched": (ctypes.c_int, [vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, vp,
                                        ctypes.POINTER(PrBatchShape), vp, ctypes.POINTER(ctypes.c_int), c_f64p, vp]),
    "pr_autotune_batched": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_char_p, ctypes.POINTER(PrBatchShape), vp]),
    "pr_adjoint": (ctypes.c_int, [vp, ctypes.c_double, vp, vp, ctypes.c_double, ctypes.c_int, vp, vp, vp,
                                  ctypes.POINTER(ctypes.c_int), c_f64p, vp]),
}

_LIBS: dict = {}
# library builds: the product, and a variant whose FP32 sums carry no
# compensation term (tests compare the two)
VARIANTS = {"": LIB_PATH, "naive": os.path.join(HERE, "libfusedpr_naive.so")}


class FusedPRError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("fusedpr error %d: %s" % (code, msg))
        self.code = code


def lib(variant: str = ""):
    """Load the in-tree HIP library (or one of its test variants); fail loudly
    when it is missing (no fallback)."""
    if variant in _LIBS:
        return _LIBS[variant]
    path = VARIANTS[variant]
    if not os.path.exists(path):
        raise ImportError("%s is not built; run __graft_entry__.build()" % path)
    L = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _LIBS[variant] = L
    return L


def check(code: int, allow_not_converged: bool = True, library=None) -> int:
    if code == PR_OK or (code == PR_NOT_CONVERGED and allow_not_converged):
        return code
    raise FusedPRError(code, (library or lib()).pr_last_error().decode(errors="replace"))
