"""ctypes binding of libhdg.so: argument marshalling only.

Every numerical step runs in the HIP library; this module passes pointers, sizes
and streams. PyTorch supplies device memory and streams.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhdg.so")

HDG_OK = 0
STATUS_NAMES = {0: "HDG_OK", 1: "HDG_ERR_INVALID_ARG", 2: "HDG_ERR_OOM", 3: "HDG_ERR_SINGULAR_LOCAL",
                4: "HDG_ERR_NONFINITE", 5: "HDG_ERR_NOT_CONVERGED", 6: "HDG_ERR_HIP"}
HDG_EULER, HDG_NS = 0, 1
HDG_FP64, HDG_MIXED, HDG_MIXED_CONDENSE = 0, 1, 2

EXPORTS = ["hdg_plan_create", "hdg_plan_sizes", "hdg_plan_faces", "hdg_plan_pattern", "hdg_assemble_condense",
           "hdg_assemble_condense_batch", "hdg_skeleton_solve", "hdg_back_substitute", "hdg_debug_element_blocks", "hdg_debug_local_solution", "hdg_debug_condense_variant",
           "hdg_set_kernel_timing", "hdg_kernel_timing", "hdg_set_cfl", "hdg_residual_norm", "hdg_apply_update",
           "hdg_cfl_schedule", "hdg_pseudo_transient_solve", "hdg_skeleton_transpose", "hdg_adjoint_rhs",
           "hdg_adjoint_local", "hdg_mark_elements", "hdg_mark_elements_noalloc", "hdg_set_poly_degree", "hdg_debug_hessenberg_eigenvalues",
           "hdg_last_error", "hdg_plan_destroy"]


class HdgParams(C.Structure):
    _fields_ = [("physics", C.c_int32), ("precision", C.c_int32), ("gamma", C.c_double), ("mach", C.c_double),
                ("aoa_rad", C.c_double), ("reynolds", C.c_double), ("prandtl", C.c_double),
                ("stab_alpha", C.c_double), ("cfl", C.c_double), ("sc_eps0", C.c_double), ("sc_beta", C.c_double)]


class HdgSizes(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("n_elements", "n_faces", "n_boundary_faces", "n_skel_dof", "np_max",
                                         "n_fields", "bsr_blocks", "bsr_values", "local_store_bytes",
                                         "workspace_bytes", "n_buckets")]


class HdgNewtonOpts(C.Structure):
    _fields_ = [("c0", C.c_double), ("c1", C.c_double), ("n0", C.c_int32), ("max_steps", C.c_int32),
                ("rel_tol", C.c_double), ("abs_tol", C.c_double), ("gmres_rtol", C.c_double),
                ("restart", C.c_int32), ("max_iter", C.c_int32)]


class HdgNewtonReport(C.Structure):
    _fields_ = [("steps", C.c_int32), ("converged", C.c_int32), ("gmres_iters", C.c_int64),
                ("gmres_not_converged", C.c_int32), ("res0", C.c_double), ("res", C.c_double)]


class HdgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libhdg.so; raise if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libhdg.so not built at {path}; run `python -m paper_1308_3995_amd.build`")
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    lib.hdg_plan_create.argtypes = [P(vp), vp, i32, vp, i32, vp, P(HdgParams), C.c_int]
    lib.hdg_plan_sizes.argtypes = [vp, P(HdgSizes)]
    lib.hdg_plan_faces.argtypes = [vp, vp, vp, vp]
    lib.hdg_plan_pattern.argtypes = [vp, vp, vp, vp]
    lib.hdg_assemble_condense.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, P(dbl), vp]
    lib.hdg_assemble_condense_batch.argtypes = [C.c_int32, vp, vp, vp, vp, vp, vp, vp, vp, P(C.c_int32), vp]
    lib.hdg_skeleton_solve.argtypes = [vp, vp, vp, vp, dbl, i32, i32, vp, vp, P(i32), P(dbl)]
    lib.hdg_back_substitute.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.hdg_debug_element_blocks.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, P(i32), P(i32)]
    lib.hdg_debug_local_solution.argtypes = [vp, vp, i64, vp, vp, P(i32), P(i32)]
    lib.hdg_debug_condense_variant.argtypes = [vp, i32]
    lib.hdg_set_kernel_timing.argtypes = [vp, i32]
    lib.hdg_kernel_timing.argtypes = [vp, i32, P(i64), P(dbl), P(dbl), i32]
    lib.hdg_set_poly_degree.argtypes = [vp, i32, i32]
    lib.hdg_debug_hessenberg_eigenvalues.argtypes = [i32, vp, vp, vp]
    lib.hdg_set_cfl.argtypes = [vp, dbl]
    lib.hdg_residual_norm.argtypes = [vp, vp, vp, P(dbl), vp]
    lib.hdg_apply_update.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hdg_cfl_schedule.argtypes = [i32, dbl, dbl, dbl, dbl, dbl, i32]
    lib.hdg_cfl_schedule.restype = dbl
    lib.hdg_pseudo_transient_solve.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, P(HdgNewtonOpts),
                                               P(HdgNewtonReport), vp, vp, vp]
    lib.hdg_skeleton_transpose.argtypes = [vp, vp, vp, vp]
    lib.hdg_adjoint_rhs.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.hdg_adjoint_local.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hdg_mark_elements.argtypes = [vp, vp, vp, dbl, dbl, vp, vp, P(i32), vp, vp]
    lib.hdg_mark_elements_noalloc.argtypes = [vp, vp, vp, dbl, dbl, vp, vp, P(i32), vp]
    lib.hdg_last_error.argtypes = []
    lib.hdg_last_error.restype = C.c_char_p
    lib.hdg_plan_destroy.argtypes = [vp]
    lib.hdg_plan_destroy.restype = None
    for name in EXPORTS:
        if name not in ("hdg_last_error", "hdg_plan_destroy", "hdg_cfl_schedule"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def check(status: int):
    if status != HDG_OK:
        raise HdgError(status, _lib.hdg_last_error().decode())
