"""ctypes declarations of the C ABI in include/tpf.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtpf.so")

TPF_OK = 0
TPF_NOT_CONVERGED = 1
TPF_STEP_REJECTED = 2
TPF_EINVAL = -1
TPF_ENOMEM = -2
TPF_EDEVICE = -3
TPF_EBREAKDOWN = -4
TPF_ESTATE = -5
TPF_FP64 = 0
TPF_MIXED = 1
TPF_MIXED16 = 2
TPF_MAX_PATCHES = 8
TPF_KR_BURDINE = 0
TPF_KR_POLY = 1

STATUS_NAMES = {0: "TPF_OK", 1: "TPF_NOT_CONVERGED", 2: "TPF_STEP_REJECTED", -1: "TPF_EINVAL",
                -2: "TPF_ENOMEM", -3: "TPF_EDEVICE", -4: "TPF_EBREAKDOWN", -5: "TPF_ESTATE"}


class Patch(C.Structure):
    _fields_ = [("axis", C.c_int32), ("side", C.c_int32), ("phase", C.c_int32), ("reserved", C.c_int32),
                ("lo", C.c_double * 2), ("hi", C.c_double * 2), ("rate", C.c_double)]


class GridDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("extent", C.c_double * 3),
                ("gravity", C.c_double * 3), ("rho", C.c_double * 2), ("mu", C.c_double * 2),
                ("s_res", C.c_double * 2), ("perm", C.POINTER(C.c_double)), ("poro", C.POINTER(C.c_double)),
                ("entry_p", C.POINTER(C.c_double)), ("bc_lambda", C.POINTER(C.c_double)),
                ("dir_mask", C.POINTER(C.c_uint8)), ("dir_value", C.POINTER(C.c_double)),
                ("patches", C.POINTER(Patch)), ("n_patches", C.c_int32), ("levels", C.c_int32),
                ("precision", C.c_int32), ("nu_pre", C.c_int32), ("nu_post", C.c_int32),
                ("limex_stages", C.c_int32), ("omega", C.c_double), ("kr_model", C.c_int32),
                ("smoother", C.c_int32), ("kr_coef", C.c_double * 2), ("vertex_source", C.POINTER(C.c_double))]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("rel_res", C.c_double),
                ("rel_res_true", C.c_double), ("fnorm", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LimexOpts(C.Structure):
    _fields_ = [("stages", C.c_int32), ("maxit", C.c_int32), ("tol", C.c_double), ("safety", C.c_double),
                ("dt_max", C.c_double), ("rtol", C.c_double)]


class LimexStats(C.Structure):
    _fields_ = [("accepted", C.c_int32), ("solves", C.c_int32), ("iters_total", C.c_int32),
                ("unconverged", C.c_int32), ("eps", C.c_double), ("dt_used", C.c_double),
                ("dt_next", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class NewtonOpts(C.Structure):
    _fields_ = [("max_newton", C.c_int32), ("max_halvings", C.c_int32), ("maxit", C.c_int32),
                ("reserved", C.c_int32), ("atol", C.c_double), ("rtol", C.c_double), ("lin_rtol", C.c_double),
                ("xtol", C.c_double)]


class NewtonStats(C.Structure):
    _fields_ = [("converged", C.c_int32), ("newton", C.c_int32), ("halvings", C.c_int32),
                ("linear_solves", C.c_int32), ("linear_iters", C.c_int32), ("criterion", C.c_int32),
                ("defect0", C.c_double), ("defect", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class KernelTime(C.Structure):
    _fields_ = [("count", C.c_int32), ("reserved", C.c_int32), ("total_ms", C.c_double)]


KERNEL_CLASSES = ["assemble", "rap", "coarse_lu", "spmv64", "smooth0", "smooth0_first", "resid0",
                  "coarse_levels", "transfer0", "line0"]

VP = C.c_void_p
DP = C.c_void_p  # device pointers are passed as integers

_SIGS = {
    "tpf_last_error": (C.c_char_p, []),
    "tpf_validate": (C.c_int32, [C.POINTER(GridDesc)]),
    "tpf_grid_bytes": (C.c_size_t, [C.POINTER(GridDesc)]),
    "tpf_create_grid": (C.c_int32, [C.POINTER(GridDesc), VP, C.c_size_t, VP, C.POINTER(VP)]),
    "tpf_destroy_grid": (None, [VP]),
    "tpf_apply_dirichlet": (C.c_int32, [VP, DP, VP]),
    "tpf_residual": (C.c_int32, [VP, DP, DP, VP]),
    "tpf_assemble_stage": (C.c_int32, [VP, DP, C.c_double, DP, VP]),
    "tpf_rescale_stage": (C.c_int32, [VP, C.c_double, VP]),
    "tpf_solve_stage_static": (C.c_int32, [VP, DP, DP, C.c_double, C.c_int32, C.POINTER(SolveStats), VP]),
    "tpf_solve_stage": (C.c_int32, [VP, DP, DP, C.c_double, C.c_int32, C.POINTER(SolveStats), VP]),
    "tpf_limex_step": (C.c_int32, [VP, DP, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(LimexOpts),
                                   C.POINTER(LimexStats), VP]),
    "tpf_storage": (C.c_int32, [VP, DP, DP, VP]),
    "tpf_ie_step": (C.c_int32, [VP, DP, C.c_double, C.POINTER(NewtonOpts), C.POINTER(NewtonStats), VP]),
    "tpf_project_pressure": (C.c_int32, [VP, DP, C.c_double, C.POINTER(NewtonOpts), C.POINTER(NewtonStats), VP]),
    "tpf_set_coarse_graph": (C.c_int32, [VP, C.c_int32]),
    "tpf_set_line_pairs": (C.c_int32, [VP, C.c_int64]),
    "tpf_levels": (C.c_int32, [VP]),
    "tpf_level_dims": (C.c_int32, [VP, C.c_int32, C.POINTER(C.c_int32)]),
    "tpf_copy_matrix": (C.c_int32, [VP, C.c_int32, C.c_int32, DP, VP]),
    "tpf_spmv": (C.c_int32, [VP, C.c_int32, DP, DP, VP]),
    "tpf_precondition": (C.c_int32, [VP, DP, DP, VP]),
    "tpf_copy_coarse_inverse": (C.c_int32, [VP, DP, VP]),
    "tpf_pdmin_ptr": (VP, [VP]),
    "tpf_profile_begin": (C.c_int32, [VP, C.c_int32, C.c_uint32]),
    "tpf_profile_end": (C.c_int32, [VP, C.POINTER(KernelTime)]),
}

_lib = None


def load():
    """Loads libtpf.so (raises if it has not been built: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().tpf_last_error().decode()


class TPFError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {last_error()}")


def check(status, where, soft_ok=False):
    if status < 0 or (status > 0 and not soft_ok):
        raise TPFError(status, where)
    return status
