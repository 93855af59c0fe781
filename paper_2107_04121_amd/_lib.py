"""ctypes binding of libfe_forms.so (the gfx950 C ABI declared in
include/fe_forms.h).  Argument marshalling only: every step of the evaluation
runs in the library's HIP kernels.  If the library is missing this module
raises; there is no fallback."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfe_forms.so")

CELLS = {"hex": 0, "tet": 1}
FORMS = {"mass": 0, "vmass": 1, "laplace": 2, "elasticity": 3, "wdot": 4,
         "convect": 5}
MODES = {"matrix": 0, "residual": 1, "eval": 2}
PRECS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
MATS = {None: 0, "none": 0, "iso_cell": 1, "iso_qp": 2, "voigt_qp": 3,
        "tensor_qp": 4}
FE_FORM_BILINEAR = 6
VARIANTS = {"auto": 0, "generic": 1, "mfma": 2, "sumfact": 3,
            "matrix_first": 4, "cellwise": 5, "mfma_jobs": 6, "mfma_ws": 7}
VARIANT_NAMES = {v: k for k, v in VARIANTS.items()}

FE_OK = 0
STATUS = {0: "FE_OK", 1: "FE_ERR_INVALID_ARG", 2: "FE_ERR_UNSUPPORTED",
          3: "FE_ERR_NONPOSITIVE_JACOBIAN", 4: "FE_ERR_INDEX_OUT_OF_RANGE",
          5: "FE_ERR_OUT_OF_MEMORY", 6: "FE_ERR_HIP", 7: "FE_ERR_NO_DEVICE"}

# every symbol the header declares, checked at load time
EXPORTS = ["fe_status_string", "fe_last_error", "fe_version",
           "fe_reference_sizes", "fe_reference_tables", "fe_plan_create",
           "fe_plan_create_ref", "fe_plan_create_bilinear", "fe_eval_sum",
           "fe_plan_info", "fe_plan_workspace_size", "fe_execute",
           "fe_execute_noalloc",
           "fe_plan_check", "fe_plan_destroy", "fe_incidence_create",
           "fe_incidence_destroy", "fe_assemble", "fe_pattern_create",
           "fe_pattern_info", "fe_pattern_copy", "fe_pattern_destroy",
           "fe_assemble_matrix",
           "fe_energy_grad_workspace_size", "fe_energy_grad",
           "fe_batch_create", "fe_batch_execute", "fe_batch_check",
           "fe_batch_tiles", "fe_batch_destroy"]


class FeError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        name = STATUS.get(status, str(status))
        super().__init__(f"{where}: {name}" + (f" ({detail})" if detail else
                                                ""))


class fe_options(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int), ("xcd_remap", ctypes.c_int),
                ("layout", ctypes.c_int), ("chunk", ctypes.c_int)]


class fe_reference(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_int), ("order", ctypes.c_int),
                ("n_basis", ctypes.c_int), ("n_qp", ctypes.c_int),
                ("weights", ctypes.POINTER(ctypes.c_double)),
                ("bf", ctypes.POINTER(ctypes.c_double)),
                ("bfg", ctypes.POINTER(ctypes.c_double))]


class fe_bilinear(ctypes.Structure):
    _fields_ = [("test_grad", ctypes.c_int), ("test_comp", ctypes.c_int),
                ("trial_grad", ctypes.c_int), ("trial_comp", ctypes.c_int),
                ("W0", ctypes.POINTER(ctypes.c_double)),
                ("P_test", ctypes.POINTER(ctypes.c_double)),
                ("P_trial", ctypes.POINTER(ctypes.c_double)),
                ("n_a", ctypes.c_int), ("n_b", ctypes.c_int),
                ("mat_transpose", ctypes.c_int)]


LAYOUTS = {"cell_major": 0, "cell_minor": 1}


class fe_group(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_int), ("order", ctypes.c_int),
                ("forms", ctypes.c_int), ("tile", ctypes.c_int),
                ("n_cells", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("coords", ctypes.c_void_p), ("conn", ctypes.c_void_p),
                ("material", ctypes.c_void_p), ("out_mass", ctypes.c_void_p),
                ("out_laplace", ctypes.c_void_p),
                ("out_elasticity", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libfe_forms.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own libamdhip64.so.7; importing it first makes the
    # library's NEEDED entry resolve to that same, already loaded runtime
    # (two HIP runtimes in one process leave torch without a device).
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} not found: build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    for name in EXPORTS:
        getattr(L, name)
    vp, i32, i64, sz = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                        ctypes.c_size_t)
    ip = ctypes.POINTER(ctypes.c_int)
    dp = ctypes.POINTER(ctypes.c_double)
    L.fe_status_string.restype = ctypes.c_char_p
    L.fe_status_string.argtypes = [i32]
    L.fe_last_error.restype = ctypes.c_char_p
    L.fe_version.restype = ctypes.c_char_p
    L.fe_reference_sizes.argtypes = [i32, i32, ip, ip]
    L.fe_reference_tables.argtypes = [i32, i32, dp, dp, dp, dp]
    L.fe_plan_create.argtypes = [i32, i32, i32, i32, i32, i32,
                                 ctypes.POINTER(fe_options),
                                 ctypes.POINTER(vp)]
    L.fe_plan_create_ref.argtypes = [ctypes.POINTER(fe_reference), i32, i32,
                                     i32, i32, ctypes.POINTER(fe_options),
                                     ctypes.POINTER(vp)]
    L.fe_plan_create_bilinear.argtypes = [i32, i32, i32, i32, i32,
                                          ctypes.POINTER(fe_bilinear),
                                          ctypes.POINTER(fe_options),
                                          ctypes.POINTER(vp)]
    L.fe_eval_sum.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, sz,
                              vp]
    L.fe_plan_info.argtypes = [vp, ip, ip, ip, ip, ip]
    L.fe_plan_workspace_size.argtypes = [vp, i64, ctypes.POINTER(sz)]
    L.fe_execute.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp, sz, vp]
    L.fe_execute_noalloc.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp,
                                     vp]
    L.fe_plan_check.argtypes = [vp, vp, vp]
    L.fe_plan_destroy.argtypes = [vp]
    dbl = ctypes.c_double
    L.fe_incidence_create.argtypes = [i64, i64, i32, vp, vp,
                                      ctypes.POINTER(vp)]
    L.fe_incidence_destroy.argtypes = [vp]
    L.fe_assemble.argtypes = [vp, i32, i32, vp, dbl, vp, vp]
    L.fe_pattern_create.argtypes = [i64, i64, i32, vp, vp, ctypes.POINTER(vp)]
    L.fe_pattern_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.fe_pattern_copy.argtypes = [vp, vp, vp, vp]
    L.fe_pattern_destroy.argtypes = [vp]
    L.fe_assemble_matrix.argtypes = [vp, vp, vp, i32, i32, vp, dbl, vp, vp]
    L.fe_energy_grad_workspace_size.argtypes = [vp, i64, ctypes.POINTER(sz)]
    L.fe_energy_grad.argtypes = [vp, vp, i64, i64, vp, vp, vp, vp, dbl, vp,
                                 vp, vp, sz, vp]
    L.fe_batch_create.argtypes = [i32, ctypes.POINTER(fe_group), i32, i32,
                                  ctypes.POINTER(vp)]
    L.fe_batch_execute.argtypes = [vp, vp]
    L.fe_batch_check.argtypes = [vp, vp]
    L.fe_batch_tiles.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_float), ip]
    L.fe_batch_destroy.argtypes = [vp]
    _lib = L
    return L


def check(status: int, where: str):
    if status != FE_OK:
        detail = lib().fe_last_error().decode(errors="replace")
        raise FeError(status, where, detail)
