"""ctypes declarations of the C ABI in include/vanka_mg.h.

Loading fails loudly when libvanka_mg.so has not been built: there is no
fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("VMG_LIBRARY") or os.path.join(HERE, "libvanka_mg.so")

VMG_OK = 0
VMG_NOT_CONVERGED = 1
VMG_INVALID_ARG = -1
VMG_HIP_ERROR = -2
VMG_OOM = -3
VMG_SINGULAR = -4
VMG_NAN_DETECTED = -5

OP_SWEEP = 0
OP_RESIDUAL = 1
OP_RESTRICT_RESIDUAL = 2
OP_PROLONG_CORRECT = 3
OP_COARSE_SOLVE = 4
OP_CYCLE = 5

KERNEL_CLASSES = ["sweep", "restrict", "prolong", "norm", "coarse", "pack", "transform", "ir", "down", "up", "edge"]
NUM_KCLASS = len(KERNEL_CLASSES)

EXPORTED = ["vanka_mg_default_opts", "vanka_mg_setup", "vanka_mg_solve", "paradiag_apply",
            "vanka_mg_shift_gradient", "paradiag_heat_residual", "paradiag_heat_solve", "paradiag_heat_gmres",
            "paradiag_transform", "paradiag_transform_noalloc", "paradiag_transform_circulant", "paradiag_apply_circulant",
            "vanka_mg_apply_op", "vanka_mg_set_timing", "vanka_mg_set_timing_mask", "vanka_mg_kernel_stats",
            "vanka_mg_level_stats", "vanka_mg_autotune", "vanka_mg_schedule", "vanka_mg_plan", "vanka_mg_set_omega", "vanka_mg_set_shifts",
            "vanka_mg_lfa_omega", "vanka_mg_optimize_omega", "vanka_mg_levels", "vanka_mg_last_stats", "vanka_mg_destroy", "vanka_mg_error_string"]


class VmgGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("h", ctypes.c_double),
                ("levels", ctypes.c_int32), ("num_systems", ctypes.c_int32)]


class VmgOpts(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32),
                ("gamma", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("smoother", ctypes.c_int32), ("ir_inner", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("graphs", ctypes.c_int32)]


_lib = None


def load():
    """Load the library once and declare every signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                           "(python -m paper_2203_11154_amd._build)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pi32 = ctypes.POINTER(ctypes.c_int32)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    pdbl = ctypes.POINTER(ctypes.c_double)
    lib.vanka_mg_default_opts.argtypes = [ctypes.POINTER(VmgOpts)]
    lib.vanka_mg_setup.argtypes = [ctypes.POINTER(VmgGrid), i32, pdbl, ctypes.POINTER(VmgOpts), vp,
                                   ctypes.POINTER(vp)]
    lib.vanka_mg_solve.argtypes = [vp, vp, vp, dbl, i32, pi32, pi32, pdbl, vp]
    lib.paradiag_apply.argtypes = [vp, vp, vp, vp, vp, dbl, i32, pi32, vp]
    lib.vanka_mg_shift_gradient.argtypes = [vp, vp, vp, vp, vp]
    lib.paradiag_heat_residual.argtypes = [vp, dbl, vp, vp, vp, i32, pdbl, vp]
    lib.paradiag_heat_solve.argtypes = [vp, vp, vp, dbl, vp, vp, dbl, dbl, i32, i32, i32, pi32, pdbl, vp]
    lib.paradiag_heat_gmres.argtypes = [vp, vp, vp, dbl, vp, vp, dbl, dbl, i32, i32, i32, pi32, pdbl, vp]
    lib.paradiag_transform.argtypes = [i32, i64, vp, i32, vp, vp, vp]
    lib.paradiag_transform_noalloc.argtypes = [i32, i64, vp, i32, vp, vp, vp]
    lib.paradiag_transform_circulant.argtypes = [i32, i64, dbl, i32, i32, vp, vp, vp]
    lib.paradiag_apply_circulant.argtypes = [vp, dbl, vp, vp, dbl, i32, pi32, vp]
    lib.vanka_mg_apply_op.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp]
    lib.vanka_mg_set_timing.argtypes = [vp, i32, i32]
    lib.vanka_mg_set_timing_mask.argtypes = [vp, i32]
    lib.vanka_mg_kernel_stats.argtypes = [vp, pi64, pdbl, pdbl]
    lib.vanka_mg_level_stats.argtypes = [vp, i32, i32, pi64, pdbl, pdbl]
    lib.vanka_mg_levels.argtypes = [vp, i32, pi32, pi32, pi32]
    lib.vanka_mg_autotune.argtypes = [vp, ctypes.c_char_p, vp]
    lib.vanka_mg_set_omega.argtypes = [vp, pdbl]
    lib.vanka_mg_set_shifts.argtypes = [vp, pdbl]
    lib.vanka_mg_lfa_omega.argtypes = [pdbl, i32, i32, pdbl, pdbl]
    lib.vanka_mg_optimize_omega.argtypes = [vp, i32]
    lib.vanka_mg_schedule.argtypes = [vp, i32, i32, pi32]
    lib.vanka_mg_plan.argtypes = [vp, i32, pi32, pi32]
    lib.vanka_mg_last_stats.argtypes = [vp, pi32, pdbl, vp]
    lib.vanka_mg_destroy.argtypes = [vp]
    lib.vanka_mg_error_string.argtypes = [ctypes.c_int]
    lib.vanka_mg_error_string.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name != "vanka_mg_error_string":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class VankaMGError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = load().vanka_mg_error_string(code).decode()
        super().__init__(f"{where}: {msg} (code {code})")


def check(code, where):
    """Raise on a negative status; return the code otherwise."""
    if code < 0:
        raise VankaMGError(code, where)
    return code
