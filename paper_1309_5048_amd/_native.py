"""ctypes binding of libstokes.so (include/stokes.h).  Argument marshalling only: every
step of the solver runs in the library's HIP kernels.  Device arrays are torch tensors
(float64, contiguous, on the current HIP device); the library works on torch's current
stream.  Loading fails loudly when the library has not been built."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstokes.so")

STOKES_OK = 0
STOKES_NOT_CONVERGED = 1
STOKES_EINVAL = -1
STOKES_ENOMEM = -2
STOKES_EHIP = -3
STOKES_EBREAKDOWN = -4

PC_IC0, PC_ICPCG, PC_JACOBI, PC_IDEAL, PC_JPCG, PC_PCGAQ, PC_IDEAL_A, PC_ICPCG_AQ = 0, 1, 2, 3, 4, 5, 6, 7
FP64, MIXED = 0, 1
CAVITY_LID, CAVITY_VERIFY = 0, 1
GEOMETRY_SQUARE, GEOMETRY_ANNULUS = 0, 1

# every exported entry point declared in include/stokes.h
EXPORTS = (
    "stokes_setup", "stokes_setup_geometry", "stokes_setup_nitsche", "stokes_sizes", "stokes_set_stream", "stokes_set_nu", "stokes_set_inner_tol",
    "stokes_set_refine_tol",
    "stokes_set_maxit", "stokes_set_restarts", "stokes_load", "stokes_load_cavity", "stokes_solve", "stokes_solve_batched", "stokes_solve_precision",
    "stokes_solve_noalloc",
    "stokes_solve_adjoint", "stokes_solve_adjoint_batched", "stokes_dnu_dot", "stokes_apply",
    "stokes_apply_precond", "stokes_export_csr", "stokes_export_pressure_mass", "stokes_levels",
    "stokes_profile", "stokes_last_error", "stokes_destroy",
)


class StokesInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("inner_iters_total", ctypes.c_int32), ("status", ctypes.c_int32),
                ("ic_shift_steps", ctypes.c_int32), ("refine_cycles", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("relres_est", ctypes.c_double),
                ("relres_true_2", ctypes.c_double), ("relres_true_Minv", ctypes.c_double),
                ("setup_ms", ctypes.c_double), ("solve_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StokesForcing(ctypes.Structure):
    _fields_ = [("manufactured", ctypes.c_int32), ("nmodes", ctypes.c_int32), ("amp", ctypes.c_void_p),
                ("wave", ctypes.c_void_p), ("phase", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libstokes.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libstokes.so not built: run `python -m paper_1309_5048_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "stokes_setup": (i32, [i32, i32, i32, dbl, P(vp)]),
        "stokes_setup_geometry": (i32, [i32, i32, i32, dbl, i32, P(vp)]),
        "stokes_setup_nitsche": (i32, [i32, i32, i32, dbl, i32, dbl, P(vp)]),
        "stokes_sizes": (i32, [vp, P(i64), P(i64)]),
        "stokes_set_stream": (i32, [vp, vp]),
        "stokes_set_nu": (i32, [vp, dbl]),
        "stokes_set_inner_tol": (i32, [vp, dbl]),
        "stokes_set_refine_tol": (i32, [vp, dbl]),
        "stokes_set_maxit": (i32, [vp, i32, i32]),
        "stokes_set_restarts": (i32, [vp, i32]),
        "stokes_load": (i32, [vp, P(StokesForcing), i32, vp]),
        "stokes_load_cavity": (i32, [vp, i32, vp]),
        "stokes_solve": (i32, [vp, vp, vp, vp, dbl, i32, P(StokesInfo)]),
        "stokes_solve_batched": (i32, [vp, i32, vp, vp, vp, dbl, i32, i32, vp]),
        "stokes_solve_precision": (i32, [vp, vp, vp, vp, dbl, i32, i32, P(StokesInfo)]),
        "stokes_solve_noalloc": (i32, [vp, vp, vp, vp, dbl, i32, P(StokesInfo)]),
        "stokes_solve_adjoint": (i32, [vp, vp, vp, dbl, i32, P(StokesInfo)]),
        "stokes_solve_adjoint_batched": (i32, [vp, i32, vp, vp, dbl, i32, vp]),
        "stokes_dnu_dot": (i32, [vp, i32, vp, vp, vp]),
        "stokes_apply": (i32, [vp, vp, vp]),
        "stokes_apply_precond": (i32, [vp, i32, vp, vp, P(i32)]),
        "stokes_export_csr": (i32, [vp, i32, P(i64), vp, vp, vp]),
        "stokes_export_pressure_mass": (i32, [vp, vp, vp]),
        "stokes_levels": (i32, [vp, P(i32), P(i32)]),
        "stokes_profile": (i32, [vp, i32, vp, vp]),
        "stokes_last_error": (ctypes.c_char_p, [vp]),
        "stokes_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L
