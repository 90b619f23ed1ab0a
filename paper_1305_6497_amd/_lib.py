"""ctypes declarations of the C ABI in include/dda.h (argument marshalling only)."""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdda.so")

DDA_OK = 0
DDA_EINVAL = -1
DDA_ENOMEM = -2
DDA_EDEVICE = -3
DDA_ENOTSUP = -4
DDA_NOT_CONVERGED = 1
DDA_WVALIDITY = 2

DDA_ALPHA_LDR = 0
DDA_ALPHA_CMRR = 1
DDA_ALPHA_FCD = 2
DDA_ALPHA_GKDLDR = 3

DDA_FP64 = 0
DDA_MIXED = 1
DDA_MIXED_V32 = 2

DDA_SHAPE_ELLIPSOID = 1
DDA_SHAPE_RCTGLPRSM = 2
DDA_SHAPE_CYLINDER1 = 3
DDA_SHAPE_HEX_PRISM = 4


class C64(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class TargetDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("n_sites", ctypes.c_int64),
                ("ijk", ctypes.POINTER(ctypes.c_int32)),
                ("comp", ctypes.POINTER(ctypes.c_uint8)),
                ("n_comp", ctypes.c_int32),
                ("m", ctypes.POINTER(C64)),
                ("kd", ctypes.c_double),
                ("alpha_kind", ctypes.c_int32),
                ("device", ctypes.c_int32)]


class Rhs(ctypes.Structure):
    _fields_ = [("khat", ctypes.c_double * 3), ("e", C64 * 3)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("solver", ctypes.c_int32), ("fold_records", ctypes.c_int32),
                ("x0", ctypes.c_void_p), ("jacobi", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("matvecs", ctypes.c_int32),
                ("outer", ctypes.c_int32), ("rel_resid", ctypes.c_double)]


class Far(ctypes.Structure):
    _fields_ = [("qsca", ctypes.c_double), ("g", ctypes.c_double), ("cos2", ctypes.c_double),
                ("n_theta", ctypes.c_int32), ("n_phi", ctypes.c_int32), ("qbk", ctypes.c_double)]


class Scat(ctypes.Structure):
    _fields_ = [("f", C64 * 2 * 2), ("s", C64 * 4), ("mueller", ctypes.c_double * 4 * 4)]


class Q(ctypes.Structure):
    _fields_ = [("qext", ctypes.c_double), ("qabs", ctypes.c_double), ("qsca", ctypes.c_double),
                ("aeff", ctypes.c_double), ("qpha", ctypes.c_double)]


class TargetInfo(ctypes.Structure):
    _fields_ = [("box", ctypes.c_int32 * 3), ("grid", ctypes.c_int32 * 3), ("n_sites", ctypes.c_int64),
                ("kd", ctypes.c_double), ("aeff", ctypes.c_double), ("device_bytes", ctypes.c_uint64),
                ("zpass_variant", ctypes.c_int32 * 2), ("xfwd_variant", ctypes.c_int32 * 2),
                ("xinv_variant", ctypes.c_int32 * 2)]


# (name, restype, argtypes) for every entry point declared in include/dda.h
_VP = ctypes.c_void_p
SIGNATURES = [
    ("dda_make_sites", ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), ctypes.c_int64]),
    ("dda_aeff", ctypes.c_double, [ctypes.c_int64]),
    ("dda_kd_from_x", ctypes.c_double, [ctypes.c_double, ctypes.c_int64]),
    ("dda_orientation_grid", ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_int32] + [ctypes.POINTER(ctypes.c_double)] * 4),
    ("dda_orient_rhs", ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.POINTER(C64),
                                      ctypes.c_int32, ctypes.POINTER(Rhs)]),
    ("dda_setup_target", ctypes.c_int, [ctypes.POINTER(TargetDesc), ctypes.POINTER(_VP)]),
    ("dda_footprint_bytes", ctypes.c_int, [ctypes.POINTER(TargetDesc), ctypes.c_int32, ctypes.POINTER(SolveOpts),
                                           ctypes.POINTER(ctypes.c_uint64)]),
    ("dda_target_get_info", ctypes.c_int, [_VP, ctypes.POINTER(TargetInfo)]),
    ("dda_set_plan_variant", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    ("dda_set_zpass_variant", ctypes.c_int, [_VP, ctypes.c_int32]),
    ("dda_set_pass_timing", ctypes.c_int, [_VP, ctypes.c_int32]),
    ("dda_get_pass_timing", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int64)]),
    ("dda_pass_plan", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int32)]),
    ("dda_zpass_plan", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    ("dda_solve", ctypes.c_int, [_VP, ctypes.POINTER(Rhs), ctypes.c_int32, ctypes.POINTER(SolveOpts), _VP,
                                 ctypes.POINTER(C64), _VP, ctypes.POINTER(SolveStats)]),
    ("dda_cross_sections", ctypes.c_int, [_VP, ctypes.POINTER(Rhs), ctypes.c_int32, _VP, ctypes.POINTER(C64), _VP,
                                          ctypes.POINTER(Q)]),
    ("dda_far_field", ctypes.c_int, [_VP, ctypes.POINTER(Rhs), ctypes.c_int32, _VP, ctypes.c_double, _VP,
                                     ctypes.POINTER(Far)]),
    ("dda_scattering_matrix", ctypes.c_int, [_VP, ctypes.POINTER(Rhs), _VP, ctypes.POINTER(ctypes.c_double),
                                             ctypes.c_int32, ctypes.POINTER(ctypes.c_double), _VP,
                                             ctypes.POINTER(Scat)]),
    ("dda_near_field", ctypes.c_int, [_VP, ctypes.POINTER(Rhs), ctypes.c_int32, _VP, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.c_int32, _VP, _VP]),
    ("dda_near_field_eb", ctypes.c_int, [_VP, ctypes.POINTER(Rhs), ctypes.c_int32, _VP,
                                         ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, _VP, _VP, _VP]),
    ("dda_apply", ctypes.c_int, [_VP, ctypes.POINTER(Rhs), ctypes.c_int32, ctypes.c_int32, _VP, _VP, _VP]),
    ("dda_apply_noalloc", ctypes.c_int, [_VP, ctypes.POINTER(Rhs), ctypes.c_int32, ctypes.c_int32, _VP, _VP, _VP]),
    ("dda_incident_field", ctypes.c_int, [_VP, ctypes.POINTER(Rhs), ctypes.c_int32, _VP, _VP]),
    ("dda_free_target", None, [_VP]),
    ("dda_profile_matvec", ctypes.c_int, [_VP, ctypes.POINTER(Rhs), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          _VP, _VP, _VP, ctypes.POINTER(ctypes.c_double)]),
    ("dda_fft_pencils", ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_double, _VP, _VP, _VP, ctypes.c_int32]),
    ("dda_next_smooth", ctypes.c_int32, [ctypes.c_int32]),
    ("dda_last_error", ctypes.c_char_p, []),
]

_lib = None


class DDAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dda error {code}: {msg}")
        self.code = code


def lib():
    """The loaded libdda.so.  Raises if it has not been built.

    PyTorch (when installed) is imported first: it ships its own HIP runtime
    with the same soname, and loading it before libdda.so makes both use that
    one runtime (two HIP runtimes in one process do not share devices).
    """
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code, ok=(DDA_OK,)):
    """Raise DDAError for a negative (or unexpected) status; return the code."""
    if code in ok:
        return code
    if code < 0:
        raise DDAError(code, lib().dda_last_error().decode())
    return code
