"""ctypes view of the C ABI in include/mpde.h (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpde.so")

MPDE_OK, MPDE_WARN_NOT_CONVERGED = 0, 1
MPDE_ERR_INVALID_ARG, MPDE_ERR_UNSUPPORTED, MPDE_ERR_OUT_OF_MEMORY = -1, -2, -3
MPDE_ERR_HIP, MPDE_ERR_NO_DEVICE, MPDE_ERR_BAD_STATE, MPDE_ERR_NONFINITE = -4, -5, -6, -7
MPDE_F32, MPDE_F64 = 0, 1
MPDE_BC_NONE, MPDE_BC_DIRICHLET, MPDE_BC_PERIODIC = 0, 1, 2
BC_CODES = {"none": MPDE_BC_NONE, "dirichlet": MPDE_BC_DIRICHLET, "periodic": MPDE_BC_PERIODIC}

EXPORTS = ("mpde_default_options", "mpde_build", "mpde_solve", "mpde_solve_adjoint",
           "mpde_free", "mpde_last_error", "mpde_levels", "mpde_kernel_stats",
           "mpde_net_create", "mpde_net_train_step", "mpde_net_attach", "mpde_net_get", "mpde_net_set",
           "mpde_net_free", "mpde_conv3d", "mpde_conv3d_wgrad", "mpde_autotune", "mpde_time_operator")
NET_PARAMS = 3 * (27 * 16 * 16 + 16)


class Options(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("inner_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int32), ("max_inner", ctypes.c_int32),
                ("nu", ctypes.c_int32), ("coarse_min", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("max_levels", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("out_f64", ctypes.c_int32), ("graph", ctypes.c_int32), ("fused", ctypes.c_int32),
                ("time_chunks", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class KStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class Desc(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("ndim", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("shape", ctypes.POINTER(ctypes.c_int32)), ("step", ctypes.POINTER(ctypes.c_double)),
                ("bc_lo", ctypes.c_int32 * 3), ("bc_hi", ctypes.c_int32 * 3),
                ("mset", ctypes.c_uint32),
                ("coeff", ctypes.c_void_p), ("rhs", ctypes.c_void_p), ("bc_values", ctypes.c_void_p),
                ("stream", ctypes.c_void_p), ("opts", ctypes.POINTER(Options))]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.POINTER(ctypes.c_int32)), ("outer", ctypes.POINTER(ctypes.c_int32)),
                ("relres", ctypes.POINTER(ctypes.c_double)), ("status", ctypes.POINTER(ctypes.c_int32)),
                ("seconds", ctypes.c_double)]


_lib = None


class NativeLibraryMissing(RuntimeError):
    pass


def load():
    """Load libmpde.so from the package directory; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise NativeLibraryMissing(
            f"{LIB_PATH} not found: build it with `python -m paper_2502_18377_amd.build` "
            "(there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    lib.mpde_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.mpde_default_options.restype = ctypes.c_int
    lib.mpde_build.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(ctypes.c_void_p)]
    lib.mpde_build.restype = ctypes.c_int
    lib.mpde_solve.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Info)]
    lib.mpde_solve.restype = ctypes.c_int
    lib.mpde_solve_adjoint.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.POINTER(Info)]
    lib.mpde_solve_adjoint.restype = ctypes.c_int
    lib.mpde_free.argtypes = [ctypes.c_void_p]
    lib.mpde_free.restype = None
    lib.mpde_last_error.argtypes = []
    lib.mpde_last_error.restype = ctypes.c_char_p
    lib.mpde_levels.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.mpde_levels.restype = ctypes.c_int
    lib.mpde_kernel_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(KStat), ctypes.c_int32]
    lib.mpde_kernel_stats.restype = ctypes.c_int
    lib.mpde_time_operator.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.mpde_time_operator.restype = ctypes.c_int
    vp, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    lib.mpde_net_create.argtypes = [i32, u64, ctypes.POINTER(vp)]
    lib.mpde_net_train_step.argtypes = [vp, vp, i32, u64, dbl, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    lib.mpde_net_attach.argtypes = [vp, vp, i32]
    lib.mpde_net_get.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i64]
    lib.mpde_net_set.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i64]
    lib.mpde_net_free.argtypes = [vp]
    lib.mpde_net_free.restype = None
    lib.mpde_conv3d.argtypes = [vp, vp, vp, vp, vp, i32, i32, i32, i32, i32, i32, ctypes.POINTER(i32), vp]
    lib.mpde_conv3d_wgrad.argtypes = [vp, vp, vp, i32, i32, i32, i32, ctypes.POINTER(i32), vp]
    lib.mpde_autotune.argtypes = [vp, vp, ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    for f in ("mpde_autotune", "mpde_net_create", "mpde_net_train_step", "mpde_net_attach", "mpde_net_get", "mpde_net_set",
              "mpde_conv3d", "mpde_conv3d_wgrad"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


class MPDEError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mpde error {code}: {msg}")
        self.code = code


def check(code):
    if code < 0:
        raise MPDEError(code, load().mpde_last_error().decode(errors="replace"))
    return code
