"""ctypes view of include/st_api.h.  Argument marshalling only: every step of
the solver runs inside libst.so; a missing library is an error, never a
fallback."""
import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libst.so")

ST_OK, ST_NOT_CONVERGED = 0, 1
ST_ERR_ARG, ST_ERR_OOM, ST_ERR_HIP, ST_ERR_BREAKDOWN, ST_ERR_STATE = -1, -2, -3, -4, -5
ST_FP64, ST_MIXED = 0, 1
ST_EDGE_X1_LO, ST_EDGE_X1_HI, ST_EDGE_X2_LO, ST_EDGE_X2_HI = 0, 1, 2, 3
ST_FLAG_TIME_KERNELS, ST_FLAG_NO_PLANE_DEDUP, ST_FLAG_COARSE_GMRES, ST_FLAG_FULL_COARSENING = 1, 2, 4, 8
ST_FLAG_SSTEP_SMOOTHER, ST_FLAG_OUTER_CGS2, ST_FLAG_ROW_MARCH = 16, 32, 64
ST_MAX_LEVELS, ST_MAX_PATCHES, ST_MAX_HIST, ST_NUM_KCLASS = 32, 4, 1024, 12

KCLASS_NAMES = ["fine_apply_fp64", "fine_apply_vcycle", "stencil_apply", "smooth_mdot_l0",
                "smooth_maxpy_l0", "transfer", "coarse_solve", "cast", "smooth_mdot_coarse",
                "smooth_maxpy_coarse", "fgmres_orth", "update"]


class st_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nt", C.c_int32),
                ("dx", C.c_double), ("dt", C.c_double)]


class st_material(C.Structure):
    _fields_ = [("k_ins", C.c_double), ("k_con", C.c_double), ("p_k", C.c_double),
                ("c_ins", C.c_double), ("c_con", C.c_double), ("p_c", C.c_double)]


class st_patch(C.Structure):
    _fields_ = [("edge", C.c_int32), ("centre", C.c_double), ("half_width", C.c_double)]


class st_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("bf16_from_level", C.c_int32), ("restart", C.c_int32),
                ("rtol", C.c_double), ("max_it", C.c_int32), ("smooth_its", C.c_int32),
                ("smooth_rtol", C.c_double), ("coarse_max_it", C.c_int32),
                ("coarse_rtol", C.c_double), ("coarse_restart", C.c_int32),
                ("lambda_crit", C.c_double), ("max_levels", C.c_int32),
                ("max_coarse_nodes", C.c_int64), ("filter_r", C.c_double), ("flags", C.c_int32),
                ("proj_beta", C.c_double), ("proj_eta", C.c_double),
                ("filter_max_it", C.c_int32), ("filter_rtol", C.c_double)]


class st_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32), ("levels", C.c_int32),
                ("level_dims", (C.c_int32 * 3) * ST_MAX_LEVELS),
                ("level_planes", C.c_int32 * ST_MAX_LEVELS),
                ("rel_res_est", C.c_double), ("true_rel_res", C.c_double),
                ("rhs_norm", C.c_double), ("t_setup_s", C.c_double), ("t_solve_s", C.c_double),
                ("n_hist", C.c_int32), ("res_hist", C.c_double * ST_MAX_HIST),
                ("kclass_ms", C.c_double * ST_NUM_KCLASS),
                ("kclass_launches", C.c_int64 * ST_NUM_KCLASS),
                ("kclass_bytes", C.c_int64 * ST_NUM_KCLASS)]


_P = C.c_void_p
_SIGS = {
    "st_opts_default": (None, [C.POINTER(st_opts)]),
    "st_status_string": (C.c_char_p, [C.c_int]),
    "st_footprint_bytes": (C.c_int, [C.POINTER(st_grid), C.POINTER(st_material),
                                     C.POINTER(st_opts), C.c_int32, C.POINTER(C.c_size_t)]),
    "st_setup": (C.c_int, [C.POINTER(st_grid), C.POINTER(st_material), _P, C.c_int32, _P, _P,
                           C.c_double, C.POINTER(st_patch), C.c_int32, C.POINTER(st_opts), _P,
                           C.c_size_t, _P, C.POINTER(_P)]),
    "st_update_density": (C.c_int, [_P, _P]),
    "st_solve": (C.c_int, [_P, _P, C.POINTER(st_info)]),
    "st_adjoint_solve": (C.c_int, [_P, _P, _P, C.POINTER(st_info)]),
    "st_sensitivity": (C.c_int, [_P, _P, _P, _P]),
    "st_objective": (C.c_int, [_P, _P, C.POINTER(C.c_double)]),
    "st_load_vector": (C.c_int, [_P, _P]),
    "st_pnorm": (C.c_int, [_P, _P, C.c_double, C.POINTER(C.c_double), _P]),
    "st_volume": (C.c_int, [_P, C.c_double, C.POINTER(C.c_double), _P]),
    "st_filter": (C.c_int, [_P, _P, _P]),
    "st_hierarchy": (C.c_int, [_P, C.POINTER(st_info)]),
    "st_set_flags": (C.c_int, [_P, C.c_int32]),
    "st_set_stream": (C.c_int, [_P, _P]),
    "st_destroy": (None, [_P]),
    "st_debug_apply": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, _P, _P]),
    "st_debug_stencil": (C.c_int, [_P, C.c_int32, _P]),
    "st_debug_diag": (C.c_int, [_P, C.c_int32, _P, _P]),
    "st_debug_transfer": (C.c_int, [_P, C.c_int32, C.c_int32, _P, _P]),
    "st_debug_smooth": (C.c_int, [_P, C.c_int32, C.c_int32, _P, _P, C.c_int32, C.c_int32,
                                  C.c_double]),
    "st_debug_vcycle": (C.c_int, [_P, C.c_int32, _P, _P]),
    "st_abi_sizes": (C.c_int, [C.POINTER(C.c_size_t), C.c_int32]),
    "st_solve_noalloc": (C.c_int, [C.POINTER(st_grid), C.POINTER(st_material), _P, C.c_int32, _P,
                                   _P, C.c_double, C.POINTER(st_patch), C.c_int32,
                                   C.POINTER(st_opts), _P, _P, C.POINTER(st_info)]),
}

_lib = None


class StError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed: {status_string(code)} ({code})")
        self.code = code


def load():
    """Load libst.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2508_09589_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def status_string(code):
    return load().st_status_string(int(code)).decode()


def check(fn, code, allow_not_converged=False):
    if code == ST_OK or (allow_not_converged and code == ST_NOT_CONVERGED):
        return code
    raise StError(fn, code)


def default_opts():
    o = st_opts()
    load().st_opts_default(C.byref(o))
    return o
