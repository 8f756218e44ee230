"""ctypes declarations of libthccp.so (include/thccp.h).  Argument
marshalling only: every step of the CP-ALS runs in the HIP library."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libthccp.so")

CPD_OK = 0
CPD_ERR_INVALID_ARG = -1
CPD_ERR_HIP = -2
CPD_ERR_NOT_SPD = -3
CPD_ERR_NONFINITE = -4
CPD_ERR_WORKSPACE = -5
CPD_ERR_UNSUPPORTED = -6

PRECISIONS = {"fp64": 0, "fp32": 1, "mixed": 2}

vp = ctypes.c_void_p
i32 = ctypes.c_int32


class CpdDesc(ctypes.Structure):
    _fields_ = [
        ("n", i32 * 4),
        ("r_thc", i32),
        ("r_cp", i32),
        ("X", vp * 4),
        ("Z", vp),
        ("init", vp * 4),
        ("precision", i32),
        ("tol", ctypes.c_double),
        ("fit_floor", ctypes.c_double),
        ("chol_fallback", i32),
        ("use_graph", i32),
        ("fit_every", i32),
        ("autotune", i32),
        ("solve_panel", i32),
        ("stream", vp),
        ("workspace", vp),
        ("workspace_bytes", ctypes.c_size_t),
        ("tied", i32),
        ("norm2", vp),
        ("fit_target", ctypes.c_double),
    ]


class CpdStats(ctypes.Structure):
    _fields_ = [
        ("sweeps", i32),
        ("converged", i32),
        ("fallbacks", i32),
        ("flags", i32),
        ("fit", ctypes.c_double),
        ("norm2", ctypes.c_double),
        ("inner", ctypes.c_double),
        ("model2", ctypes.c_double),
        ("cond_est", ctypes.c_double),
        ("fp64_path", i32),
        ("reserved", i32),
    ]


class CpdError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = _lib.cpd_status_string(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} ({code})")


_lib = None

EXPORTS = {
    "cpd_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(CpdDesc)]),
    "cpd_init": (i32, [ctypes.POINTER(CpdDesc), ctypes.POINTER(vp)]),
    "cpd_sweep": (i32, [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)]),
    "cpd_fit": (i32, [vp, ctypes.POINTER(ctypes.c_double)]),
    "cpd_get_factors": (i32, [vp, vp * 4, vp]),
    "cpd_set_factors": (i32, [vp, vp * 4, vp, ctypes.c_double, i32]),
    "cpd_stats": (i32, [vp, ctypes.POINTER(CpdStats)]),
    "cpd_mttkrp": (i32, [vp, i32, vp]),
    "cpd_kernel_times": (i32, [vp, i32, ctypes.POINTER(ctypes.c_double)]),
    "cpd_batch_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(CpdDesc), i32]),
    "cpd_batch_init": (i32, [ctypes.POINTER(CpdDesc), i32, vp, ctypes.c_size_t, ctypes.POINTER(vp)]),
    "cpd_batch_sweep": (i32, [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)]),
    "cpd_batch_states": (i32, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32), ctypes.POINTER(i32)]),
    "cpd_batch_count": (i32, [vp]),
    "cpd_batch_get_factors": (i32, [vp, i32, vp * 4, vp]),
    "cpd_batch_stats": (i32, [vp, i32, ctypes.POINTER(CpdStats)]),
    "cpd_autotune_log": (i32, [vp, ctypes.c_char_p, i32]),
    "cpd_lt_scale_rows": (i32, [vp, vp, i32, i32, ctypes.c_double, ctypes.c_double, vp, vp]),
    "cpd_lt_exchange_workspace": (ctypes.c_size_t, [i32, i32, i32, i32, i32, i32]),
    "cpd_df_to_thc": (i32, [i32, i32, vp, vp, vp, vp, vp, vp]),
    "cpd_lt_mp2_workspace": (ctypes.c_size_t, [i32, i32, i32, i32, i32, i32]),
    "cpd_lt_mp2": (i32, [i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, i32, i32, vp, vp, vp, vp, ctypes.c_size_t,
                         vp]),
    "cpd_lt_exchange": (i32, [i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                              vp, vp, vp, ctypes.c_size_t, vp]),
    "cpd_destroy": (i32, [vp]),
    "cpd_status_string": (ctypes.c_char_p, [i32]),
    "cpd_test_gemm": (i32, [i32, i32, i32, i32, vp, i32, i32, vp, vp, i32, i32, vp, i32, vp]),
    "cpd_test_solve_workspace": (ctypes.c_size_t, [i32, i32, i32]),
    "cpd_test_solve": (i32, [i32, i32, i32, vp, vp, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(i32), i32]),
    "cpd_test_flow_spin_limit": (i32, [i32]),
    "cpd_test_bwd_form": (i32, [i32]),
    "cpd_test_split_force": (i32, [i32]),
    "cpd_test_split_workspace": (ctypes.c_size_t, [i32, i32, i32]),
    "cpd_test_gemm_split": (i32, [i32, i32, i32, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp, i32, i32, i32]),
    "cpd_test_mfma_probe": (i32, [i32, i32, vp, vp, vp, vp]),
    "cpd_ws_workspace_size": (ctypes.c_size_t, [i32, i32, i32]),
    "cpd_ws_features": (i32, [i32, i32, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]),
    "cpd_ws_features_noalloc": (i32, [i32, i32, vp, vp, vp, vp, vp]),
    "cpd_ws_select_init": (i32, [ctypes.POINTER(i32), i32, i32, vp * 4, vp, vp, i32, ctypes.POINTER(vp * 4),
                                 ctypes.c_double, vp * 4, vp, ctypes.c_size_t, vp]),
    "cpd_ws_labels": (i32, [ctypes.POINTER(i32), i32, i32, vp * 4, vp * 4, vp, vp, vp, vp, vp,
                            ctypes.c_size_t, vp]),
    "cpd_ws_init": (i32, [ctypes.POINTER(i32), i32, i32, vp * 4, vp, vp, ctypes.POINTER(vp * 4), ctypes.c_double,
                          vp * 4, ctypes.POINTER(i32), vp, ctypes.c_size_t, vp]),
    "cpd_mlp_param_count": (i32, []),
    "cpd_mlp_workspace_size": (ctypes.c_size_t, [i32]),
    "cpd_mlp_packed_size": (ctypes.c_size_t, []),
    "cpd_mlp_forward": (i32, [vp, vp, vp, i32, vp, vp, ctypes.c_size_t, vp]),
    "cpd_mlp_loss": (i32, [vp, vp, vp, vp, vp, i32, vp, vp, vp, ctypes.c_size_t, vp]),
    "cpd_mlp_backward": (i32, [vp, vp, vp, vp, i32, vp, vp, ctypes.c_size_t, vp]),
    "cpd_mlp_adam": (i32, [vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                           ctypes.c_float, vp]),
    "cpd_mlp_pack": (i32, [vp, vp, vp]),
    "cpd_mlp_infer_bf16": (i32, [vp, vp, i32, vp, vp]),
}


def load():
    """Load libthccp.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2502_17683_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code, where):
    if code != CPD_OK:
        raise CpdError(code, where)
