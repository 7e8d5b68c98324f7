"""ctypes declarations of the C ABI in include/ah.h (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libah.so")

AH_OK = 0
AH_E_INVAL = -1
AH_E_NOMEM = -2
AH_E_DEVICE = -3
AH_E_STATE = -4
AH_E_AGAIN = -5

AH_FP64 = 0
AH_FP32 = 1
AH_COMPACT = 0
AH_NONCOMPACT = 1
AH_FLAG_UNSTABLE = 1
AH_FLAG_NONFINITE = 2


class ah_params(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int32), ("precision", ctypes.c_int32), ("gauge_action", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("dx", ctypes.c_double), ("deta", ctypes.c_double),
        ("lambda0", ctypes.c_double), ("e0", ctypes.c_double), ("sigma", ctypes.c_double),
        ("m", ctypes.c_double), ("alpha", ctypes.c_double),
        ("s_early", ctypes.c_double), ("s_late", ctypes.c_double), ("eta_switch", ctypes.c_double),
        ("eta0", ctypes.c_double), ("eta_ref", ctypes.c_double),
        ("damp_gamma", ctypes.c_double), ("eta_damp", ctypes.c_double),
    ]


class ah_measurement(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("eta", ctypes.c_double), ("a", ctypes.c_double), ("f", ctypes.c_double),
        ("winding_sum_abs", ctypes.c_int64), ("L_W", ctypes.c_double), ("xi_W", ctypes.c_double),
        ("sum_L", ctypes.c_double), ("xi_L", ctypes.c_double), ("R", ctypes.c_double), ("v2_phi", ctypes.c_double),
        ("energy", ctypes.c_double), ("e_kin", ctypes.c_double), ("e_grad", ctypes.c_double),
        ("e_pot", ctypes.c_double), ("e_el", ctypes.c_double), ("e_mag", ctypes.c_double),
        ("gauss_rms", ctypes.c_double), ("gauss_max", ctypes.c_double), ("gauss_rel", ctypes.c_double),
        ("nonfinite", ctypes.c_int64), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
        ("v2_omega", ctypes.c_double),
    ]


AH_KERNEL_AUTO = 0
AH_KERNEL_SITE = 1
AH_KERNEL_TILE = 2
AH_KERNEL_TILE2 = 3


class ah_step_config(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("zchunk", ctypes.c_int32)]


class ah_pool_info(ctypes.Structure):
    _fields_ = [("budget", ctypes.c_size_t), ("bytes_in_use", ctypes.c_size_t), ("largest_free", ctypes.c_size_t),
                ("active", ctypes.c_int32), ("max_slots", ctypes.c_int32), ("graph_launches", ctypes.c_int64),
                ("graph_captures", ctypes.c_int64)]


class AHError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def load():
    """Load libah.so; raises if the HIP library has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built: run paper_2005_14454_amd.build.build() "
                           "(or __graft_entry__.build()) first")
    # torch ships its own HIP runtime under the same soname as the system one
    # libah.so links against; whichever is loaded first serves the whole
    # process.  Importing torch first makes it torch's, the runtime that owns
    # the device memory and streams handed to the library (loading the system
    # one first leaves torch on a runtime it was not built with, and device
    # calls then fail).
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64
    sig = {
        "ah_params_default": ([P(ah_params)], ctypes.c_int),
        "ah_required_bytes": ([P(ah_params), P(ctypes.c_size_t)], ctypes.c_int),
        "ah_stability_margin": ([P(ah_params), i64, P(ctypes.c_double)], ctypes.c_int),
        "ah_create": ([P(ah_params), vp, ctypes.c_size_t, vp, P(vp)], ctypes.c_int),
        "ah_init": ([vp, ctypes.c_uint64], ctypes.c_int),
        "ah_set_state": ([vp, P(ctypes.c_double), i64], ctypes.c_int),
        "ah_get_state": ([vp, P(ctypes.c_double), P(i64)], ctypes.c_int),
        "ah_get_step": ([vp, P(i64)], ctypes.c_int),
        "ah_gather": ([vp, P(i64), i64, P(ctypes.c_double)], ctypes.c_int),
        "ah_gather_noalloc": ([vp, P(i64), i64, P(ctypes.c_double)], ctypes.c_int),
        "ah_step": ([vp, i64], ctypes.c_int),
        "ah_measure": ([vp, P(ah_measurement)], ctypes.c_int),
        "ah_step_measured": ([vp, i64, ctypes.c_int32, P(ah_measurement), ctypes.c_int32, P(ctypes.c_int32)],
                             ctypes.c_int),
        "ah_get_timing_split": ([vp, P(ctypes.c_double), P(i64)], ctypes.c_int),
        "ah_get_winding": ([vp, P(ctypes.c_int8)], ctypes.c_int),
        "ah_set_step_config": ([vp, P(ah_step_config)], ctypes.c_int),
        "ah_get_step_config": ([vp, P(ah_step_config)], ctypes.c_int),
        "ah_synchronize": ([vp], ctypes.c_int),
        "ah_set_timing": ([vp, ctypes.c_int], ctypes.c_int),
        "ah_get_timing": ([vp, P(ctypes.c_double), P(i64)], ctypes.c_int),
        "ah_destroy": ([vp], ctypes.c_int),
        "ah_autotune": ([P(ah_params), ctypes.c_int32, P(ah_step_config), P(ctypes.c_double)], ctypes.c_int),
        "ah_tune_lookup": ([P(ah_params), P(ah_step_config)], ctypes.c_int),
        "ah_tune_set": ([P(ah_params), P(ah_step_config)], ctypes.c_int),
        "ah_tune_clear": ([], ctypes.c_int),
        "ah_tune_save": ([ctypes.c_char_p], ctypes.c_int),
        "ah_tune_load": ([ctypes.c_char_p], ctypes.c_int),
        "ah_pool_create": ([ctypes.c_size_t, ctypes.c_int32, vp, P(vp)], ctypes.c_int),
        "ah_pool_footprint": ([P(ah_params), i64, ctypes.c_int32, P(ctypes.c_size_t)], ctypes.c_int),
        "ah_pool_submit": ([vp, P(ah_params), ctypes.c_uint64, i64, ctypes.c_int32, P(i64)], ctypes.c_int),
        "ah_pool_advance": ([vp, ctypes.c_int32], ctypes.c_int),
        "ah_pool_poll": ([vp, P(i64), ctypes.c_int32, P(ctypes.c_int32)], ctypes.c_int),
        "ah_pool_poll_async": ([vp, P(i64), ctypes.c_int32, P(ctypes.c_int32)], ctypes.c_int),
        "ah_pool_progress": ([vp, i64, P(i64), P(i64)], ctypes.c_int),
        "ah_pool_step_config": ([vp, i64, P(ah_step_config)], ctypes.c_int),
        "ah_pool_get_state": ([vp, i64, P(ctypes.c_double), P(i64)], ctypes.c_int),
        "ah_pool_results": ([vp, i64, P(ah_measurement), ctypes.c_int32, P(ctypes.c_int32)], ctypes.c_int),
        "ah_pool_stats": ([vp, P(ah_pool_info)], ctypes.c_int),
        "ah_pool_synchronize": ([vp], ctypes.c_int),
        "ah_pool_last_error": ([vp], ctypes.c_char_p),
        "ah_pool_destroy": ([vp], ctypes.c_int),
        "ah_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "ah_hbm_probe": ([ctypes.c_size_t, ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_double),
                          P(ctypes.c_double)], ctypes.c_int),
        "ah_last_error": ([vp], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(rc, handle=None, what="", pool=None):
    if rc == AH_OK:
        return
    lib = load()
    msg = lib.ah_strerror(rc).decode()
    if pool:
        detail = lib.ah_pool_last_error(pool).decode()
        if detail:
            msg = f"{msg}: {detail}"
    if handle:
        detail = lib.ah_last_error(handle).decode()
        if detail:
            msg = f"{msg}: {detail}"
    raise AHError(rc, f"{what}: {msg}" if what else msg)
