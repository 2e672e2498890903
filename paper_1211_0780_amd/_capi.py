"""ctypes declarations of libxy.so, the C ABI in include/xy.h.

Argument marshalling only: every step of the hot path runs in the HIP
kernels behind these entry points.  Importing this module fails loudly when
the library has not been built; there is no fallback implementation.
"""
import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libxy.so")

XY_OK, XY_ERR_ARG, XY_ERR_ODD_L, XY_ERR_OOM, XY_ERR_HIP, XY_ERR_STATE, XY_ERR_UNSUPPORTED = range(7)
XY_FP32, XY_FP64 = 0, 1
XY_START_RANDOM, XY_START_ORDERED = 0, 1
XY_F_NO_RECHECK = 0x1
XY_F_NO_FUSED_OR = 0x2

STATUS_NAMES = {0: "XY_OK", 1: "XY_ERR_ARG", 2: "XY_ERR_ODD_L", 3: "XY_ERR_OOM", 4: "XY_ERR_HIP",
                5: "XY_ERR_STATE", 6: "XY_ERR_UNSUPPORTED"}

EXPORTS = ["xy_angles_bytes", "xy_init", "xy_sweep", "xy_measure", "xy_exchange", "xy_run",
           "xy_get_angles", "xy_set_angles", "xy_get_counters", "xy_get_permutation",
           "xy_get_metro_accepts", "xy_get_state", "xy_set_state", "xy_last_error",
           "xy_destroy", "xy_set_tiling", "xy_get_tiling", "xy_sweep_profiled", "xy_autotune", "xy_get_sites", "xy_run_ex", "xy_get_bond_sums", "xy_get_swap_accepts", "xy_set_tiling_fused", "xy_get_tiling_fused",
           "xy_set_proposal_window", "xy_get_recheck_overflow", "xy_get_sites_noalloc",
           "xy_get_angles_fused_mid"]
XY_NOALLOC_MAX_SITES = 1 << 18


class XYConfig(ctypes.Structure):
    _fields_ = [
        ("n_lattices", ctypes.c_int32),
        ("L", ctypes.POINTER(ctypes.c_int32)),
        ("n_replicas", ctypes.POINTER(ctypes.c_int32)),
        ("beta", ctypes.POINTER(ctypes.c_double)),
        ("seed", ctypes.c_uint64),
        ("prec", ctypes.c_int32),
        ("start", ctypes.c_int32),
        ("angles_dev", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
        ("flags", ctypes.c_uint32),
    ]


class XYError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -m paper_1211_0780_amd.build_lib or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u32, i64p = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        cfgp = ctypes.POINTER(XYConfig)
        L.xy_angles_bytes.argtypes = [cfgp]
        L.xy_angles_bytes.restype = ctypes.c_size_t
        L.xy_init.argtypes = [cfgp, ctypes.POINTER(vp)]
        L.xy_init.restype = i32
        L.xy_sweep.argtypes = [vp, i32, i32]
        L.xy_sweep.restype = i32
        L.xy_measure.argtypes = [vp, vp, i32]
        L.xy_measure.restype = i32
        L.xy_exchange.argtypes = [vp, i64p]
        L.xy_exchange.restype = i32
        L.xy_run.argtypes = [vp, i32, i32, i32, i32, vp]
        L.xy_run.restype = i32
        L.xy_get_angles.argtypes = [vp, i32, i32, dp]
        L.xy_get_angles.restype = i32
        L.xy_get_angles_fused_mid.argtypes = [vp, i32, i32, dp]
        L.xy_get_angles_fused_mid.restype = i32
        L.xy_set_angles.argtypes = [vp, i32, i32, dp]
        L.xy_set_angles.restype = i32
        L.xy_get_counters.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
        L.xy_get_counters.restype = i32
        L.xy_get_permutation.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int32)]
        L.xy_get_permutation.restype = i32
        L.xy_get_metro_accepts.argtypes = [vp, i64p]
        L.xy_get_metro_accepts.restype = i32
        L.xy_get_recheck_overflow.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
        L.xy_get_recheck_overflow.restype = i32
        L.xy_get_state.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_size_t)]
        L.xy_get_state.restype = i32
        L.xy_set_state.argtypes = [vp, vp, ctypes.c_size_t]
        L.xy_set_state.restype = i32
        L.xy_last_error.argtypes = [vp]
        L.xy_last_error.restype = ctypes.c_char_p
        L.xy_set_tiling.argtypes = [vp, i32, i32, i32, i32]
        L.xy_set_tiling.restype = i32
        ip = ctypes.POINTER(ctypes.c_int32)
        L.xy_get_tiling.argtypes = [vp, i32, ip, ip, ip]
        L.xy_get_tiling.restype = i32
        L.xy_sweep_profiled.argtypes = [vp, i32, i32, dp, ip]
        L.xy_sweep_profiled.restype = i32
        L.xy_autotune.argtypes = [vp, i32, i32, i32]
        L.xy_autotune.restype = i32
        L.xy_get_sites.argtypes = [vp, i32, i32, ctypes.c_int64, i64p, dp]
        L.xy_get_sites.restype = i32
        L.xy_get_sites_noalloc.argtypes = [vp, i32, i32, ctypes.c_int64, i64p, dp]
        L.xy_get_sites_noalloc.restype = i32
        L.xy_run_ex.argtypes = [vp, i32, i32, i32, i32, vp, vp]
        L.xy_run_ex.restype = i32
        L.xy_get_bond_sums.argtypes = [vp, vp, i32]
        L.xy_get_bond_sums.restype = i32
        L.xy_get_swap_accepts.argtypes = [vp, i64p]
        L.xy_get_swap_accepts.restype = i32
        L.xy_set_tiling_fused.argtypes = [vp, i32, i32, i32]
        L.xy_set_tiling_fused.restype = i32
        L.xy_get_tiling_fused.argtypes = [vp, i32, ip, ip]
        L.xy_get_tiling_fused.restype = i32
        L.xy_set_proposal_window.argtypes = [vp, ctypes.c_double]
        L.xy_set_proposal_window.restype = i32
        L.xy_destroy.argtypes = [vp]
        L.xy_destroy.restype = None
        _lib = L
    return _lib


def check(status, ctx=None):
    if status != XY_OK:
        msg = lib().xy_last_error(ctx)
        raise XYError(status, msg.decode() if msg else "")
