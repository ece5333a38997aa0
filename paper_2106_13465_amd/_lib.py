"""ctypes binding of libhydro.so (include/hydro.h).  Argument marshalling only:
every step of the method runs in the library's HIP kernels.  There is no
fallback: if the library is missing, loading raises."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhydro.so")

HYDRO_BC_REFLECT, HYDRO_BC_OUTFLOW, HYDRO_BC_PERIODIC = 1, 2, 3
HYDRO_DIR_X, HYDRO_DIR_Y = 0, 1
HYDRO_F64, HYDRO_F32 = 0, 1
HYDRO_GUESS_PTR, HYDRO_GUESS_MLP = 0, 1
HYDRO_OK, HYDRO_EINVAL, HYDRO_ENOMEM, HYDRO_EDEVICE, HYDRO_ENONPHYS, HYDRO_ESTATE = 0, -1, -2, -3, -4, -5
HYDRO_MAX_NITER = 32
HYDRO_NOALLOC_MAX_GRIDS = 16
HYDRO_PHASE_DT, HYDRO_PHASE_SWEEP_X, HYDRO_PHASE_SWEEP_Y, HYDRO_NPHASES = 0, 1, 2, 3
PHASE_NAMES = ("dt", "sweep_x", "sweep_y")

ERROR_NAMES = {
    HYDRO_EINVAL: "HYDRO_EINVAL",
    HYDRO_ENOMEM: "HYDRO_ENOMEM",
    HYDRO_EDEVICE: "HYDRO_EDEVICE",
    HYDRO_ENONPHYS: "HYDRO_ENONPHYS",
    HYDRO_ESTATE: "HYDRO_ESTATE",
}


class hydro_options_t(ctypes.Structure):
    _fields_ = [
        ("niter", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("guess", ctypes.c_int),
        ("stats", ctypes.c_int),
        ("seg_x", ctypes.c_int),
        ("seg_y", ctypes.c_int),
        ("learned_gate", ctypes.c_double),
        ("limiter", ctypes.c_int),
        ("order", ctypes.c_int),
        ("riemann", ctypes.c_int),
        ("ysweep", ctypes.c_int),
    ]


HYDRO_LEARNED_GATE_DEFAULT = 1.0
HYDRO_LIMITER_MINMOD, HYDRO_LIMITER_MC, HYDRO_LIMITER_VANLEER = 0, 1, 2
HYDRO_ORDER_XY, HYDRO_ORDER_ALTERNATE = 0, 1
HYDRO_RIEMANN_TWO_SHOCK, HYDRO_RIEMANN_EXACT, HYDRO_RIEMANN_HLLC = 0, 1, 2
HYDRO_YSWEEP_MARCH, HYDRO_YSWEEP_TILE = 0, 1
HYDRO_MAX_SCALARS = 1


class hydro_stats_t(ctypes.Structure):
    _fields_ = [
        ("interfaces", ctypes.c_longlong),
        ("hist", ctypes.c_longlong * (HYDRO_MAX_NITER + 1)),
        ("fallbacks", ctypes.c_longlong),
        ("wave_hist", ctypes.c_longlong * (HYDRO_MAX_NITER + 1)),
    ]


class hydro_tune_t(ctypes.Structure):
    _fields_ = [
        ("seg_x", ctypes.c_int),
        ("seg_y", ctypes.c_int),
        ("blocks_x", ctypes.c_uint),
        ("blocks_y", ctypes.c_uint),
        ("ms_x", ctypes.c_double),
        ("ms_y", ctypes.c_double),
        ("candidates", ctypes.c_int),
        ("cached", ctypes.c_int),
    ]


class HydroError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_vp = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_L = ctypes.POINTER(ctypes.c_long)
_LL = ctypes.POINTER(ctypes.c_longlong)

SIGNATURES = {
    "hydro_create": (_vp, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int]),
    "hydro_destroy": (None, [_vp]),
    "hydro_last_error": (ctypes.c_char_p, []),
    "hydro_bind": (ctypes.c_int, [_vp, _vp, ctypes.c_long, ctypes.c_int, _vp]),
    "hydro_invalidate": (ctypes.c_int, [_vp]),
    "hydro_set_options": (ctypes.c_int, [_vp, ctypes.POINTER(hydro_options_t)]),
    "hydro_get_options": (ctypes.c_int, [_vp, ctypes.POINTER(hydro_options_t)]),
    "hydro_compute_dt": (ctypes.c_double, [_vp]),
    "hydro_sweep": (ctypes.c_int, [_vp, ctypes.c_int]),
    "hydro_step": (ctypes.c_int, [_vp]),
    "hydro_conserved_totals": (ctypes.c_int, [_vp, _D]),
    "hydro_set_scalars": (ctypes.c_int, [_vp, ctypes.c_int]),
    "hydro_get_clock": (ctypes.c_int, [_vp, _D, ctypes.POINTER(ctypes.c_long), _D]),
    "hydro_set_clock": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_long]),
    "hydro_riemann_stats": (ctypes.c_int, [_vp, ctypes.POINTER(hydro_stats_t), ctypes.c_int]),
    "hydro_graph_steps": (ctypes.c_int, [_vp, ctypes.c_int]),
    "hydro_set_profiling": (ctypes.c_int, [_vp, ctypes.c_int]),
    "hydro_get_profile": (ctypes.c_int, [_vp, _D, ctypes.POINTER(ctypes.c_longlong), ctypes.c_int]),
    "hydro_autotune": (ctypes.c_int, [_vp, ctypes.POINTER(hydro_tune_t), ctypes.c_int]),
    "hydro_step_noalloc": (ctypes.c_int, [ctypes.c_int, _I, _I, _I, _LL, _L, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_double, _vp, _vp, _vp, _vp,
                                          _vp]),
    # measurement: streaming copy
    "hydro_stream_copy": (ctypes.c_int, [_vp, _vp, ctypes.c_longlong, _vp]),
    # learned guess
    "hydro_mlp_dev_bytes": (ctypes.c_size_t, []),
    "hydro_mlp_pack": (ctypes.c_int, [_vp, _vp, _vp]),
    "hydro_mlp_features": (ctypes.c_int, [_vp, ctypes.c_longlong, ctypes.c_double, _vp, _vp, _vp]),
    "hydro_mlp_forward": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_longlong, _vp]),
    "hydro_mlp_grad_scratch_bytes": (ctypes.c_size_t, [ctypes.c_longlong]),
    "hydro_mlp_grad": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_longlong, _vp, _vp, _vp, _vp]),
    "hydro_mlp_adam": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_longlong, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double, _vp]),
    "hydro_set_mlp": (ctypes.c_int, [_vp, _vp]),
    "hydro_set_logger": (ctypes.c_int, [_vp, _vp, ctypes.c_longlong, ctypes.c_ulonglong,
                                        ctypes.c_double, ctypes.c_double]),
    "hydro_logger_count": (ctypes.c_longlong, [_vp]),
    # batches
    "hydro_batch_create": (_vp, [ctypes.c_int, _I, _I, ctypes.c_double, ctypes.c_double, _I]),
    "hydro_batch_destroy": (None, [_vp]),
    "hydro_batch_layout": (ctypes.c_longlong, [_vp, ctypes.c_int, _LL, _L]),
    "hydro_batch_bind": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp]),
    "hydro_batch_set_options": (ctypes.c_int, [_vp, ctypes.POINTER(hydro_options_t)]),
    "hydro_batch_set_scalars": (ctypes.c_int, [_vp, ctypes.c_int]),
    "hydro_batch_invalidate": (ctypes.c_int, [_vp]),
    "hydro_batch_compute_dt": (ctypes.c_int, [_vp, _D]),
    "hydro_batch_step": (ctypes.c_int, [_vp]),
    "hydro_batch_graph_steps": (ctypes.c_int, [_vp, ctypes.c_int]),
    "hydro_batch_totals": (ctypes.c_int, [_vp, _D]),
    "hydro_batch_get_clock": (ctypes.c_int, [_vp, _D, _L, _D]),
    "hydro_batch_riemann_stats": (ctypes.c_int, [_vp, ctypes.POINTER(hydro_stats_t), ctypes.c_int]),
    "hydro_batch_autotune": (ctypes.c_int, [_vp, ctypes.POINTER(hydro_tune_t), ctypes.c_int]),
    "hydro_batch_set_profiling": (ctypes.c_int, [_vp, ctypes.c_int]),
    "hydro_batch_get_profile": (ctypes.c_int, [_vp, _D, ctypes.POINTER(ctypes.c_longlong),
                                               ctypes.c_int]),
    "hydro_batch_set_mlp": (ctypes.c_int, [_vp, _vp]),
    "hydro_batch_set_logger": (ctypes.c_int, [_vp, _vp, ctypes.c_longlong, ctypes.c_ulonglong,
                                              ctypes.c_double, ctypes.c_double]),
    "hydro_batch_logger_count": (ctypes.c_longlong, [_vp]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libhydro.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2106_13465_amd.build` "
            "(there is no non-HIP fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().hydro_last_error().decode()


def check(rc) -> None:
    if rc != HYDRO_OK:
        raise HydroError(int(rc), last_error())
