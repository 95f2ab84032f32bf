"""ctypes loader and struct mirrors of include/gw.h.

Loads ``libgwmi.so`` from this package directory.  There is no fallback: if
the library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgwmi.so")

c_float_p = ctypes.POINTER(ctypes.c_float)

GW_OK, GW_EINVAL, GW_ENOMEM, GW_EDEVICE, GW_ENUMERIC, GW_ESTATE, GW_EUNSUPPORTED, GW_EBUSY, GW_ECANCELLED = range(9)
STATUS_NAMES = ["GW_OK", "GW_EINVAL", "GW_ENOMEM", "GW_EDEVICE", "GW_ENUMERIC", "GW_ESTATE",
                "GW_EUNSUPPORTED", "GW_EBUSY", "GW_ECANCELLED"]

PEN_SQEUCLID, PEN_POWER, PEN_FEATURES = 0, 1, 2
FP32, BF16, BF16X3 = 0, 1, 2
MODE_AUTO, MODE_SAFE, MODE_STABILISED = 0, 1, 2


class GwParams(ctypes.Structure):
    _fields_ = [
        ("eps_start", ctypes.c_double),
        ("eps_end", ctypes.c_double),
        ("n_outer", ctypes.c_int32),
        ("n_inner", ctypes.c_int32),
        ("symmetric", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("use_init_potentials", ctypes.c_int32),
        ("tol_gamma", ctypes.c_double),
        ("anneal_final", ctypes.c_int32),
        ("adaptive_inner", ctypes.c_int32),
    ]


class GwResult(ctypes.Structure):
    _fields_ = [
        ("f", ctypes.c_void_p),
        ("g", ctypes.c_void_p),
        ("gamma", ctypes.c_void_p),
        ("loss_lift", ctypes.c_double),
        ("egw_objective", ctypes.c_double),
        ("kl", ctypes.c_double),
        ("marginal_err", ctypes.c_double),
        ("constant_c", ctypes.c_double),
        ("sum_pi_nm", ctypes.c_double),
        ("gamma_step", ctypes.c_double),
        ("eps_final", ctypes.c_double),
        ("outer_done", ctypes.c_int32),
        ("dim_x", ctypes.c_int32),
        ("dim_y", ctypes.c_int32),
        ("safe_iters", ctypes.c_int32),
        ("n_inner_final", ctypes.c_int32),
        ("inner_doublings", ctypes.c_int32),
    ]


class GwSgwResult(ctypes.Structure):
    _fields_ = [
        ("sgw", ctypes.c_double),
        ("gw_xy", ctypes.c_double),
        ("gw_xx", ctypes.c_double),
        ("gw_yy", ctypes.c_double),
        ("marginal_err", ctypes.c_double),
        ("dim_x", ctypes.c_int32),
        ("dim_y", ctypes.c_int32),
    ]


class GwMsgwOpts(ctypes.Structure):
    _fields_ = [
        ("rho", ctypes.c_double),
        ("n_lloyd", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
    ]


class GwMsgwInfo(ctypes.Structure):
    _fields_ = [
        ("n_coarse", ctypes.c_int64),
        ("m_coarse", ctypes.c_int64),
        ("coarse_loss_lift", ctypes.c_double),
        ("coarse_egw_objective", ctypes.c_double),
        ("coarse_marginal_err", ctypes.c_double),
        ("ms_coarsen", ctypes.c_double),
        ("ms_coarse_solve", ctypes.c_double),
        ("ms_interpolate", ctypes.c_double),
        ("ms_fine_solve", ctypes.c_double),
    ]


class GwRequest(ctypes.Structure):
    _fields_ = [
        ("x", ctypes.c_void_p), ("n", ctypes.c_int64), ("dx", ctypes.c_int32), ("a", ctypes.c_void_p),
        ("y", ctypes.c_void_p), ("m", ctypes.c_int64), ("dy", ctypes.c_int32), ("b", ctypes.c_void_p),
        ("params", GwParams),
        ("penalty", ctypes.c_int32),
        ("p", ctypes.c_double),
        ("lifted_dim", ctypes.c_int32),
        ("n_landmarks", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("f", ctypes.c_void_p), ("g", ctypes.c_void_p), ("gamma", ctypes.c_void_p),
        ("gamma0", ctypes.c_void_p),
    ]


class GwServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
        ("cancelled", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
        ("active", ctypes.c_int32), ("queued", ctypes.c_int32),
        ("busy_seconds", ctypes.c_double),
        ("device_bytes", ctypes.c_uint64), ("peak_device_bytes", ctypes.c_uint64),
    ]


GW_PROF_CLASSES = 8
PROF_NAMES = ["pass_stab", "pass_safe", "combine", "covariance", "prologue", "check", "lift", "grad"]


class GwProfile(ctypes.Structure):
    _fields_ = [
        ("launches", ctypes.c_int64 * GW_PROF_CLASSES),
        ("milliseconds", ctypes.c_double * GW_PROF_CLASSES),
        ("entries_per_pass", ctypes.c_int64),
        ("idle_launches", ctypes.c_int64 * GW_PROF_CLASSES),
        ("idle_milliseconds", ctypes.c_double * GW_PROF_CLASSES),
    ]


# name -> (restype, argtypes); mirrors include/gw.h
SIGNATURES = {
    "gw_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t]),
    "gw_set_penalty": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_uint64]),
    "gw_set_landmarks": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]),
    "gw_seeded_landmarks": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int, ctypes.c_uint64,
                                           ctypes.POINTER(ctypes.c_int64)]),
    "gw_lift": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                               ctypes.c_void_p, ctypes.c_void_p]),
    "gw_feature_dim": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "gw_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                ctypes.POINTER(GwParams), ctypes.c_void_p, ctypes.POINTER(GwResult)]),
    "gw_solve_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.POINTER(GwParams), ctypes.c_void_p,
                                        ctypes.POINTER(GwResult)]),
    "gw_solve_begin": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.POINTER(GwParams), ctypes.c_void_p, ctypes.POINTER(GwResult)]),
    "gw_solve_advance": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int32)]),
    "gw_solve_end": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(GwResult)]),
    "gw_sgw": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                              ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                              ctypes.POINTER(GwParams), ctypes.POINTER(GwSgwResult)]),
    "gw_sgw_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                   ctypes.POINTER(GwParams), ctypes.POINTER(GwSgwResult), ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "gw_sgw_barycenter": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int,
                                         ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, ctypes.POINTER(GwParams),
                                         ctypes.POINTER(ctypes.c_double)]),
    "gw_kpca_full": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                    ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "gw_kmeans": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                 ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "gw_interpolate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_void_p]),
    "gw_msgw": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                               ctypes.POINTER(GwParams), ctypes.POINTER(GwParams), ctypes.POINTER(GwMsgwOpts),
                               ctypes.c_void_p, ctypes.POINTER(GwResult), ctypes.POINTER(GwMsgwInfo)]),
    "gw_loss_and_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.POINTER(GwParams), ctypes.c_void_p,
                                        ctypes.POINTER(GwResult), ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "gw_destroy": (None, [ctypes.c_void_p]),
    "gw_set_profiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "gw_get_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(GwProfile)]),
    "gw_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "gw_server_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "gw_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(GwRequest), ctypes.POINTER(ctypes.c_uint64)]),
    "gw_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(GwResult),
                                      ctypes.POINTER(ctypes.c_double)]),
    "gw_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(GwResult),
                                      ctypes.POINTER(ctypes.c_double)]),
    "gw_server_cancel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "gw_server_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(GwServerStats)]),
    "gw_server_destroy": (None, [ctypes.c_void_p]),
}

_LIB = None


def load(path: str | None = None):
    """Load libgwmi.so (raises if it is missing)."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libgwmi.so not found at {p}: build it with paper_2602_06658_amd/build.py")
    lib = ctypes.CDLL(p)
    missing = []
    for name, (res, args) in SIGNATURES.items():
        try:
            fn = getattr(lib, name)
        except AttributeError:
            missing.append(name)
            continue
        fn.restype = res
        fn.argtypes = args
    if missing:
        raise RuntimeError(f"{p} does not export {', '.join(missing)}: rebuild it")
    if path is None:
        _LIB = lib
    return lib


def exported_symbols(path: str | None = None) -> set[str]:
    """Names from SIGNATURES that the shared library exports."""
    lib = ctypes.CDLL(path or LIB_PATH)
    out = set()
    for name in SIGNATURES:
        try:
            getattr(lib, name)
            out.add(name)
        except AttributeError:
            pass
    return out


class GWError(RuntimeError):
    def __init__(self, code: int, msg: str):
        self.code = code
        name = STATUS_NAMES[code] if 0 <= code < len(STATUS_NAMES) else str(code)
        super().__init__(f"{name}: {msg}")


def seeded_landmarks(n: int, n_landmarks: int, seed: int):
    """Landmark indices the library's seeded choice gives for n points
    (gw_seeded_landmarks; host only): a sorted list of min(n_landmarks, n)
    indices."""
    lib = load()
    k = min(int(n_landmarks), int(n))
    out = (ctypes.c_int64 * max(k, 1))()
    rc = lib.gw_seeded_landmarks(int(n), int(n_landmarks), ctypes.c_uint64(seed), out)
    if rc != GW_OK:
        raise GWError(rc, "gw_seeded_landmarks failed")
    return [int(v) for v in out[:k]]
