"""ctypes declarations of include/agg.h.  Loads the in-tree libagg.so and fails
loudly when it is missing: there is no other implementation to fall back to."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libagg.so")
AGG_MAX_D = 8

AGG_OK, AGG_PENDING = 0, 1
AGG_EINVAL, AGG_ENOMEM, AGG_EHIP, AGG_ENONFINITE = -1, -2, -3, -4
AGG_ENOTFOUND, AGG_ECANCELLED, AGG_EUNSUPPORTED = -5, -6, -7
STATUS_NAMES = {0: "AGG_OK", 1: "AGG_PENDING", -1: "AGG_EINVAL", -2: "AGG_ENOMEM", -3: "AGG_EHIP",
                -4: "AGG_ENONFINITE", -5: "AGG_ENOTFOUND", -6: "AGG_ECANCELLED",
                -7: "AGG_EUNSUPPORTED"}
PREC = {"fp64": 0, "fp32": 1, "fp32c": 2}

DP = ctypes.POINTER(ctypes.c_double)


class agg_term(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("rank", ctypes.c_int32), ("U", DP * AGG_MAX_D), ("weight", DP)]


KERNEL_FN = ctypes.CFUNCTYPE(None, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, ctypes.c_int32,
                             ctypes.POINTER(ctypes.c_double), ctypes.c_void_p)


class agg_tt_term(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("ranks", ctypes.c_int32 * (AGG_MAX_D + 1)), ("H", DP * AGG_MAX_D)]


class agg_solve_stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("rhs_evals", ctypes.c_int64), ("t_final", ctypes.c_double),
                ("m0_initial", ctypes.c_double), ("m1_initial", ctypes.c_double),
                ("m0_final", ctypes.c_double), ("m1_final", ctypes.c_double),
                ("nonfinite", ctypes.c_int64)]


class agg_engine_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("mem_budget", ctypes.c_int64), ("max_slots", ctypes.c_int32)]


class agg_request_stats(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_finish", ctypes.c_double),
                ("steps", ctypes.c_int64), ("status", ctypes.c_int32)]


# (name, restype, argtypes) of every export declared in include/agg.h
EXPORTS = [
    ("agg_plan_create", ctypes.c_int32, [ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(agg_term), ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    ("agg_plan_create_tt", ctypes.c_int32, [ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(agg_tt_term),
                                            ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_void_p)]),
    ("agg_plan_tables_tt", ctypes.c_int32, [ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(agg_tt_term),
                                            ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                            ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    ("agg_plan_destroy", ctypes.c_int32, [ctypes.c_void_p]),
    ("agg_plan_set_tilt", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_double]),
    ("agg_rhs", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("agg_rhs_noalloc", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    ("agg_rk2_step", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double]),
    ("agg_solve", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                   ctypes.POINTER(agg_solve_stats)]),
    ("agg_profile_pass", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_double)]),
    ("agg_plan_tables", ctypes.c_int32, [ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(agg_term), ctypes.c_int32,
                                         ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_int64)]),
    ("agg_twiddles", ctypes.c_int32, [ctypes.c_int64, DP]),
    ("agg_expsum_fit", ctypes.c_int32, [DP, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                        DP, DP, DP]),
    ("agg_tt_expand", ctypes.c_int32, [ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(DP), ctypes.c_int64, DP, ctypes.POINTER(ctypes.c_int64)]),
    ("agg_tt_cross", ctypes.c_int32, [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                      ctypes.POINTER(ctypes.c_int32), DP, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_int64), DP]),
    ("agg_engine_create", ctypes.c_int32, [ctypes.POINTER(agg_engine_config), ctypes.POINTER(ctypes.c_void_p)]),
    ("agg_engine_destroy", ctypes.c_int32, [ctypes.c_void_p]),
    ("agg_submit", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(agg_term),
                                    ctypes.c_int32, DP, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_uint64)]),
    ("agg_submit_tt", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(agg_tt_term),
                                       ctypes.c_int32, DP, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_uint64)]),
    ("agg_poll", ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64, DP, ctypes.POINTER(agg_request_stats)]),
    ("agg_engine_counters", ctypes.c_int32, [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int64)] * 4),
    ("agg_last_error", ctypes.c_char_p, []),
]

_lib = None


class AggError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    """The loaded libagg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python -m paper_1905_09071_amd.build); there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in EXPORTS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status < 0:
        raise AggError(status, lib().agg_last_error().decode(errors="replace"))
    return status
