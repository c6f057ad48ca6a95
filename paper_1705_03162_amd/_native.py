"""ctypes binding of libswept.so (the C interface declared in include/swept.h).

Argument marshalling only: every step of every solve runs in the library's HIP
kernels.  The library is loaded on first use; if it has not been built the call
fails loudly (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libswept.so")

SW_OK, SW_EINVAL, SW_ENOMEM, SW_EDEVICE, SW_EUNSUPPORTED, SW_EBUSY, SW_ENOTREADY, SW_ENAN = (
    0, -1, -2, -3, -4, -5, -6, -7)
SW_HEAT, SW_KS, SW_EULER = 0, 1, 2
SW_PERIODIC, SW_DIRICHLET, SW_REFLECTIVE = 0, 1, 2
SW_PROBLEM_LIMITER_RECIPROCAL = 1
SW_TUNE_NO_GRAPH, SW_TUNE_CHECK_NAN, SW_TUNE_HYBRID, SW_TUNE_LDS = 1, 2, 4, 8
SW_NOALLOC_SCRATCH_BYTES = 32 << 20
SW_TICKET_QUEUED, SW_TICKET_RUNNING, SW_TICKET_DONE, SW_TICKET_FAILED, SW_TICKET_CANCELLED = range(5)


class SwProblem(ctypes.Structure):
    _fields_ = [
        ("scheme", ctypes.c_int32), ("bc", ctypes.c_int32),
        ("n", ctypes.c_int64), ("nsteps", ctypes.c_int64),
        ("dt", ctypes.c_double), ("dx", ctypes.c_double),
        ("alpha", ctypes.c_double), ("gamma", ctypes.c_double),
        ("bc_left", ctypes.c_double * 3), ("bc_right", ctypes.c_double * 3),
        ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
    ]


class SwTuning(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("threads", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("classic_threads", ctypes.c_int32)]


class SwPlanInfo(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("threads", ctypes.c_int32),
        ("points_per_lane", ctypes.c_int32), ("radius", ctypes.c_int32),
        ("substeps", ctypes.c_int32), ("nvars", ctypes.c_int32),
        ("swept_ok", ctypes.c_int32), ("classic_threads", ctypes.c_int32),
        ("nodes", ctypes.c_int64), ("levels", ctypes.c_int64),
        ("levels_per_phase", ctypes.c_int64), ("full_phases", ctypes.c_int64),
        ("remainder", ctypes.c_int64), ("swept_launches", ctypes.c_int64),
        ("classic_launches", ctypes.c_int64), ("scratch_bytes", ctypes.c_int64),
    ]


class SwBatchConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("points_per_lane", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


SW_BATCH_SERVE, SW_BATCH_PERSISTENT = 1, 2


class SwTicketInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("swept", ctypes.c_int32), ("width", ctypes.c_int32),
                ("phases", ctypes.c_int32), ("submit_s", ctypes.c_double),
                ("start_s", ctypes.c_double), ("end_s", ctypes.c_double),
                ("resident_bytes", ctypes.c_int64)]


def problem_struct(problem, limiter: int = 0) -> SwProblem:
    """Fill an sw_problem from any object with the workloads.Problem fields."""
    s = SwProblem()
    s.scheme = int(problem.scheme)
    s.bc = int(problem.bc)
    s.n = int(problem.n)
    s.nsteps = int(problem.nsteps)
    s.dt = float(problem.dt)
    s.dx = float(problem.dx)
    s.alpha = float(problem.alpha)
    s.gamma = float(problem.gamma)
    for v in range(3):
        s.bc_left[v] = float(problem.bc_left[v])
        s.bc_right[v] = float(problem.bc_right[v])
    s.flags = SW_PROBLEM_LIMITER_RECIPROCAL if limiter else 0
    s.reserved = 0
    return s


_lib = None

# exported symbol -> (restype, argtypes)
_VP = ctypes.c_void_p
SIGNATURES = {
    "swept_plan": (ctypes.c_int, [ctypes.POINTER(SwProblem), ctypes.POINTER(SwTuning),
                                  ctypes.POINTER(_VP)]),
    "swept_plan_info": (ctypes.c_int, [_VP, ctypes.POINTER(SwPlanInfo)]),
    "swept_solve": (ctypes.c_int, [_VP, _VP, _VP]),
    "classic_solve": (ctypes.c_int, [_VP, _VP, _VP]),
    "swept_plan_destroy": (None, [_VP]),
    "swept_profile_phase": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int32, _VP,
                                           ctypes.POINTER(ctypes.c_double)]),
    "swept_solve_noalloc": (ctypes.c_int, [ctypes.POINTER(SwProblem), ctypes.POINTER(SwTuning), _VP, _VP]),
    "batch_create": (ctypes.c_int, [ctypes.POINTER(SwBatchConfig), ctypes.POINTER(_VP)]),
    "batch_submit": (ctypes.c_int, [_VP, ctypes.POINTER(SwProblem), _VP,
                                    ctypes.POINTER(ctypes.c_uint64)]),
    "batch_submit_async": (ctypes.c_int, [_VP, ctypes.POINTER(SwProblem), _VP, _VP,
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "batch_run": (ctypes.c_int, [_VP, _VP]),
    "batch_poll": (ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]),
    "batch_wait": (ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.c_int64]),
    "batch_cancel": (ctypes.c_int, [_VP, ctypes.c_uint64]),
    "batch_ticket_info": (ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(SwTicketInfo)]),
    "batch_destroy": (None, [_VP]),
    "sw_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "sw_last_error": (ctypes.c_char_p, []),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name, None)
            if fn is None:   # older build: the entry point fails when called, not at load
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class SweptError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        msg = L.sw_strerror(status).decode()
        detail = L.sw_last_error().decode()
        super().__init__(f"{where}: {msg} ({status}): {detail}")
        self.status = status


def check(status: int, where: str) -> int:
    if status != SW_OK:
        raise SweptError(status, where)
    return status
