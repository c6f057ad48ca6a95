"""CPU oracle for the swept/classic stencil solvers -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library (`paper_1705_03162_amd`):
its arithmetic lives in `oracle.c` (plain C + OpenMP, binary64, no implicit FMA
contraction).  Each scheme of Appendices B-D is there in two rounding orders:
form="literal", the equation as printed, every operation rounded on its own;
and form="canonical" (the default), one fixed order with products fused into
the sums that consume them and the KS right-hand side collected by symmetric
stencil pair.  The canonical order is frozen: the GPU library has to reproduce
it bit for bit, which long chaotic KS runs need.  Exact-arithmetic tests tie
both forms to the printed equations one level at a time.

Parity pins (what checks this oracle against something other than itself) live
in `tests/test_oracle_*.py`.  One reading is not pinned by any printed value:
the orientation of the limiter ratio in Eqs. limitleft/limitright ("parity
unpinned" for that choice; both orientations are provided).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = [os.path.join(_HERE, "oracle.c")]
CFLAGS = ["-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-mfma",
          "-fPIC", "-shared", "-Wall"]


class _Problem(ctypes.Structure):
    _fields_ = [
        ("scheme", ctypes.c_int32), ("bc", ctypes.c_int32),
        ("n", ctypes.c_int64), ("nsteps", ctypes.c_int64),
        ("dt", ctypes.c_double), ("dx", ctypes.c_double),
        ("alpha", ctypes.c_double), ("gamma", ctypes.c_double),
        ("bc_left", ctypes.c_double * 3), ("bc_right", ctypes.c_double * 3),
        ("limiter", ctypes.c_int32), ("form", ctypes.c_int32),
    ]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (called by the package build step)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", *CFLAGS, *SOURCES, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(LIB_PATH)
        lib.oracle_solve_timed.argtypes = [ctypes.POINTER(_Problem),
                                           ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_double)]
        lib.oracle_solve_timed.restype = ctypes.c_int
        lib.oracle_stage.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), ctypes.c_int]
        lib.oracle_stage.restype = ctypes.c_int
        lib.oracle_euler_flux.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                          ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        lib.oracle_euler_flux.restype = None
        lib.oracle_threads.argtypes = [ctypes.c_int]
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


FORMS = {"canonical": 0, "literal": 1}


def _to_struct(problem, limiter: int, form: str = "canonical") -> _Problem:
    s = _Problem()
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
    s.limiter = int(limiter)
    s.form = FORMS[form]
    return s


def solve(problem, state: np.ndarray, nthreads: int = 0, limiter: int = 0,
          timed: bool = False, form: str = "canonical"):
    """Return the state after problem.nsteps steps (input array is not modified).

    `problem` is a `workloads.Problem`; `state` is float64 of shape (nvars, n).
    With timed=True returns (result, seconds_of_step_loop).
    """
    nv = 3 if problem.scheme == 2 else 1
    out = np.array(state, dtype=np.float64, order="C", copy=True).reshape(nv, problem.n)
    s = _to_struct(problem, limiter, form)
    secs = ctypes.c_double(0.0)
    rc = _load().oracle_solve_timed(ctypes.byref(s),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    int(nthreads), ctypes.byref(secs))
    if rc != 0:
        raise ValueError("oracle_solve rejected the problem")
    return (out, secs.value) if timed else out


def stage(problem, src: np.ndarray, base: Optional[np.ndarray] = None, final: bool = False,
          limiter: int = 0, form: str = "canonical", nthreads: int = 1) -> np.ndarray:
    """One sub-step: base + coef f(src) with coef dt/2 (predictor) or dt (final);
    for the heat equation the next FTCS level of src (base ignored)."""
    nv = 3 if problem.scheme == 2 else 1
    src = np.ascontiguousarray(np.asarray(src, dtype=np.float64).reshape(nv, problem.n))
    base = src if base is None else np.ascontiguousarray(
        np.asarray(base, dtype=np.float64).reshape(nv, problem.n))
    out = np.empty_like(src)
    s = _to_struct(problem, limiter, form)
    P = ctypes.POINTER(ctypes.c_double)
    rc = _load().oracle_stage(ctypes.byref(s), 1 if final else 0, src.ctypes.data_as(P),
                              base.ctypes.data_as(P), out.ctypes.data_as(P), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_stage rejected the problem")
    return out


def euler_flux(cells, gamma: float = 1.4, limiter: int = 0) -> np.ndarray:
    """Interface flux between cells[1] and cells[2]; cells is (4, 3) conserved states."""
    c = np.ascontiguousarray(np.asarray(cells, dtype=np.float64).reshape(4, 3))
    out = np.zeros(3)
    _load().oracle_euler_flux(c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(gamma),
                              int(limiter), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def threads(nthreads: int = 0) -> int:
    return int(_load().oracle_threads(int(nthreads)))
