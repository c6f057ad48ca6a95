"""Swept time-space decomposition of explicit 1D stencils on AMD MI355X (gfx950).

Python face of libswept.so (include/swept.h).  PyTorch only supplies device
memory and streams; every time step runs in the library's HIP kernels.

    import torch, paper_1705_03162_amd as sw, workloads as W
    prob, ic = W.cfg_sweep(W.KS, 20)
    state = torch.tensor(ic, dtype=torch.float64, device="cuda")
    with sw.Plan(prob) as plan:
        plan.swept(state)          # or plan.classic(state)
"""
from __future__ import annotations

import ctypes
from typing import Optional

from . import _native as N
from ._native import (SW_DIRICHLET, SW_EULER, SW_HEAT, SW_KS, SW_PERIODIC, SW_REFLECTIVE, SW_TUNE_CHECK_NAN,
                      SW_TUNE_HYBRID, SW_TUNE_LDS, SW_TUNE_NO_GRAPH, SweptError, problem_struct)

__all__ = ["Plan", "Batch", "swept_plan", "swept_solve", "classic_solve", "swept_solve_noalloc", "SweptError",
           "SW_HEAT", "SW_KS", "SW_EULER", "SW_PERIODIC", "SW_DIRICHLET", "SW_REFLECTIVE",
           "SW_TUNE_NO_GRAPH", "SW_TUNE_CHECK_NAN", "SW_TUNE_HYBRID", "SW_TUNE_LDS"]


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _state_ptr(state, problem) -> int:
    import torch
    if not isinstance(state, torch.Tensor):
        raise TypeError("state must be a torch tensor")
    if state.dtype != torch.float64 or not state.is_cuda or not state.is_contiguous():
        raise ValueError("state must be a contiguous float64 CUDA tensor")
    nv = 3 if problem.scheme == SW_EULER else 1
    if state.numel() != nv * problem.n:
        raise ValueError(f"state has {state.numel()} values, expected {nv}*{problem.n}")
    return state.data_ptr()


class Plan:
    """A validated problem with its tile shape, scratch memory and cached graphs."""

    def __init__(self, problem, width: int = 0, threads: int = 0, flags: int = 0,
                 limiter: int = 0, classic_threads: int = 0):
        self.problem = problem
        self._p = problem_struct(problem, limiter)
        tun = N.SwTuning(int(width), int(threads), int(flags), int(classic_threads))
        h = ctypes.c_void_p()
        N.check(N.lib().swept_plan(ctypes.byref(self._p), ctypes.byref(tun), ctypes.byref(h)),
                "swept_plan")
        self._h = h

    def info(self) -> dict:
        i = N.SwPlanInfo()
        N.check(N.lib().swept_plan_info(self._h, ctypes.byref(i)), "swept_plan_info")
        return {k: getattr(i, k) for k, _ in N.SwPlanInfo._fields_}

    def swept(self, state, stream=None):
        N.check(N.lib().swept_solve(self._h, _state_ptr(state, self.problem),
                                    _stream_handle(stream)), "swept_solve")
        return state

    def classic(self, state, stream=None):
        N.check(N.lib().classic_solve(self._h, _state_ptr(state, self.problem),
                                      _stream_handle(stream)), "classic_solve")
        return state

    def profile_phase(self, state, kind: int = 1, reps: int = 20, stream=None) -> float:
        """Mean duration (us) of `reps` launches of one phase kind (0 Up, 1 Diamond, 2 Down),
        timed with HIP events on the stream; leaves `state` unspecified."""
        us = ctypes.c_double()
        N.check(N.lib().swept_profile_phase(self._h, _state_ptr(state, self.problem), int(kind),
                                            int(reps), _stream_handle(stream), ctypes.byref(us)),
                "swept_profile_phase")
        return us.value

    def close(self):
        if getattr(self, "_h", None):
            N.lib().swept_plan_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def swept_plan(problem, width: int = 0, threads: int = 0, flags: int = 0, limiter: int = 0,
               classic_threads: int = 0) -> Plan:
    return Plan(problem, width, threads, flags, limiter, classic_threads)


def swept_solve(plan: Plan, state, stream=None):
    return plan.swept(state, stream)


def swept_solve_noalloc(problem, state, width: int = 0, threads: int = 0, limiter: int = 0,
                        stream=None):
    """The allocation-free swept solve (edges in the library's static device scratch)."""
    p = problem_struct(problem, limiter)
    tun = N.SwTuning(int(width), int(threads), 0)
    N.check(N.lib().swept_solve_noalloc(ctypes.byref(p), ctypes.byref(tun), _state_ptr(state, problem),
                                        _stream_handle(stream)), "swept_solve_noalloc")
    return state


def classic_solve(plan: Plan, state, stream=None):
    return plan.classic(state, stream)


class Batch:
    """Independent solves admitted under a device-memory budget (batch_* API).

    serve=False: queue solves with submit(), then run() executes them all (ensemble);
    persistent=True runs each tile group as one persistent launch with device-side
    dependency counters instead of one launch per phase index.
    serve=True: a worker thread admits and advances solves as they are submitted
    (continuous batching); use poll()/wait()/info().
    points_per_lane: one-wave tile shape of every solve (0: tuned per size class).
    """

    def __init__(self, budget_bytes: int, max_slots: int = 0, serve: bool = False,
                 persistent: bool = False, points_per_lane: int = 0):
        flags = (N.SW_BATCH_SERVE if serve else 0) | (N.SW_BATCH_PERSISTENT if persistent else 0)
        cfg = N.SwBatchConfig(int(budget_bytes), int(max_slots), flags, int(points_per_lane), 0)
        h = ctypes.c_void_p()
        N.check(N.lib().batch_create(ctypes.byref(cfg), ctypes.byref(h)), "batch_create")
        self._h = h
        self._keep = {}

    def submit(self, problem, state, limiter: int = 0, stream=None, asynchronous: bool = False) -> int:
        """Queue a solve.  asynchronous=True: the state may still be being written on
        `stream` (default: torch's current stream); the solve waits for that work."""
        p = problem_struct(problem, limiter)
        t = ctypes.c_uint64()
        if asynchronous:
            N.check(N.lib().batch_submit_async(self._h, ctypes.byref(p), _state_ptr(state, problem),
                                               _stream_handle(stream), ctypes.byref(t)), "batch_submit_async")
        else:
            N.check(N.lib().batch_submit(self._h, ctypes.byref(p), _state_ptr(state, problem),
                                         ctypes.byref(t)), "batch_submit")
        self._keep[t.value] = state
        return t.value

    def run(self, stream=None):
        N.check(N.lib().batch_run(self._h, _stream_handle(stream)), "batch_run")

    def poll(self, ticket: int) -> int:
        s = ctypes.c_int32()
        N.check(N.lib().batch_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(s)), "batch_poll")
        return s.value

    def wait(self, ticket: int, timeout_us: int = -1):
        N.check(N.lib().batch_wait(self._h, ctypes.c_uint64(ticket), int(timeout_us)), "batch_wait")

    def cancel(self, ticket: int):
        N.check(N.lib().batch_cancel(self._h, ctypes.c_uint64(ticket)), "batch_cancel")

    def info(self, ticket: int) -> dict:
        i = N.SwTicketInfo()
        N.check(N.lib().batch_ticket_info(self._h, ctypes.c_uint64(ticket), ctypes.byref(i)),
                "batch_ticket_info")
        return {k: getattr(i, k) for k, _ in N.SwTicketInfo._fields_}

    def close(self):
        if getattr(self, "_h", None):
            N.lib().batch_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
