"""The swept tile schedule, emulated on the host, equals the oracle bit for bit.

`tests/hostsim` runs the library's own launch sequence, tile geometry and
per-point rules on the CPU with a software work-group (no GPU).  Because the
swept rule performs the classic operations in a different order and place
(Sec. 2), the result must be bitwise identical to the oracle's classic
time-stepping for every tile shape, step count (full phases, remainders,
fewer levels than one phase) and boundary type.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import workloads as W
from paper_1705_03162_amd._native import SwProblem, problem_struct

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "hostsim", "hostsim.cpp")
# the library's host routine of the Hybrid variant, tested here on the CPU
HYBRID_SRC = os.path.join(ROOT, "paper_1705_03162_amd", "csrc", "hybrid.cpp")
LIB = os.path.join(HERE, "hostsim", "libhostsim.so")


def build_hostsim():
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wno-unknown-pragmas", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1705_03162_amd", "csrc"), SRC, HYBRID_SRC, "-o", f"{LIB}.{os.getpid()}.tmp"]
    subprocess.run(cmd, check=True)
    os.replace(f"{LIB}.{os.getpid()}.tmp", LIB)


@pytest.fixture(scope="module")
def hostsim():
    build_hostsim()
    L = ctypes.CDLL(LIB)
    L.hostsim_swept.argtypes = [ctypes.POINTER(SwProblem), ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_double)]
    L.hostsim_swept.restype = ctypes.c_int
    L.hostsim_swept_mode.argtypes = [ctypes.POINTER(SwProblem), ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    L.hostsim_swept_mode.restype = ctypes.c_int
    L.hostsim_dataflow.argtypes = [ctypes.POINTER(SwProblem), ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_double), ctypes.c_uint64]
    L.hostsim_dataflow.restype = ctypes.c_int
    L.hostsim_phases.argtypes = [ctypes.POINTER(SwProblem), ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_int32), ctypes.c_int]
    L.hostsim_phases.restype = ctypes.c_int
    return L


def emulate(L, prob, ic, width, threads, limiter=0):
    out = np.array(ic, dtype=np.float64, copy=True, order="C")
    s = problem_struct(prob, limiter)
    rc = L.hostsim_swept(ctypes.byref(s), width, threads,
                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == 0, rc
    return out


def phases(L, prob, width, threads):
    s = problem_struct(prob)
    buf = (ctypes.c_int32 * 3000)()
    cnt = L.hostsim_phases(ctypes.byref(s), width, threads, buf, 1000)
    return [tuple(buf[3 * i:3 * i + 3]) for i in range(cnt)]


HEAT_CASES = [  # (n, steps, width, threads)
    (64, 40, 64, 64),        # K = 1, several phases
    (256, 32, 64, 64),       # exactly one phase (Q = 1, no remainder)
    (256, 97, 64, 64),       # remainder
    (256, 5, 64, 64),        # fewer levels than a phase
    (512, 300, 128, 64),     # P = 2
    (1024, 777, 512, 64),    # P = 8
    (1024, 1000, 256, 128),  # two waves
    (2048, 1500, 1024, 256), # four waves, P = 4
    (1024, 1, 64, 64),
]


@pytest.mark.parametrize("n,steps,width,threads", HEAT_CASES)
@pytest.mark.parametrize("bc", [W.PERIODIC, W.DIRICHLET, W.REFLECTIVE])
def test_heat_swept_equals_oracle(hostsim, oracle_mod, n, steps, width, threads, bc):
    prob = W.heat_problem(n, steps, bc=bc, bc_left=0.3, bc_right=-0.7)
    ic = W.fourier_ic(n, seed=n + steps) + 0.1 * W.random_ic(n, 1, seed=steps)
    assert np.array_equal(emulate(hostsim, prob, ic, width, threads), oracle_mod.solve(prob, ic))


KS_CASES = [
    (128, 20, 128, 64),
    (256, 33, 128, 64),       # remainder, odd step count
    (512, 64, 512, 64),       # P = 8, exactly one phase = 128 levels
    (1024, 250, 256, 128),
    (1024, 3, 1024, 64),      # P = 16, fewer levels than a phase
    (2048, 700, 1024, 512),
    (64, 45, 64, 64),         # one point per lane (P = 1 < r = 2), K = 1
    (320, 77, 64, 64),        # N = 64 * 5: only w = 64 divides it
    (1024, 130, 256, 256),    # P = 1 across four waves
]


@pytest.mark.parametrize("n,steps,width,threads", KS_CASES)
@pytest.mark.parametrize("bc", [W.PERIODIC, W.DIRICHLET])
def test_ks_swept_equals_oracle(hostsim, oracle_mod, n, steps, width, threads, bc):
    prob = W.ks_problem(n, steps, bc=bc)
    if bc == W.DIRICHLET:
        prob = W.Problem(W.KS, n, steps, prob.dt, prob.dx, bc=bc, bc_left=(0.4, 0, 0),
                         bc_right=(-0.2, 0, 0))
    ic = W.fourier_ic(n, seed=7 * n + steps)
    assert np.array_equal(emulate(hostsim, prob, ic, width, threads), oracle_mod.solve(prob, ic))


EULER_CASES = [
    (256, 60, 128, 64),
    (512, 130, 256, 64),      # P = 4
    (1024, 300, 512, 64),     # P = 8
    (1024, 201, 256, 128),
    (2048, 10, 512, 128),
    (448, 90, 64, 64),        # P = 1, N = 64 * 7
    (1024, 75, 128, 128),     # P = 1 across two waves
]


@pytest.mark.parametrize("n,steps,width,threads", EULER_CASES)
@pytest.mark.parametrize("limiter", [0, 1])
def test_euler_sod_swept_equals_oracle(hostsim, oracle_mod, n, steps, width, threads, limiter):
    prob = W.sod_problem(n, steps)
    ic = W.sod_ic(n)
    got = emulate(hostsim, prob, ic, width, threads, limiter)
    assert np.array_equal(got, oracle_mod.solve(prob, ic, limiter=limiter))


def test_euler_periodic_smooth_swept_equals_oracle(hostsim, oracle_mod):
    n = 512
    x = (np.arange(n) + 0.5) / n
    rho = 1 + 0.3 * np.sin(2 * np.pi * x)
    u = 0.5 * np.cos(2 * np.pi * x)
    p = 1 + 0.2 * np.sin(4 * np.pi * x)
    ic = np.array([rho, rho * u, p / 0.4 + 0.5 * rho * u * u])
    prob = W.Problem(W.EULER, n, 150, 0.2 / n, 1.0 / n, bc=W.PERIODIC)
    assert np.array_equal(emulate(hostsim, prob, ic, 256, 64), oracle_mod.solve(prob, ic))


def test_phase_sequence_shape(hostsim):
    # heat, w=64: H=32; 10,000 levels = 312 full phases + 16
    prob, _ = W.cfg_heat_small()
    ph = phases(hostsim, prob, 64, 64)
    assert ph[0] == (0, 32, 0)
    assert all(p[0] == 1 and p[1] == 63 for p in ph[1:312])
    assert [p[2] for p in ph[1:5]] == [1, 0, 1, 0]
    assert ph[312] == (2, 32, 0)          # Down after 311 diamonds: 312 shifts, offset 0
    assert ph[313:] == [(0, 16, 0), (2, 16, 1)]
    assert len(ph) == 315
    # KS, w=1024: H=256 levels = 128 steps per phase (Sec. 4.3: two sub-steps per step)
    ph = phases(hostsim, W.ks_problem(1 << 20, 50_000), 1024, 64)
    # 100,000 levels = 390 phases of 256 + 160: Up, 389 Diamonds, Down, Up(160), Down(160)
    assert ph[0] == (0, 256, 0) and len(ph) == 393 and ph[-2:] == [(0, 160, 0), (2, 160, 1)]


HYBRID_CASES = [  # (problem, ic, width, threads): non-periodic, with full phases and remainders
    (W.heat_problem(1024, 777, bc=W.REFLECTIVE), W.fourier_ic(1024, 31), 128, 64),
    (W.heat_problem(2048, 1301, bc=W.DIRICHLET, bc_left=0.25, bc_right=-0.5), W.fourier_ic(2048, 32), 256, 64),
    (W.heat_problem(512, 200, bc=W.REFLECTIVE), W.fourier_ic(512, 33), 512, 64),       # K = 1
    (W.Problem(W.KS, 1024, 333, 2.0 ** -8, 0.5, bc=W.DIRICHLET, bc_left=(0.4, 0, 0), bc_right=(-0.2, 0, 0)),
     W.fourier_ic(1024, 34), 256, 64),
    (W.sod_problem(1024, 450), W.sod_ic(1024), 128, 64),
    (W.sod_problem(2048, 97), W.sod_ic(2048), 512, 64),
]


@pytest.mark.parametrize("case", range(len(HYBRID_CASES)))
def test_hybrid_host_tile_equals_oracle(hostsim, oracle_mod, case):
    """Hybrid variant: with the straddling tile of every shifted phase computed by the
    library's host routine (hybrid_tile_host) and the other tiles by the emulated
    work-group, the result still equals the oracle bit for bit."""
    prob, ic, width, threads = HYBRID_CASES[case]
    out = np.array(ic, dtype=np.float64, copy=True, order="C")
    s = problem_struct(prob)
    rc = hostsim.hostsim_swept_mode(ctypes.byref(s), width, threads,
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1)
    assert rc == 0, rc
    assert np.array_equal(out.reshape(prob.nvars, prob.n), oracle_mod.solve(prob, ic))


DATAFLOW_CASES = [  # several tiles, full phases and remainders, every boundary type, Q = 0 and 1
    (W.heat_problem(1024, 333), W.fourier_ic(1024, 51), 128, 64),
    (W.heat_problem(1024, 40), W.fourier_ic(1024, 52), 128, 64),            # fewer levels than a phase
    (W.heat_problem(512, 100, bc=W.REFLECTIVE), W.fourier_ic(512, 53), 64, 64),
    (W.ks_problem(1024, 301), W.fourier_ic(1024, 54), 128, 64),
    (W.ks_problem(512, 16), W.fourier_ic(512, 55), 64, 64),                  # Q = 1 and a remainder
    (W.Problem(W.KS, 512, 200, 2.0 ** -8, 0.5, bc=W.DIRICHLET, bc_left=(0.4, 0, 0), bc_right=(-0.2, 0, 0)),
     W.fourier_ic(512, 56), 128, 64),
    (W.sod_problem(512, 150), W.sod_ic(512), 64, 64),
    (W.heat_problem(256, 77), W.fourier_ic(256, 57), 256, 64),               # K = 1
]


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("case", range(len(DATAFLOW_CASES)))
def test_dataflow_order_equals_oracle(hostsim, oracle_mod, case, seed):
    """The persistent batched kernel runs a tile as soon as the tiles of the previous
    phase named by phase_deps are done.  Tiles executed in random orders that respect
    only those dependencies (not the phase order) give the oracle's result bit for bit,
    so the dependencies cover every read-after-write and write-after-read between
    phases (edge slots and state)."""
    prob, ic, width, threads = DATAFLOW_CASES[case]
    out = np.array(ic, dtype=np.float64, copy=True, order="C")
    s = problem_struct(prob)
    rc = hostsim.hostsim_dataflow(ctypes.byref(s), width, threads,
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), seed)
    assert rc == 0, rc
    assert np.array_equal(out.reshape(prob.nvars, prob.n), oracle_mod.solve(prob, ic))
