"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only *draws* inputs: problem descriptions (scheme, grid size, step
size, boundary type) and initial conditions.  It contains none of the
time-stepping arithmetic of the method; both the CPU oracle and the GPU library
receive the very same arrays built here, so transcendental-function differences
between libraries can never leak into a parity comparison.

The paper uses no dataset: every workload is a synthetic initial-value problem
(heat equation, Kuramoto-Sivashinsky equation, Sod shock tube; Sec. 5.2 and
Appendices B-D).  The concrete recipes below (mode counts, seeds, step sizes)
are this project's stand-ins for the paper's workloads.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np

# Scheme and boundary identifiers (same numeric values as the C interfaces).
HEAT, KS, EULER = 0, 1, 2
PERIODIC, DIRICHLET, REFLECTIVE = 0, 1, 2
SCHEME_NAMES = {HEAT: "heat", KS: "ks", EULER: "euler"}
NVARS = {HEAT: 1, KS: 1, EULER: 3}

# Sod shock tube end states (Appendix D, Eq. SodCond) as primitive (rho, u, P).
SOD_LEFT_PRIM = (1.0, 0.0, 1.0)
SOD_RIGHT_PRIM = (0.125, 0.0, 0.1)
# The same end states as conserved (rho, rho*u, E): E = P/(gamma-1) + rho*u^2/2,
# which for u = 0 and gamma = 1.4 is exactly 2.5 and 0.25.
SOD_LEFT_CONS = (1.0, 0.0, 2.5)
SOD_RIGHT_CONS = (0.125, 0.0, 0.25)
SOD_GAMMA = 1.4
SOD_T_END = 0.2
SOD_CFL = 0.4
SOD_SMAX = 2.2  # bound above the largest |u|+c of the exact Sod solution (~2.19)


@dataclass(frozen=True)
class Problem:
    """One initial-value problem: the fields of the paper's problem statement."""
    scheme: int
    n: int
    nsteps: int
    dt: float
    dx: float
    bc: int = PERIODIC
    alpha: float = 1.0
    gamma: float = SOD_GAMMA
    bc_left: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    bc_right: Tuple[float, float, float] = (0.0, 0.0, 0.0)

    @property
    def nvars(self) -> int:
        return NVARS[self.scheme]

    @property
    def point_updates(self) -> int:
        return self.n * self.nsteps

    def with_steps(self, nsteps: int) -> "Problem":
        return replace(self, nsteps=int(nsteps))


# ---------------------------------------------------------------------------
# Problem constructors
# ---------------------------------------------------------------------------

def heat_problem(n: int, nsteps: int, bc: int = PERIODIC, fo: float = 0.25,
                 bc_left: float = 0.0, bc_right: float = 0.0) -> Problem:
    """Heat equation with alpha = 1, dx = 1, dt = Fo (so Fo = alpha*dt/dx^2 exactly)."""
    return Problem(HEAT, int(n), int(nsteps), dt=float(fo), dx=1.0, bc=bc, alpha=1.0,
                   bc_left=(bc_left, 0.0, 0.0), bc_right=(bc_right, 0.0, 0.0))


def ks_problem(n: int, nsteps: int, dx: float = 0.5, dt: float = 2.0 ** -8,
               bc: int = PERIODIC) -> Problem:
    """Kuramoto-Sivashinsky equation; dx = 0.5, dt = 2^-8 make every constant dyadic."""
    return Problem(KS, int(n), int(nsteps), dt=float(dt), dx=float(dx), bc=bc)


def sod_steps(n: int) -> Tuple[float, float, int]:
    """(dx, dt, nsteps) for the Sod tube on [0, 1] with n cells run to t = 0.2.

    A fixed step is needed because the swept decomposition cannot perform a
    global max-reduction inside a phase: dt = CFL*dx/S_max with S_max = 2.2,
    then rounded so that nsteps*dt = 0.2.
    """
    dx = 1.0 / n
    dt0 = SOD_CFL * dx / SOD_SMAX
    nsteps = int(math.ceil(SOD_T_END / dt0))
    return dx, SOD_T_END / nsteps, nsteps


def sod_problem(n: int, nsteps: Optional[int] = None) -> Problem:
    dx, dt, full = sod_steps(n)
    return Problem(EULER, int(n), int(full if nsteps is None else nsteps), dt=dt, dx=dx,
                   bc=DIRICHLET, gamma=SOD_GAMMA, bc_left=SOD_LEFT_CONS,
                   bc_right=SOD_RIGHT_CONS)


# ---------------------------------------------------------------------------
# Initial conditions (all float64, shape (nvars, n), C-contiguous)
# ---------------------------------------------------------------------------

def sine_modes_ic(n: int, seed: int = 1, modes: int = 8) -> np.ndarray:
    """u_i = sum_{k=1..modes} a_k sin(2 pi k i / n), a_k ~ U(-1, 1)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=modes)
    i = np.arange(n, dtype=np.float64)
    u = np.zeros(n)
    for k in range(1, modes + 1):
        u += a[k - 1] * np.sin(2.0 * np.pi * k * i / n)
    return u.reshape(1, n).copy()


def fourier_ic(n: int, seed: int, kmax: int = 16) -> np.ndarray:
    """Smooth periodic field: sum_{k=1..kmax} a_k cos(2 pi k i/n) + b_k sin(2 pi k i/n)."""
    rng = np.random.default_rng(seed)
    kmax = max(1, min(kmax, n // 8)) if n >= 8 else 1
    a = rng.uniform(-1.0, 1.0, size=kmax)
    b = rng.uniform(-1.0, 1.0, size=kmax)
    i = np.arange(n, dtype=np.float64)
    u = np.zeros(n)
    for k in range(1, kmax + 1):
        th = 2.0 * np.pi * k * i / n
        u += a[k - 1] * np.cos(th) + b[k - 1] * np.sin(th)
    return u.reshape(1, n).copy()


def sod_ic(n: int) -> np.ndarray:
    """Conserved Sod state, left state for cell centres x_i = (i + 1/2)/n < 1/2."""
    q = np.empty((3, n))
    half = n // 2  # (i + 1/2)/n < 1/2 holds exactly for i < n // 2
    for v in range(3):
        q[v, :half] = SOD_LEFT_CONS[v]
        q[v, half:] = SOD_RIGHT_CONS[v]
    return q


def random_ic(n: int, nvars: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(nvars, n))


def ic_for(problem: Problem, seed: int) -> np.ndarray:
    """Default initial condition for a problem: smooth modes, or Sod for Euler."""
    if problem.scheme == EULER:
        return sod_ic(problem.n)
    return fourier_ic(problem.n, seed)


# ---------------------------------------------------------------------------
# Named configurations of the benchmark suite
# ---------------------------------------------------------------------------

def cfg_heat_small() -> Tuple[Problem, np.ndarray]:
    """Heat FTCS, N = 1024 periodic, Fo = 0.25, 10,000 steps, 8 seeded sine modes."""
    return heat_problem(1024, 10_000), sine_modes_ic(1024, seed=1, modes=8)


def cfg_sweep(scheme: int, log2n: int, nsteps: int = 50_000) -> Tuple[Problem, np.ndarray]:
    """Heat or KS at N = 2^log2n, periodic, 50,000 steps, Fourier modes k <= 16."""
    n = 1 << log2n
    ic = fourier_ic(n, seed=2 + log2n, kmax=16)
    if scheme == HEAT:
        return heat_problem(n, nsteps), ic
    if scheme == KS:
        return ks_problem(n, nsteps), ic
    raise ValueError("sweep configs cover heat and KS only")


def cfg_sod(log2n: int, nsteps: Optional[int] = None) -> Tuple[Problem, np.ndarray]:
    n = 1 << log2n
    return sod_problem(n, nsteps), sod_ic(n)


@dataclass
class EnsembleMember:
    problem: Problem
    ic_seed: int


def round64(x: float) -> int:
    return max(64, int(64 * round(x / 64.0)))


def ensemble(count: int = 4096, seed: int = 4, nsteps: int = 10_000,
             nmin: int = 256, nmax: int = 65536) -> List[EnsembleMember]:
    """Independent heat/KS solves with N log-uniform in [nmin, nmax], multiples of 64."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        n = round64(math.exp(rng.uniform(math.log(nmin), math.log(nmax))))
        scheme = HEAT if rng.uniform() < 0.5 else KS
        prob = heat_problem(n, nsteps) if scheme == HEAT else ks_problem(n, nsteps)
        out.append(EnsembleMember(prob, ic_seed=int(seed * 1_000_003 + j)))
    return out


def ensemble_ic(member: EnsembleMember) -> np.ndarray:
    n = member.problem.n
    return fourier_ic(n, member.ic_seed, kmax=min(16, n // 8))


@dataclass
class Request:
    arrival_s: float
    problem: Problem
    ic_seed: int


def poisson_trace(rate: float = 2000.0, duration_s: float = 10.0, seed: int = 5,
                  nmin: int = 512, nmax: int = 1 << 18, smin: int = 1000,
                  smax: int = 20000, schemes=(HEAT, KS, EULER)) -> List[Request]:
    """Poisson arrivals of mixed heat/KS/Sod solves (the serving workload)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    j = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration_s:
            break
        scheme = schemes[int(rng.integers(0, len(schemes)))]
        n = round64(math.exp(rng.uniform(math.log(nmin), math.log(nmax))))
        steps = int(rng.integers(smin, smax + 1))
        if scheme == HEAT:
            prob = heat_problem(n, steps)
        elif scheme == KS:
            prob = ks_problem(n, steps)
        else:
            prob = sod_problem(n, steps)
        out.append(Request(t, prob, ic_seed=int(seed * 1_000_003 + j)))
        j += 1
    return out


def request_ic(req: Request) -> np.ndarray:
    p = req.problem
    if p.scheme == EULER:
        return sod_ic(p.n)
    return fourier_ic(p.n, req.ic_seed, kmax=min(16, p.n // 8))
