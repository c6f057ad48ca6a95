"""Exact solution of the Riemann problem for the 1D Euler equations (ideal gas).

Independent of the oracle: a pressure-function Newton iteration for the star
state followed by sampling of the self-similar wave pattern at x/t, following
the standard exact Riemann solver (E. F. Toro, "Riemann Solvers and Numerical
Methods for Fluid Dynamics", ch. 4).  Used to pin the oracle's finite-volume
Euler scheme (Appendix D) on the Sod problem of Eq. SodCond.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np


def _fk(p, rho, pk, ck, g):
    """Pressure function f_K(p) and its derivative for one side."""
    if p > pk:  # shock
        a = 2.0 / ((g + 1.0) * rho)
        b = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(a / (p + b))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (b + p))
    # rarefaction
    pr = p / pk
    f = 2.0 * ck / (g - 1.0) * (pr ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho * ck) * pr ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, g: float = 1.4, tol: float = 1e-15) -> Tuple[float, float]:
    """(p*, u*) for primitive states left=(rho,u,p), right=(rho,u,p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    du = ur - ul
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(200):
        fl, dfl = _fk(p, rl, pl, cl, g)
        fr, dfr = _fk(p, rr, pr, cr, g)
        pn = p - (fl + fr + du) / (dfl + dfr)
        if pn < 0.0:
            pn = tol
        if abs(pn - p) / (0.5 * (pn + p)) < tol:
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, cl, g)
    fr, _ = _fk(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, s: float, g: float = 1.4, star=None):
    """Primitive (rho, u, p) at similarity coordinate s = (x - x0)/t."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = star if star is not None else star_state(left, right, g)
    gm = (g - 1.0) / (g + 1.0)
    if s <= us:
        if ps > pl:  # left shock
            sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
            if s <= sl:
                return rl, ul, pl
            return rl * ((ps / pl + gm) / (gm * ps / pl + 1.0)), us, ps
        shl = ul - cl
        if s <= shl:
            return rl, ul, pl
        csl = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
        stl = us - csl
        if s >= stl:
            return rl * (ps / pl) ** (1.0 / g), us, ps
        u = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * ul + s)
        c = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * (ul - s))
        return rl * (c / cl) ** (2.0 / (g - 1.0)), u, pl * (c / cl) ** (2.0 * g / (g - 1.0))
    if ps > pr:  # right shock
        sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
        if s >= sr:
            return rr, ur, pr
        return rr * ((ps / pr + gm) / (gm * ps / pr + 1.0)), us, ps
    shr = ur + cr
    if s >= shr:
        return rr, ur, pr
    csr = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
    st = us + csr
    if s <= st:
        return rr * (ps / pr) ** (1.0 / g), us, ps
    u = 2.0 / (g + 1.0) * (-cr + (g - 1.0) / 2.0 * ur + s)
    c = 2.0 / (g + 1.0) * (cr - (g - 1.0) / 2.0 * (ur - s))
    return rr * (c / cr) ** (2.0 / (g - 1.0)), u, pr * (c / cr) ** (2.0 * g / (g - 1.0))


def sod_exact(n: int, t: float, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1),
              g: float = 1.4, x0: float = 0.5) -> np.ndarray:
    """Primitive exact solution (3, n) at the cell centres x_i = (i + 1/2)/n."""
    star = star_state(left, right, g)
    out = np.empty((3, n))
    for i in range(n):
        x = (i + 0.5) / n
        out[:, i] = sample(left, right, (x - x0) / t, g, star)
    return out


def max_wave_speed(left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), g: float = 1.4,
                   samples: int = 4001) -> float:
    """Largest |u| + c over the exact self-similar solution."""
    star = star_state(left, right, g)
    best = 0.0
    for s in np.linspace(-3.0, 3.0, samples):
        r, u, p = sample(left, right, float(s), g, star)
        best = max(best, abs(u) + math.sqrt(g * p / r))
    return best
