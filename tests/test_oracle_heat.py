"""Pins for the oracle's heat-equation scheme (Appendix B, Eq. Heatdisc).

Each test checks the oracle against something fixed by the mathematics rather
than against a retyped copy of its own update:
  * discrete Fourier-mode closed form (periodic and homogeneous Dirichlet),
  * maximum principle and conservation of the sum (periodic),
  * exact dyadic arithmetic on small-integer data (brute force with Fractions).
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import workloads as W

EPS = 2.0 ** -53


def _closed_form_periodic(n, m, amps, fo):
    """u_i^m = sum_k a_k sin(2 pi k i/n) g_k^m with g_k = 1 - 4 Fo sin^2(pi k/n)."""
    mpmath.mp.dps = 40
    out = np.zeros(n)
    for k, a in enumerate(amps, start=1):
        g = 1 - 4 * mpmath.mpf(fo) * mpmath.sin(mpmath.pi * k / n) ** 2
        gm = g ** m
        for i in range(n):
            out[i] += float(mpmath.mpf(a) * mpmath.sin(2 * mpmath.pi * k * i / n) * gm)
    return out


def test_heat_periodic_closed_form_cfg1(oracle_mod):
    """N=1024, Fo=1/4, 10,000 steps: each sine mode decays by cos^2(pi k/N) per step."""
    prob, ic = W.cfg_heat_small()
    rng = np.random.default_rng(1)
    amps = rng.uniform(-1.0, 1.0, size=8)
    got = oracle_mod.solve(prob, ic)[0]
    want = _closed_form_periodic(prob.n, prob.nsteps, amps, 0.25)
    # Fo <= 1/2 makes every update a convex combination, so rounding errors do not
    # grow: at most ~1.5 ulp of ||u0|| per step plus the initial-condition rounding.
    bound = (8 + 1.5 * prob.nsteps) * EPS * np.abs(ic).max()
    assert np.abs(got - want).max() <= bound


@pytest.mark.parametrize("fo", [0.25, 0.1, 0.5])
def test_heat_dirichlet_zero_closed_form(oracle_mod, fo):
    """Zero Dirichlet ghosts: modes sin(pi k (i+1)/(N+1)) decay by 1 - 4 Fo sin^2(pi k/(2(N+1)))."""
    n, m = 96, 300
    mpmath.mp.dps = 40
    ks = [1, 3, 7]
    amps = [0.7, -0.4, 0.25]
    ic = np.zeros(n)
    want = np.zeros(n)
    for k, a in zip(ks, amps):
        g = 1 - 4 * mpmath.mpf(fo) * mpmath.sin(mpmath.pi * k / (2 * (n + 1))) ** 2
        for i in range(n):
            s = mpmath.sin(mpmath.pi * k * (i + 1) / (n + 1))
            ic[i] += float(a * s)
            want[i] += float(a * s * g ** m)
    prob = W.heat_problem(n, m, bc=W.DIRICHLET, fo=fo)
    got = oracle_mod.solve(prob, ic.reshape(1, n))[0]
    assert np.abs(got - want).max() <= (8 + 1.5 * m) * EPS * np.abs(ic).max() * 4


@pytest.mark.parametrize("fo", [0.25, 0.4])
def test_heat_reflective_closed_form(oracle_mod, fo):
    """Insulated ends (Eq. heatcond, mirror ghosts T_{-1} = T_1, T_N = T_{N-2}): modes
    cos(pi k i/(N-1)) are eigenvectors with factor 1 - 4 Fo sin^2(pi k/(2(N-1)))."""
    n, m = 80, 400
    mpmath.mp.dps = 40
    ks, amps = [0, 1, 4, 9], [0.3, 0.7, -0.4, 0.25]
    ic = np.zeros(n)
    want = np.zeros(n)
    for k, a in zip(ks, amps):
        g = 1 - 4 * mpmath.mpf(fo) * mpmath.sin(mpmath.pi * k / (2 * (n - 1))) ** 2
        for i in range(n):
            c = mpmath.cos(mpmath.pi * k * i / (n - 1))
            ic[i] += float(a * c)
            want[i] += float(a * c * g ** m)
    prob = W.heat_problem(n, m, bc=W.REFLECTIVE, fo=fo)
    got = oracle_mod.solve(prob, ic.reshape(1, n))[0]
    assert np.abs(got - want).max() <= (8 + 1.5 * m) * EPS * np.abs(ic).max() * 4


def test_heat_reflective_conserves_trapezoid_sum(oracle_mod):
    """With mirror ghosts the trapezoid-weighted sum (end points weighted 1/2) is
    conserved: the flux through each insulated end vanishes."""
    n = 123
    ic = W.random_ic(n, 1, seed=31)[0]
    got = oracle_mod.solve(W.heat_problem(n, 300, bc=W.REFLECTIVE), ic.reshape(1, n))[0]
    trap = lambda u: u[1:-1].sum() + 0.5 * (u[0] + u[-1])
    assert abs(trap(got) - trap(ic)) < 1e-12 * n


def test_heat_max_principle_and_conservation(oracle_mod):
    n = 777
    ic = W.random_ic(n, 1, seed=11)
    prob = W.heat_problem(n, 500)
    got = oracle_mod.solve(prob, ic)
    assert np.abs(got).max() <= np.abs(ic).max()
    # sum is conserved up to rounding (telescoping differences, periodic)
    assert abs(got.sum() - ic.sum()) <= 500 * n * EPS * 4 * np.abs(ic).max()


def test_heat_exact_dyadic_bruteforce(oracle_mod):
    """Small integers with Fo = 1/4 stay exactly representable: compare with Fractions."""
    n, steps = 16, 18
    rng = np.random.default_rng(5)
    ic = rng.integers(-500, 500, size=n).astype(np.float64)
    u = [Fraction(int(x)) for x in ic]
    q = Fraction(1, 4)
    for _ in range(steps):
        u = [q * (u[(i + 1) % n] + u[(i - 1) % n]) + (1 - 2 * q) * u[i] for i in range(n)]
    got = oracle_mod.solve(W.heat_problem(n, steps), ic.reshape(1, n))[0]
    assert [Fraction(float(x)) for x in got] == u


def test_heat_thread_count_invariance(oracle_mod):
    prob, ic = W.cfg_heat_small()
    prob = prob.with_steps(300)
    a = oracle_mod.solve(prob, ic, nthreads=1)
    b = oracle_mod.solve(prob, ic, nthreads=0)
    assert np.array_equal(a, b)


def test_zero_steps_is_identity(oracle_mod):
    ic = W.random_ic(50, 1, seed=2)
    assert np.array_equal(oracle_mod.solve(W.heat_problem(50, 0), ic), ic)


def test_invalid_problem_rejected(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.solve(W.Problem(W.HEAT, 0, 1, 0.25, 1.0), np.zeros((1, 1)))
