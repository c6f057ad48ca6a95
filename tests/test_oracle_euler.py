"""Pins for the oracle's finite-volume Euler scheme (Appendix D).

  * Sod tube: the density converges to the exact Riemann solution (independent
    solver in exact_riemann.py) as the grid is refined, with positive density and
    pressure throughout;
  * conservation: sum(rho) and sum(E) are constant while the waves stay inside
    the tube; sum(rho u) grows by (dt/dx)(P_L - P_R) per step (pressure force);
  * smooth periodic flow: one step with tiny dt reproduces -dF/dx of Eq.
    EulerGeneral with an error that shrinks under refinement;
  * uniform states are exact fixed points; mirror symmetry x -> 1-x, u -> -u;
  * hand-worked interface fluxes: the limiter orientation as printed in Eqs.
    limitleft/limitright, and the Roe-averaged spectral radius on contacts.
"""
import math

import numpy as np
import pytest

import exact_riemann as ER
import workloads as W

G = 1.4
GM1 = 1.4 - 1.0


def _prim(q):
    rho, m, E = q
    u = m / rho
    return rho, u, GM1 * (E - 0.5 * m * u)


def test_sod_max_wave_speed_below_fixed_dt_bound():
    """The fixed step dt = 0.4 dx / 2.2 is a true CFL-0.4 step: max |u|+c < 2.2."""
    smax = ER.max_wave_speed()
    assert 2.18 < smax < W.SOD_SMAX


def test_sod_star_state_textbook_values():
    """Commonly tabulated star state for Sod's problem: p* = 0.30313, u* = 0.92745."""
    p, u = ER.star_state(W.SOD_LEFT_PRIM, W.SOD_RIGHT_PRIM)
    assert abs(p - 0.30313) < 1e-5 and abs(u - 0.92745) < 1e-5


@pytest.mark.parametrize("limiter", [0, 1])
def test_sod_converges_to_exact_riemann(oracle_mod, limiter):
    errs = []
    for l in range(7, 12):
        prob, ic = W.cfg_sod(l)
        q = oracle_mod.solve(prob, ic, limiter=limiter)
        rho, u, p = _prim(q)
        assert rho.min() > 0 and p.min() > 0
        ex = ER.sod_exact(prob.n, W.SOD_T_END)
        errs.append(np.abs(rho - ex[0]).mean())
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(r > 1.3 for r in ratios), ratios
    assert errs[-1] < 2e-3


def test_sod_conservation_and_momentum_growth(oracle_mod):
    prob, ic = W.cfg_sod(9)
    steps = 250
    lam = prob.dt / prob.dx
    q = ic
    prev = q.sum(axis=1)
    p_left = GM1 * W.SOD_LEFT_CONS[2]
    p_right = GM1 * W.SOD_RIGHT_CONS[2]
    for _ in range(5):
        q = oracle_mod.solve(prob.with_steps(steps // 5), q)
        cur = q.sum(axis=1)
        assert abs(cur[0] - prev[0]) < 1e-12 * prob.n
        assert abs(cur[2] - prev[2]) < 1e-12 * prob.n
        growth = (cur[1] - prev[1]) / (steps // 5)
        assert abs(growth - lam * (p_left - p_right)) < 1e-12 * prob.n
        prev = cur


@pytest.mark.parametrize("bc", [W.PERIODIC, W.DIRICHLET])
def test_uniform_state_fixed_point(oracle_mod, bc):
    state = (0.8, -0.24, 3.1)
    ic = np.array([[v] * 64 for v in state])
    prob = W.Problem(W.EULER, 64, 40, 1e-3, 1.0 / 64, bc=bc, bc_left=state, bc_right=state)
    assert np.array_equal(oracle_mod.solve(prob, ic), ic)


def _smooth_state(x):
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x)
    u = 0.3 + 0.1 * np.cos(2 * np.pi * x)
    p = 1.0 + 0.1 * np.sin(4 * np.pi * x)
    return rho, u, p


def _smooth_dqdt(x):
    """-dF/dx for the smooth state, from the analytic derivatives of rho, u, p."""
    rho, u, p = _smooth_state(x)
    rx = 0.2 * 2 * np.pi * np.cos(2 * np.pi * x)
    ux = -0.1 * 2 * np.pi * np.sin(2 * np.pi * x)
    px = 0.1 * 4 * np.pi * np.cos(4 * np.pi * x)
    E = p / GM1 + 0.5 * rho * u * u
    Ex = px / GM1 + 0.5 * rx * u * u + rho * u * ux
    f0x = rx * u + rho * ux
    f1x = rx * u * u + 2 * rho * u * ux + px
    f2x = ux * (E + p) + u * (Ex + px)
    return -np.array([f0x, f1x, f2x])


def test_smooth_flow_consistency(oracle_mod):
    dt = 1e-9
    errs = []
    for n in (64, 128, 256, 512):
        dx = 1.0 / n
        x = (np.arange(n) + 0.5) * dx
        rho, u, p = _smooth_state(x)
        q0 = np.array([rho, rho * u, p / GM1 + 0.5 * rho * u * u])
        prob = W.Problem(W.EULER, n, 1, dt, dx, bc=W.PERIODIC)
        q1 = oracle_mod.solve(prob, q0)
        want = _smooth_dqdt(x)
        errs.append(np.abs((q1 - q0) / dt - want).mean() / np.abs(want).mean())
    assert errs[-1] < 1e-2
    assert all(errs[i] / errs[i + 1] > 1.6 for i in range(len(errs) - 1)), errs


def test_mirror_symmetry(oracle_mod):
    prob, ic = W.cfg_sod(8)
    prob = prob.with_steps(200)
    a = oracle_mod.solve(prob, ic)
    mir = lambda q: np.array([q[0, ::-1], -q[1, ::-1], q[2, ::-1]])
    # mirrored problem: right state on the left, left state on the right
    pm = W.Problem(W.EULER, prob.n, prob.nsteps, prob.dt, prob.dx, bc=W.DIRICHLET,
                   bc_left=W.SOD_RIGHT_CONS, bc_right=W.SOD_LEFT_CONS)
    b = oracle_mod.solve(pm, mir(ic))
    assert np.abs(mir(a) - b).max() < 1e-12


def test_limiter_orientation_as_printed(oracle_mod):
    """Cells at rest with pressures 1, 2, 4, 5: Pr_b = 2 and 1/Pr_c = 2, so both printed
    limiters take the full half-jump, Q^L = Q^R = (Q_b + Q_c)/2, and the energy flux
    vanishes.  The reciprocal orientation gives Q^L_E = 6.25, Q^R_E = 8.75 instead."""
    cells = [[1.0, 0.0, p / 0.4] for p in (1.0, 2.0, 4.0, 5.0)]
    f = oracle_mod.euler_flux(cells, G, limiter=0)
    assert f[0] == 0.0 and f[2] == 0.0
    assert abs(f[1] - GM1 * 7.5) < 1e-15 * 3
    f1 = oracle_mod.euler_flux(cells, G, limiter=1)
    rs = math.sqrt(G * (GM1 * 7.5))
    assert abs(f1[1] - 0.5 * (GM1 * 6.25 + GM1 * 8.75)) < 1e-14
    assert abs(f1[2] - 0.5 * rs * (6.25 - 8.75)) < 1e-14


def test_roe_spectral_radius_stationary_contact(oracle_mod):
    """Density jump 4 | 1 at rest in uniform pressure: no limiting (Pr = 0/0), the Roe
    state is rho_s = sqrt(4*1) = 2 with e_s = E, so r_sp = sqrt(gamma P / 2) and the
    mass flux is r_sp (rho_L - rho_R)/2."""
    E = 1.0 / GM1
    L, R = [4.0, 0.0, E], [1.0, 0.0, E]
    f = oracle_mod.euler_flux([L, L, R, R], G)
    p = GM1 * E
    rs = math.sqrt(G * p / 2.0)
    assert abs(f[0] - 0.5 * rs * 3.0) < 1e-15
    assert abs(f[1] - p) < 1e-15
    assert f[2] == 0.0


def test_roe_spectral_radius_moving_contact(oracle_mod):
    """Same contact advected at u = 1/2: Roe velocity 1/2, Roe energy (2*3 + 1*2.625)/3."""
    rl, rr, u, p = 4.0, 1.0, 0.5, 1.0
    L = [rl, rl * u, p / GM1 + 0.5 * rl * u * u]
    R = [rr, rr * u, p / GM1 + 0.5 * rr * u * u]
    f = oracle_mod.euler_flux([L, L, R, R], G)
    es = (2.0 * L[2] + 1.0 * R[2]) / 3.0
    ps = GM1 * (es - 0.5 * (2.0 * u) * u)
    rs = math.sqrt(G * ps / 2.0) + u
    fl = np.array([rl * u, rl * u * u + p, u * (L[2] + p)])
    fr = np.array([rr * u, rr * u * u + p, u * (R[2] + p)])
    want = 0.5 * (fl + fr + rs * (np.array(L) - np.array(R)))
    assert np.abs(f - want).max() < 1e-14


def test_euler_thread_count_invariance(oracle_mod):
    prob, ic = W.cfg_sod(10)
    prob = prob.with_steps(300)
    assert np.array_equal(oracle_mod.solve(prob, ic, nthreads=1),
                          oracle_mod.solve(prob, ic, nthreads=0))


def test_time_integration_second_order(oracle_mod):
    """The RK2 midpoint scheme (Eqs. RKm/RKf reused for Euler) is second order in time.
    A contact at rest (u = 0, uniform E, hence uniform P) keeps m = 0 and E uniform
    exactly, so the limiter stays in one branch and only rho evolves, under a smooth
    ODE: on a fixed grid, halving dt cuts the distance to a fine-dt solution ~4x."""
    n, T = 64, 0.05
    dx = 1.0 / n
    x = (np.arange(n) + 0.5) * dx
    q0 = np.array([1.0 + 0.5 * np.sin(2 * np.pi * x), 0.0 * x, 2.5 + 0.0 * x])

    def run(steps):
        return oracle_mod.solve(W.Problem(W.EULER, n, steps, T / steps, dx, bc=W.PERIODIC), q0)

    ref = run(1280)
    errs = [np.abs(run(s) - ref).max() for s in (10, 20, 40)]
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.7 < r < 4.3 for r in ratios), ratios
    out = run(40)
    assert np.array_equal(out[1], q0[1]) and np.array_equal(out[2], q0[2])
