"""Pins for the oracle's Kuramoto-Sivashinsky scheme (Appendix C, Eqs. KSDisc, RKm, RKf).

  * linear limit: a tiny Fourier mode is an eigenvector of the linearised
    periodic scheme; its amplification per step is the RK2 polynomial
    1 + z + z^2/2 of the symbol z = dt (4 s^2/dx^2 - 16 s^4/dx^4), s = sin(pi k/N)
    (pins the second- and fourth-difference coefficients and signs);
  * consistency: for a smooth periodic field, one step with tiny dt reproduces
    -(u u_x + u_xx + u_xxxx) of Eq. KSfull with an error that falls 4x per grid
    doubling (pins the nonlinear term's coefficient and sign as well);
  * invariants: conservation of sum(u), constant states are fixed points,
    bitwise translation equivariance and bitwise mirror antisymmetry.
"""
import math

import numpy as np
import pytest

import workloads as W

EPS = 2.0 ** -53


@pytest.mark.parametrize("k", [1, 3, 5, 9, 17, 31])
def test_ks_linear_limit_mode_amplification(oracle_mod, k):
    n, steps, amp = 64, 400, 1e-8
    dx, dt = 0.5, 2.0 ** -8
    i = np.arange(n)
    ic = amp * np.cos(2 * np.pi * k * i / n)
    got = oracle_mod.solve(W.ks_problem(n, steps, dx=dx, dt=dt), ic.reshape(1, n))[0]
    s = math.sin(math.pi * k / n)
    z = dt * (4 * s * s / dx ** 2 - 16 * s ** 4 / dx ** 4)
    g = 1 + z + z * z / 2
    want = ic * g ** steps
    scale = amp * max(1.0, abs(g) ** steps)
    # the nonlinear term contributes O(amp^2) per unit time: ~1e-8 relative here
    assert np.abs(got - want).max() <= 1e-6 * scale


def _pde_rhs(x, L):
    """-(u u_x + u_xx + u_xxxx) for u = 0.8 sin(q1 x) + 0.6 cos(q2 x)."""
    q1, q2 = 2 * np.pi * 5 / L, 2 * np.pi * 7 / L
    u = 0.8 * np.sin(q1 * x) + 0.6 * np.cos(q2 * x)
    ux = 0.8 * q1 * np.cos(q1 * x) - 0.6 * q2 * np.sin(q2 * x)
    uxx = -0.8 * q1 ** 2 * np.sin(q1 * x) - 0.6 * q2 ** 2 * np.cos(q2 * x)
    uxxxx = 0.8 * q1 ** 4 * np.sin(q1 * x) + 0.6 * q2 ** 4 * np.cos(q2 * x)
    return u, -(u * ux + uxx + uxxxx)


def test_ks_consistency_second_order(oracle_mod):
    L = 2 * np.pi * 8
    dt = 1e-9
    errs = []
    for n in (128, 256, 512):
        dx = L / n
        x = dx * np.arange(n)
        u0, rhs = _pde_rhs(x, L)
        u1 = oracle_mod.solve(W.ks_problem(n, 1, dx=dx, dt=dt), u0.reshape(1, n))[0]
        errs.append(np.abs((u1 - u0) / dt - rhs).max() / np.abs(rhs).max())
    assert errs[-1] < 5e-3
    assert 3.5 < errs[0] / errs[1] < 4.5
    assert 3.5 < errs[1] / errs[2] < 4.5


def test_ks_sum_conserved(oracle_mod):
    n = 512
    ic = W.fourier_ic(n, seed=9)
    got = oracle_mod.solve(W.ks_problem(n, 2000), ic)
    assert abs(got.sum() - ic.sum()) < 1e-10


def test_ks_constant_state_fixed_point(oracle_mod):
    ic = np.full((1, 40), 0.7318)
    assert np.array_equal(oracle_mod.solve(W.ks_problem(40, 50), ic), ic)


@pytest.mark.parametrize("shift", [1, 7, 64, 333])
def test_ks_translation_equivariance_bitwise(oracle_mod, shift):
    n = 512
    ic = W.fourier_ic(n, seed=12) + 0.1 * W.random_ic(n, 1, seed=13)
    prob = W.ks_problem(n, 700)
    a = oracle_mod.solve(prob, ic)
    b = oracle_mod.solve(prob, np.roll(ic, shift, axis=1))
    assert np.array_equal(np.roll(a, shift, axis=1), b)


def test_ks_mirror_antisymmetry_bitwise(oracle_mod):
    """v_i = -u_{-i}  =>  the scheme maps v to the mirror image of its image of u."""
    n = 384
    ic = W.fourier_ic(n, seed=21) + 0.05 * W.random_ic(n, 1, seed=22)
    mirror = lambda a: -np.roll(a[:, ::-1], 1, axis=1)   # index i -> -i mod n
    prob = W.ks_problem(n, 900)
    a = oracle_mod.solve(prob, ic)
    b = oracle_mod.solve(prob, mirror(ic))
    assert np.array_equal(mirror(a), b)


def test_ks_dirichlet_constant_ghosts_fixed_point(oracle_mod):
    """With ghosts equal to the interior constant, Dirichlet KS is also a fixed point."""
    c = -0.375
    prob = W.Problem(W.KS, 50, 30, 2.0 ** -8, 0.5, bc=W.DIRICHLET,
                     bc_left=(c, 0, 0), bc_right=(c, 0, 0))
    ic = np.full((1, 50), c)
    assert np.array_equal(oracle_mod.solve(prob, ic), ic)


def test_ks_time_integration_second_order(oracle_mod):
    """RK2 midpoint (Eqs. RKm, RKf): halving dt cuts the error vs a fine-dt run ~4x."""
    n, T, dx = 64, 0.5, 0.5
    ic = W.fourier_ic(n, seed=31, kmax=6)

    def run(steps):
        return oracle_mod.solve(W.ks_problem(n, steps, dx=dx, dt=T / steps), ic)

    ref = run(2048)
    errs = [np.abs(run(s) - ref).max() for s in (64, 128, 256)]
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.5 < r < 4.5 for r in ratios), ratios
