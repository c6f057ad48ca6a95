"""Exact-arithmetic pins: one level of each printed equation against both oracle forms.

The oracle evaluates every scheme in two rounding orders: the literal form (each
equation of Appendices B-D as printed, after the readings of its typos) and the
canonical form (products fused into the sums that consume them, the KS
right-hand side collected by symmetric stencil pair), which the GPU library
reproduces bit for bit.  Here one level of the printed equations is evaluated
in exact arithmetic -- Python Fractions for heat and KS, 50-digit mpmath for the
Euler flux (square roots) -- from the very same binary64 inputs, and compared
with the oracle's one-level output:

  * on dyadic data whose exact result is representable both forms must match
    the exact value bit for bit;
  * otherwise both must lie within K u S of it, u = 2^-53, with S the same
    expression evaluated on absolute values (the sum of the magnitudes of its
    terms) and K the longest chain of roundings in either form plus the
    rounding of the host constants (derived in the design notes).

A mistake in a coefficient, a sign, an index or the RK stage source changes the
result by a fraction of S itself, many orders of magnitude above K u S, so each
of the oracle's arithmetic paths is tied to the printed equation independently
of the other and of the GPU library.
"""
from fractions import Fraction as Fr

import mpmath
import numpy as np
import pytest

import workloads as W

U = Fr(1, 2 ** 53)


def _periodic(v, i):
    return v[i % len(v)]


# ---------------------------------------------------------------------------
# Heat, Appendix B, Eq. Heatdisc: T' = Fo (T_{i+1} + T_{i-1}) + (1 - 2 Fo) T_i
# ---------------------------------------------------------------------------

def _heat_exact(prob, t):
    fo = Fr((prob.alpha * prob.dt) / (prob.dx * prob.dx))   # the host constant Fo
    c0 = 1 - 2 * fo                                          # exact, not rounded
    n = prob.n
    T = [Fr(float(x)) for x in t]
    val = [fo * (_periodic(T, i + 1) + _periodic(T, i - 1)) + c0 * T[i] for i in range(n)]
    scale = [abs(fo) * (abs(_periodic(T, i + 1)) + abs(_periodic(T, i - 1))) + abs(c0) * abs(T[i])
             for i in range(n)]
    return val, scale


@pytest.mark.parametrize("form", ["literal", "canonical"])
@pytest.mark.parametrize("n", [8, 16])
def test_heat_level_exact_on_dyadic_data(oracle_mod, form, n):
    rng = np.random.default_rng(100 + n)
    t = rng.integers(-64, 65, size=n) / 64.0          # multiples of 2^-6 in [-1, 1]
    prob = W.heat_problem(n, 1, fo=0.25)
    got = oracle_mod.stage(prob, t, form=form)[0]
    want, _ = _heat_exact(prob, t)
    assert all(Fr(float(g)) == w for g, w in zip(got, want))


@pytest.mark.parametrize("form", ["literal", "canonical"])
@pytest.mark.parametrize("fo", [0.25, 0.1, 0.3, 0.5])
def test_heat_level_within_rounding_bound(oracle_mod, form, fo):
    n = 16
    rng = np.random.default_rng(7)
    t = rng.uniform(-1.0, 1.0, size=n)
    prob = W.heat_problem(n, 1, fo=fo)
    got = oracle_mod.stage(prob, t, form=form)[0]
    want, scale = _heat_exact(prob, t)
    K = 5   # sum, two products (literal) or one fused product, final add, and c0's rounding
    for g, w, s in zip(got, want, scale):
        assert abs(Fr(float(g)) - w) <= K * U * s


# ---------------------------------------------------------------------------
# KS, Appendix C, Eq. KSDisc (second difference with -2 u_i) and Eqs. RKm, RKf:
#   f_i(v) = -( (v_{i+1}^2 - v_{i-1}^2)/(4 dx) + (v_{i+1} + v_{i-1} - 2 v_i)/dx^2
#               + (v_{i+2} - 4 v_{i+1} + 6 v_i - 4 v_{i-1} + v_{i-2})/dx^4 )
#   predictor: u + (dt/2) f(u);  final: u + dt f(u^{m+1/2})
# ---------------------------------------------------------------------------

def _ks_exact(prob, src, base, final):
    dx = Fr(prob.dx)
    coef = Fr(prob.dt) if final else Fr(prob.dt) / 2
    n = prob.n
    v = [Fr(float(x)) for x in src]
    b = [Fr(float(x)) for x in base]
    val, scale = [], []
    for i in range(n):
        vm2, vm1, v0, vp1, vp2 = (_periodic(v, i + d) for d in (-2, -1, 0, 1, 2))
        f = -((vp1 * vp1 - vm1 * vm1) / (4 * dx) + (vp1 + vm1 - 2 * v0) / dx ** 2
              + (vp2 - 4 * vp1 + 6 * v0 - 4 * vm1 + vm2) / dx ** 4)
        val.append(b[i] + coef * f)
        # magnitudes of every term; the advection term as (|v+| + |v-|)^2, which covers
        # both the difference of squares and its factored form (v+ - v-)(v+ + v-)
        sf = ((abs(vp1) + abs(vm1)) ** 2 / (4 * dx)
              + (abs(vp1) + abs(vm1) + 2 * abs(v0)) / dx ** 2
              + (abs(vp2) + 4 * abs(vp1) + 6 * abs(v0) + 4 * abs(vm1) + abs(vm2)) / dx ** 4)
        scale.append(abs(b[i]) + coef * sf)
    return val, scale


@pytest.mark.parametrize("form", ["literal", "canonical"])
@pytest.mark.parametrize("n", [8, 16])
def test_ks_predictor_exact_on_dyadic_data(oracle_mod, form, n):
    """dx = 1/2, dt = 2^-8: every constant is a power of two or a small integer, and
    for data on a 2^-6 grid the predictor level is exactly representable."""
    rng = np.random.default_rng(200 + n)
    u = rng.integers(-64, 65, size=n) / 64.0
    prob = W.ks_problem(n, 1)
    got = oracle_mod.stage(prob, u, final=False, form=form)[0]
    want, _ = _ks_exact(prob, u, u, final=False)
    assert all(Fr(float(g)) == w for g, w in zip(got, want))


@pytest.mark.parametrize("form", ["literal", "canonical"])
@pytest.mark.parametrize("n", [8, 16])
@pytest.mark.parametrize("dx,dt", [(0.5, 2.0 ** -8), (0.3, 1e-3), (1.7, 0.05)])
def test_ks_stages_within_rounding_bound(oracle_mod, form, n, dx, dt):
    """Both stages from random data (the final stage from the oracle's own predictor
    output, so a wrong stage source shows), non-dyadic grid spacings included."""
    rng = np.random.default_rng(300 + n)
    u = rng.uniform(-1.5, 1.5, size=n)
    prob = W.ks_problem(n, 1, dx=dx, dt=dt)
    half = oracle_mod.stage(prob, u, final=False, form=form)[0]
    want, scale = _ks_exact(prob, u, u, final=False)
    # longest rounding chain: squares/differences/sums of f (<= 8), stage product and
    # sum (2), plus the host constants 1/(4dx), 1/dx^2, 1/dx^4, dt/2 (<= 4)
    K = 16
    for g, w, s in zip(half, want, scale):
        assert abs(Fr(float(g)) - w) <= K * U * s
    new = oracle_mod.stage(prob, half, base=u, final=True, form=form)[0]
    want, scale = _ks_exact(prob, half, u, final=True)
    for g, w, s in zip(new, want, scale):
        assert abs(Fr(float(g)) - w) <= K * U * s


@pytest.mark.parametrize("form", ["literal", "canonical"])
def test_ks_full_step_matches_two_exact_stages(oracle_mod, form):
    """oracle.solve for one step = predictor then final from the same u^m."""
    n = 16
    rng = np.random.default_rng(11)
    u = rng.uniform(-1.0, 1.0, size=n)
    prob = W.ks_problem(n, 1)
    step = oracle_mod.solve(prob, u.reshape(1, n), form=form)[0]
    half = oracle_mod.stage(prob, u, final=False, form=form)[0]
    new = oracle_mod.stage(prob, half, base=u, final=True, form=form)[0]
    assert np.array_equal(step, new)


# ---------------------------------------------------------------------------
# Euler, Appendix D, in 50-digit arithmetic from the same binary64 cells
# ---------------------------------------------------------------------------

def _mp(x):
    return mpmath.mpf(float(x))


def _mp_pressure(q, gm1):
    rho, m, e = q
    u = m / rho
    return gm1 * (e - rho * u * u / 2)


def _mp_flux(qa, qb, qc, qd, gamma, limiter):
    """Interface flux between cells b and c (Eqs. Pratio, limitleft, limitright,
    EulerF, the Roe average and the spectral radius), exact to 50 digits; the ratio
    tests follow reading R8 (NaN, zero, negative or infinite ratios take the
    first-order branch)."""
    gm1 = _mp(gamma) - 1
    pa, pb, pc, pd = (_mp_pressure(q, gm1) for q in (qa, qb, qc, qd))

    def ratio(num, den):
        if den == 0:
            return None                              # +-inf or NaN: first order
        return num / den

    pr_b, pr_c = ratio(pc - pb, pb - pa), ratio(pd - pc, pc - pb)

    def inv(x):
        return None if x is None or x == 0 else 1 / x

    tl = pr_b if limiter == 0 else inv(pr_b)
    tr = inv(pr_c) if limiter == 0 else pr_c
    okl = tl is not None and tl > 0
    okr = tr is not None and tr > 0
    ql = [qb[v] + min(tl, 1) / 2 * (qc[v] - qb[v]) if okl else qb[v] for v in range(3)]
    qr = [qc[v] + min(tr, 1) / 2 * (qb[v] - qc[v]) if okr else qc[v] for v in range(3)]

    def phys(q):
        u = q[1] / q[0]
        p = _mp_pressure(q, gm1)
        return [q[1], q[0] * u * u + p, u * (q[2] + p)], u

    fl, ul = phys(ql)
    fr, ur = phys(qr)
    sl, sr = mpmath.sqrt(ql[0]), mpmath.sqrt(qr[0])
    rho_sp = mpmath.sqrt(ql[0] * qr[0])
    u_sp = (sl * ul + sr * ur) / (sl + sr)
    e_sp = (sl * ql[2] + sr * qr[2]) / (sl + sr)
    p_sp = gm1 * (e_sp - rho_sp * u_sp * u_sp / 2)
    r_sp = mpmath.sqrt(_mp(gamma) * p_sp / rho_sp) + abs(u_sp)
    flux = [(fr[v] + fl[v] + r_sp * (ql[v] - qr[v])) / 2 for v in range(3)]
    mag = [(abs(fr[v]) + abs(fl[v]) + r_sp * (abs(ql[v]) + abs(qr[v]))) / 2 for v in range(3)]
    return flux, mag


def _euler_exact(prob, src, base, final, limiter):
    mpmath.mp.dps = 50
    n = prob.n
    lam = _mp(prob.dt / prob.dx)                   # the host constant dt/dx
    coef = lam if final else lam / 2

    def cell(q, j):
        if 0 <= j < n:
            return [_mp(q[v][j]) for v in range(3)]
        if prob.bc == W.PERIODIC:
            return [_mp(q[v][j % n]) for v in range(3)]
        side = prob.bc_left if j < 0 else prob.bc_right
        return [_mp(side[v]) for v in range(3)]

    val = np.zeros((3, n), dtype=object)
    scale = np.zeros((3, n), dtype=object)
    for i in range(n):
        c = [cell(src, i + d) for d in (-2, -1, 0, 1, 2)]
        fm, mm = _mp_flux(c[0], c[1], c[2], c[3], prob.gamma, limiter)
        fp, mp_ = _mp_flux(c[1], c[2], c[3], c[4], prob.gamma, limiter)
        for v in range(3):
            b = _mp(base[v][i])
            val[v, i] = b + coef * (fm[v] - fp[v])
            scale[v, i] = abs(b) + coef * (mm[v] + mp_[v])
    return val, scale


def _euler_cases():
    rng = np.random.default_rng(400)
    cases = []
    for n in (8, 16):
        # smooth random positive states, periodic
        rho = rng.uniform(0.5, 1.5, n)
        u = rng.uniform(-0.5, 0.5, n)
        p = rng.uniform(0.5, 1.5, n)
        q = np.stack([rho, rho * u, p / 0.4 + 0.5 * rho * u * u])
        prob = W.Problem(W.EULER, n, 1, dt=0.01, dx=1.0 / n, bc=W.PERIODIC, gamma=1.4)
        cases.append((f"random-periodic-{n}", prob, q))
        # the Sod tube with its Dirichlet ends, and a few steps into the run (uniform
        # regions give 0/0 ratios, the shock gives large ones)
        sod = W.sod_problem(n, 3)
        cases.append((f"sod-ic-{n}", sod, W.sod_ic(n)))
        # cells drawn from three states of distinct pressure: exactly equal neighbours
        # give zero ratios of either sign, infinite ratios and 0/0, so every branch of
        # the ratio tests (reading R8) is taken
        states = np.array([[1.0, 0.2, 2.5], [0.5, -0.1, 1.0], [0.8, 0.0, 1.75]])
        pick = rng.integers(0, 3, size=n)
        prob3 = W.Problem(W.EULER, n, 1, dt=0.01, dx=1.0 / n, bc=W.PERIODIC, gamma=1.4)
        cases.append((f"three-state-{n}", prob3, states[pick].T.copy()))
    return cases


@pytest.mark.parametrize("form", ["literal", "canonical"])
@pytest.mark.parametrize("limiter", [0, 1])
@pytest.mark.parametrize("case", range(6), ids=[c[0] for c in _euler_cases()])
def test_euler_stages_within_rounding_bound(oracle_mod, form, limiter, case):
    name, prob, q0 = _euler_cases()[case]
    q = q0
    if name.startswith("sod"):
        q = oracle_mod.solve(prob, q0, limiter=limiter, form=form)   # 3 steps into the run
    # flux chains reach about 30 roundings (pressures, ratio, limiter, Roe average,
    # square roots, divisions); K = 64 keeps a factor two of margin
    K = 64
    half = oracle_mod.stage(prob, q, final=False, limiter=limiter, form=form)
    want, scale = _euler_exact(prob, q, q, final=False, limiter=limiter)
    tol = float(K * U)
    for v in range(3):
        for i in range(prob.n):
            assert abs(mpmath.mpf(float(half[v, i])) - want[v, i]) <= tol * scale[v, i], (v, i)
    new = oracle_mod.stage(prob, half, base=q, final=True, limiter=limiter, form=form)
    want, scale = _euler_exact(prob, half, q, final=True, limiter=limiter)
    for v in range(3):
        for i in range(prob.n):
            assert abs(mpmath.mpf(float(new[v, i])) - want[v, i]) <= tol * scale[v, i], (v, i)


# ---------------------------------------------------------------------------
# The two forms over whole runs: same arithmetic, different rounding
# ---------------------------------------------------------------------------

def test_heat_forms_agree_over_cfg1(oracle_mod):
    """Fo <= 1/2: each update is a convex combination, so rounding differences do not
    grow; 10,000 steps keep the two forms within (3 + 3m) u ||u0||."""
    prob, ic = W.cfg_heat_small()
    a = oracle_mod.solve(prob, ic, form="canonical")
    b = oracle_mod.solve(prob, ic, form="literal")
    assert np.abs(a - b).max() <= (3 + 3 * prob.nsteps) * 2.0 ** -53 * np.abs(ic).max()


def test_ks_forms_agree_before_chaos(oracle_mod):
    """KS before the chaotic growth sets in (500 steps = 2 time units): the forms
    differ only by rounding, far below the 1e-12 bar."""
    prob, ic = W.cfg_sweep(W.KS, 12, nsteps=500)
    a = oracle_mod.solve(prob, ic, form="canonical")
    b = oracle_mod.solve(prob, ic, form="literal")
    assert np.abs(a - b).max() / np.abs(b).max() <= 1e-13


def test_sod_forms_agree(oracle_mod):
    """Sod at N = 256.  For the first 50 steps the forms agree to 1e-13 relative per
    variable.  Later they part at the contact discontinuity: pressure is continuous
    there while density jumps, so the pressure ratio of Eq. Pratio is a quotient of two
    rounding-level differences, and the slope it selects for the density jump depends
    on the rounding order.  Over the whole run to t = 0.2 the forms then differ by a
    few 1e-10 (bounded here by 1e-8); this is a property of the limiter, which is
    why the GPU's parity with the oracle is taken against the canonical form, bit
    for bit, and the literal form is tied to the equations one level at a time."""
    prob, ic = W.cfg_sod(8)
    early = prob.with_steps(50)
    a = oracle_mod.solve(early, ic, form="canonical")
    b = oracle_mod.solve(early, ic, form="literal")
    for v in range(3):
        assert np.abs(a[v] - b[v]).max() / np.abs(b[v]).max() <= 1e-13
    a = oracle_mod.solve(prob, ic, form="canonical")
    b = oracle_mod.solve(prob, ic, form="literal")
    for v in range(3):
        assert np.abs(a[v] - b[v]).max() / np.abs(b[v]).max() <= 1e-8
