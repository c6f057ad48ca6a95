"""GPU parity: the HIP swept and classic solvers against the CPU oracle.

Bar (stated per test): max over variables of ||x - y||_inf / ||y||_inf <= 1e-12
against the oracle, and swept == classic bit for bit on the GPU.  All solves go
through the C interface (libswept.so) via the ctypes binding.
"""
import ctypes
import dataclasses

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
import paper_1705_03162_amd as sw  # noqa: E402
from paper_1705_03162_amd import _native as N  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-12


def relerr(got, want):
    got = np.atleast_2d(got)
    want = np.atleast_2d(want)
    worst = 0.0
    for g, w in zip(got, want):
        scale = np.abs(w).max()
        worst = max(worst, np.abs(g - w).max() / (scale if scale > 0 else 1.0))
    return worst


def gpu_solve(prob, ic, kind="swept", width=0, threads=0, flags=0, limiter=0):
    print(f"[gpu] {kind} scheme={prob.scheme} bc={prob.bc} n={prob.n} steps={prob.nsteps} "
          f"w={width} T={threads} flags={flags}", flush=True)
    with sw.Plan(prob, width, threads, flags, limiter) as plan:
        x = torch.tensor(ic, dtype=torch.float64, device=DEV)
        getattr(plan, kind)(x)
        torch.cuda.synchronize()
    return x.cpu().numpy()


# ---------------------------------------------------------------- small cases

SMALL = [  # (problem factory, width, threads)
    (lambda: (W.heat_problem(1024, 333), W.fourier_ic(1024, 1)), 64, 64),
    (lambda: (W.heat_problem(1024, 777, bc=W.DIRICHLET, bc_left=0.3, bc_right=-0.7),
              W.fourier_ic(1024, 2)), 256, 128),
    (lambda: (W.heat_problem(4096, 1500), W.fourier_ic(4096, 3)), 1024, 256),
    (lambda: (W.heat_problem(2048, 600), W.fourier_ic(2048, 4)), 2048, 128),   # K = 1, P = 16
    (lambda: (W.ks_problem(1024, 400), W.fourier_ic(1024, 5)), 128, 64),
    (lambda: (W.ks_problem(4096, 333), W.fourier_ic(4096, 6)), 512, 64),
    (lambda: (W.ks_problem(4096, 1000), W.fourier_ic(4096, 7)), 1024, 128),
    (lambda: (W.Problem(W.KS, 2048, 257, 2.0 ** -8, 0.5, bc=W.DIRICHLET, bc_left=(0.4, 0, 0),
                        bc_right=(-0.2, 0, 0)), W.fourier_ic(2048, 8)), 2048, 256),
    (lambda: (W.sod_problem(1024, 500), W.sod_ic(1024)), 256, 64),
    (lambda: (W.sod_problem(2048, 901), W.sod_ic(2048)), 512, 128),
    (lambda: (W.sod_problem(4096, 64), W.sod_ic(4096)), 512, 64),
    # one point per lane (P = 1 < r = 2): halos pass through two lanes
    (lambda: (W.ks_problem(320, 301), W.fourier_ic(320, 11)), 64, 64),
    (lambda: (W.ks_problem(1024, 257), W.fourier_ic(1024, 12)), 256, 256),
    (lambda: (W.sod_problem(448, 350), W.sod_ic(448)), 64, 64),
    (lambda: (W.sod_problem(1024, 200), W.sod_ic(1024)), 128, 128),
    # insulated (reflective) heat ends: wall tile at the centre of shifted phases
    (lambda: (W.heat_problem(1024, 501, bc=W.REFLECTIVE), W.fourier_ic(1024, 13)), 64, 64),
    (lambda: (W.heat_problem(4096, 1999, bc=W.REFLECTIVE), W.fourier_ic(4096, 14)), 1024, 256),
    (lambda: (W.heat_problem(2048, 700, bc=W.REFLECTIVE), W.fourier_ic(2048, 15)), 2048, 128),
    (lambda: (W.heat_problem(512, 333, bc=W.REFLECTIVE), W.fourier_ic(512, 16)), 128, 128),
    # one-wave tiles of 16 points per lane (rows staged through LDS on load and store), with
    # a remainder (Up that stops below its tip), Dirichlet and insulated walls
    (lambda: (W.heat_problem(4096, 1777), W.fourier_ic(4096, 17)), 1024, 64),
    (lambda: (W.heat_problem(3072, 1201, bc=W.DIRICHLET, bc_left=0.3, bc_right=-0.7),
              W.fourier_ic(3072, 18)), 1024, 64),
    (lambda: (W.heat_problem(2048, 1313, bc=W.REFLECTIVE), W.fourier_ic(2048, 19)), 1024, 64),
    (lambda: (W.ks_problem(4096, 555), W.fourier_ic(4096, 20)), 1024, 64),
    (lambda: (W.Problem(W.KS, 3072, 421, 2.0 ** -8, 0.5, bc=W.DIRICHLET, bc_left=(0.4, 0, 0),
                        bc_right=(-0.2, 0, 0)), W.fourier_ic(3072, 21)), 1024, 64),
    (lambda: (W.sod_problem(2048, 777), W.sod_ic(2048)), 512, 64),        # P = 8, three variables
    # heat on one-wave tiles of 8 points per lane (select-free narrowing in the 8-point class),
    # an odd tile count, remainders, Dirichlet and insulated walls
    (lambda: (W.heat_problem(2560, 1111, bc=W.DIRICHLET, bc_left=-0.4, bc_right=0.9),
              W.fourier_ic(2560, 22)), 512, 64),
    (lambda: (W.heat_problem(1536, 700, bc=W.REFLECTIVE), W.fourier_ic(1536, 23)), 512, 64),
    # Sod on one-wave tiles of 1, 2 and 4 points per lane (lane exchange of pressures, ratios
    # and fluxes), an odd tile count and remainders
    (lambda: (W.sod_problem(1280, 641), W.sod_ic(1280)), 256, 64),
    (lambda: (W.sod_problem(1024, 900), W.sod_ic(1024)), 128, 64),
    (lambda: (W.sod_problem(768, 333), W.sod_ic(768)), 64, 64),
]


@pytest.mark.parametrize("case", range(len(SMALL)))
def test_classic_matches_oracle(oracle_mod, case):
    factory, _, _ = SMALL[case]
    prob, ic = factory()
    got = gpu_solve(prob, ic, "classic")
    want = oracle_mod.solve(prob, ic)
    assert relerr(got, want) <= TOL
    assert np.array_equal(got, want)  # same operation order, correctly rounded / and sqrt


@pytest.mark.parametrize("case", range(len(SMALL)))
def test_swept_matches_classic_bitwise_and_oracle(oracle_mod, case):
    factory, width, threads = SMALL[case]
    prob, ic = factory()
    swept = gpu_solve(prob, ic, "swept", width, threads)
    classic = gpu_solve(prob, ic, "classic", width, threads)
    assert np.array_equal(swept, classic)
    assert relerr(swept, oracle_mod.solve(prob, ic)) <= TOL


@pytest.mark.parametrize("shape", [(512, 128), (256, 64), (128, 64)])
@pytest.mark.parametrize("limiter", [0, 1])
def test_euler_limiter_orientations(oracle_mod, limiter, shape):
    """Both limiter orientations, on a multi-wave tile (plain rule) and on one-wave tiles
    (pressures, ratios and fluxes exchanged between lanes)."""
    prob, ic = W.cfg_sod(11)
    prob = prob.with_steps(700)
    got = gpu_solve(prob, ic, "swept", *shape, limiter=limiter)
    assert np.array_equal(got, oracle_mod.solve(prob, ic, limiter=limiter))


# ---------------------------------------------------------- named workloads

def test_cfg_heat_n1024_10k_steps_w64(oracle_mod):
    """Heat FTCS, N = 1024 periodic, Fo = 1/4, 10,000 steps, triangle width 64."""
    prob, ic = W.cfg_heat_small()
    got = gpu_solve(prob, ic, "swept", 64, 64)
    want = oracle_mod.solve(prob, ic)
    assert relerr(got, want) <= TOL
    assert np.array_equal(got, want)


@pytest.mark.parametrize("scheme", [W.HEAT, W.KS])
def test_cfg_sweep_n4096_50k_steps(oracle_mod, scheme):
    prob, ic = W.cfg_sweep(scheme, 12)
    got = gpu_solve(prob, ic, "swept")
    want = oracle_mod.solve(prob, ic)
    assert relerr(got, want) <= TOL


def test_cfg_sod_n4096_to_t02(oracle_mod):
    prob, ic = W.cfg_sod(12)
    got = gpu_solve(prob, ic, "swept")
    assert relerr(got, oracle_mod.solve(prob, ic)) <= TOL
    assert np.array_equal(got, gpu_solve(prob, ic, "classic"))


# ------------------------------------------------- full size (bench configuration)

def _heat_closed_form(n, m, seed):
    """Exact discrete solution of periodic FTCS at Fo = 1/4 for the Fourier-mode IC."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=16).astype(np.longdouble)
    b = rng.uniform(-1.0, 1.0, size=16).astype(np.longdouble)
    i = np.arange(n, dtype=np.longdouble)
    pi = np.longdouble(np.pi)
    out = np.zeros(n, dtype=np.longdouble)
    for k in range(1, 17):
        g = np.cos(pi * k / n) ** 2
        th = 2 * pi * k * i / n
        out += (a[k - 1] * np.cos(th) + b[k - 1] * np.sin(th)) * g ** m
    return out.astype(np.float64)


def test_full_size_heat_n2p20_50k_steps():
    """Bench configuration: heat, N = 2^20, 50,000 steps, default (tuned) tile shape.
    Swept == classic bitwise; both within 1e-12 of the discrete closed form."""
    prob, ic = W.cfg_sweep(W.HEAT, 20)
    swept = gpu_solve(prob, ic, "swept")
    classic = gpu_solve(prob, ic, "classic")
    assert np.array_equal(swept, classic)
    assert relerr(swept[0], _heat_closed_form(prob.n, prob.nsteps, 2 + 20)) <= TOL


def test_full_size_ks_n2p20_swept_equals_classic():
    """Bench configuration: KS, N = 2^20, 50,000 steps: swept == classic bitwise and the
    mean is conserved (the flux-form differences telescope on the periodic grid)."""
    prob, ic = W.cfg_sweep(W.KS, 20)
    swept = gpu_solve(prob, ic, "swept")
    classic = gpu_solve(prob, ic, "classic")
    assert np.array_equal(swept, classic)
    assert np.isfinite(swept).all()
    assert abs(swept.sum() - ic.sum()) < 1e-7 * prob.n


def test_full_size_ks_sampled_against_oracle_windows(oracle_mod):
    """KS, N = 2^20, 2,000 steps: a point after m steps depends only on the 4m points on
    each side, so the oracle on a window of 2*(4m)+1 points reproduces it exactly."""
    m = 2000
    prob, ic = W.cfg_sweep(W.KS, 20, nsteps=m)
    got = gpu_solve(prob, ic, "swept")
    reach = 2 * 2 * m
    for center in (0, 123_457, prob.n // 2 + 31, prob.n - 1):
        idx = (center + np.arange(-reach - 8, reach + 9)) % prob.n
        win = W.ks_problem(len(idx), m)
        ref = oracle_mod.solve(win, ic[:, idx])
        mid = reach + 8
        assert got[0, center] == ref[0, mid], center


def test_full_size_sod_n2p20_prefix_swept_equals_classic():
    """Sod at N = 2^20 (1.15M steps to t = 0.2), the first 20,000 steps in the tuned tile
    shape: swept == classic bitwise, density and pressure stay positive."""
    prob, ic = W.cfg_sod(20)
    prob = prob.with_steps(20_000)
    swept = gpu_solve(prob, ic, "swept")
    classic = gpu_solve(prob, ic, "classic")
    assert np.array_equal(swept, classic)
    rho, m, e = swept
    assert (rho > 0).all() and (e - 0.5 * m * m / rho > 0).all()


def test_full_size_sod_sampled_against_oracle_windows(oracle_mod):
    """Sod, N = 2^20, 2,000 steps: a cell after m steps depends only on the 4m cells on
    each side (two sub-steps of radius 2), so the oracle on a window with the same
    Dirichlet ends reproduces it exactly; the windows cover both tube ends and the
    initial discontinuity."""
    m = 2000
    prob, ic = W.cfg_sod(20, nsteps=m)
    got = gpu_solve(prob, ic, "swept")
    reach = 2 * 2 * m
    for center in (0, 7, prob.n // 2 - 1, prob.n // 2 + 5, 700_001, prob.n - 1):
        lo, hi = max(0, center - reach - 8), min(prob.n, center + reach + 9)
        win = W.Problem(W.EULER, hi - lo, m, prob.dt, prob.dx, bc=W.DIRICHLET, gamma=prob.gamma,
                        bc_left=prob.bc_left, bc_right=prob.bc_right)
        ref = oracle_mod.solve(win, ic[:, lo:hi])
        assert np.array_equal(got[:, center], ref[:, center - lo]), center


def test_largest_size_heat_and_ks_n2p26(oracle_mod):
    """N = 2^26 (the out-of-cache size the benchmark's anchors use), 300 steps, tuned
    shapes: swept == classic bitwise, and sampled points equal the oracle run on the
    window of points they depend on."""
    n, m = 1 << 26, 300
    for prob, reach in ((W.heat_problem(n, m), m), (W.ks_problem(n, m), 4 * m)):
        ic = W.random_ic(n, 1, seed=26 + prob.scheme)
        swept = gpu_solve(prob, ic, "swept")
        assert np.array_equal(swept, gpu_solve(prob, ic, "classic"))
        for center in (0, 12_345_679, n - 1):
            idx = (center + np.arange(-reach - 4, reach + 5)) % n
            ref = oracle_mod.solve(dataclasses.replace(prob, n=len(idx)), ic[:, idx])
            assert swept[0, center] == ref[0, reach + 4], (prob.scheme, center)


@pytest.mark.parametrize("scheme", [W.HEAT, W.KS, W.EULER])
def test_ragged_n_only_narrow_tiles_divide(oracle_mod, scheme):
    """N = 64 x 12293 (an odd multiple of 64: only the 64-point tile divides it), tuned
    plan: swept equals the oracle bit for bit."""
    n = 64 * 12293
    if scheme == W.EULER:
        prob, ic = W.sod_problem(n, 150), W.sod_ic(n)
    else:
        prob = W.heat_problem(n, 700) if scheme == W.HEAT else W.ks_problem(n, 300)
        ic = W.fourier_ic(n, seed=5)
    with sw.Plan(prob) as plan:
        assert plan.info()["width"] == 64 and plan.info()["swept_ok"] == 1
    assert np.array_equal(gpu_solve(prob, ic, "swept"), oracle_mod.solve(prob, ic))


# ------------------------------------------------------------ invariances

def test_repeat_runs_bitwise_identical():
    """One plan solved 100 times from the same state (multi-wave and one-wave tiles, and the
    classic path): every result is bit-identical (no races between waves or launches)."""
    prob, ic = W.cfg_sweep(W.KS, 14, nsteps=600)
    for width, threads, kind in ((1024, 128, "swept"), (512, 64, "swept"), (0, 0, "classic")):
        print(f"[gpu] 100 repeats of {kind} w={width} T={threads}", flush=True)
        with sw.Plan(prob, width, threads) as plan:
            x0 = torch.tensor(ic, dtype=torch.float64, device=DEV)
            ref = None
            for _ in range(100):
                x = x0.clone()
                getattr(plan, kind)(x)
                if ref is None:
                    ref = x
                else:
                    assert torch.equal(x, ref)
            torch.cuda.synchronize()


@pytest.mark.parametrize("scheme", [W.KS, W.HEAT])
def test_tile_shape_invariance_bitwise(scheme):
    """Every tile shape gives the same bits: one-wave tiles of 2 to 16 points per lane (whose
    classes select or update select-free) and multi-wave tiles."""
    prob, ic = W.cfg_sweep(scheme, 14, nsteps=2000)
    shapes = [(128, 64), (256, 64), (512, 64), (1024, 64), (1024, 128), (2048, 128), (2048, 256),
              (4096, 512), (1024, 512), (8192, 512)]
    outs = [gpu_solve(prob, ic, "swept", w, t) for w, t in shapes]
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


def test_resume_invariant_bitwise():
    """solve(a) then solve(b) == solve(a + b)."""
    prob, ic = W.cfg_sweep(W.HEAT, 13, nsteps=1000)
    once = gpu_solve(prob, ic, "swept", 512, 64)
    half = gpu_solve(prob.with_steps(377), ic, "swept", 512, 64)
    twice = gpu_solve(prob.with_steps(623), half, "swept", 512, 64)
    assert np.array_equal(once, twice)


def test_no_graph_flag_same_result():
    prob, ic = W.cfg_sweep(W.KS, 13, nsteps=900)
    a = gpu_solve(prob, ic, "swept", 512, 64)
    b = gpu_solve(prob, ic, "swept", 512, 64, flags=sw.SW_TUNE_NO_GRAPH)
    c = gpu_solve(prob, ic, "classic", 512, 64, flags=sw.SW_TUNE_NO_GRAPH)
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_plan_reuse_and_graph_recapture_on_new_buffer():
    prob, ic = W.cfg_sweep(W.HEAT, 12, nsteps=700)
    with sw.Plan(prob, 256, 64) as plan:
        xs = [torch.tensor(ic, dtype=torch.float64, device=DEV) for _ in range(3)]
        for x in xs:
            plan.swept(x)
        plan.swept(xs[0])
        torch.cuda.synchronize()
        single = xs[1].cpu().numpy()
        assert np.array_equal(xs[1].cpu().numpy(), xs[2].cpu().numpy())
        double = gpu_solve(prob.with_steps(1400), ic, "swept", 256, 64)
        assert np.array_equal(xs[0].cpu().numpy(), double)
        assert not np.array_equal(single, double)


# ------------------------------------------------------------------ edge cases

def test_zero_steps_is_identity():
    prob = W.heat_problem(1024, 0)
    ic = W.fourier_ic(1024, 9)
    assert np.array_equal(gpu_solve(prob, ic, "swept"), ic)
    assert np.array_equal(gpu_solve(prob, ic, "classic"), ic)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 100])
@pytest.mark.parametrize("scheme", [W.HEAT, W.KS])
def test_tiny_and_ragged_grids_classic(oracle_mod, n, scheme):
    prob = W.heat_problem(n, 37) if scheme == W.HEAT else W.ks_problem(n, 37)
    ic = W.random_ic(n, 1, seed=n)
    got = gpu_solve(prob, ic, "classic")
    assert np.array_equal(got, oracle_mod.solve(prob, ic))


@pytest.mark.parametrize("n", [2, 3, 5, 100])
def test_tiny_reflective_heat_classic(oracle_mod, n):
    prob = W.heat_problem(n, 41, bc=W.REFLECTIVE)
    ic = W.random_ic(n, 1, seed=100 + n)
    assert np.array_equal(gpu_solve(prob, ic, "classic"), oracle_mod.solve(prob, ic))


def test_ragged_grid_euler_dirichlet_classic(oracle_mod):
    prob = W.sod_problem(1000, 300)
    ic = W.sod_ic(1000)
    assert np.array_equal(gpu_solve(prob, ic, "classic"), oracle_mod.solve(prob, ic))


def test_swept_unsupported_when_no_width_divides_n():
    prob = W.heat_problem(1000, 10)
    with sw.Plan(prob) as plan:
        x = torch.zeros((1, 1000), dtype=torch.float64, device=DEV)
        with pytest.raises(sw.SweptError) as e:
            plan.swept(x)
        assert e.value.status == N.SW_EUNSUPPORTED
        plan.classic(x)
        torch.cuda.synchronize()


def test_host_pointer_rejected():
    prob = W.heat_problem(1024, 10)
    host = np.zeros(1024)
    with sw.Plan(prob, 64, 64) as plan:
        rc = N.lib().swept_solve(plan._h, host.ctypes.data, None)
        assert rc == N.SW_EINVAL
        assert b"device" in N.lib().sw_last_error()


def test_nan_check_flag():
    prob = W.heat_problem(1024, 50)
    ic = W.fourier_ic(1024, 1)
    ic[0, 100] = np.nan
    with sw.Plan(prob, 64, 64, flags=sw.SW_TUNE_CHECK_NAN) as plan:
        x = torch.tensor(ic, dtype=torch.float64, device=DEV)
        with pytest.raises(sw.SweptError) as e:
            plan.swept(x)
        assert e.value.status == N.SW_ENAN


def test_large_dirichlet_heat_and_sod_swept_equals_classic():
    for prob, ic in ((W.heat_problem(1 << 18, 5000, bc=W.DIRICHLET, bc_left=1.0, bc_right=-1.0),
                      W.fourier_ic(1 << 18, 3)),
                     (W.heat_problem(1 << 18, 5000, bc=W.REFLECTIVE), W.fourier_ic(1 << 18, 4)),
                     (W.sod_problem(1 << 16, 3000), W.sod_ic(1 << 16))):
        assert np.array_equal(gpu_solve(prob, ic, "swept"), gpu_solve(prob, ic, "classic"))


# ------------------------------------------------------------------ Hybrid variant

HYBRID = [  # non-periodic problems: the host computes the straddling tile of every shifted phase
    (lambda: (W.heat_problem(4096, 2000, bc=W.REFLECTIVE), W.fourier_ic(4096, 41)), 512, 64),
    (lambda: (W.heat_problem(1 << 16, 3000, bc=W.REFLECTIVE), W.fourier_ic(1 << 16, 42)), 0, 0),
    (lambda: (W.heat_problem(2048, 999, bc=W.DIRICHLET, bc_left=0.3, bc_right=-0.6), W.fourier_ic(2048, 43)),
     256, 128),
    (lambda: (W.heat_problem(1024, 333, bc=W.REFLECTIVE), W.fourier_ic(1024, 44)), 1024, 64),   # K = 1
    (lambda: (W.Problem(W.KS, 4096, 700, 2.0 ** -8, 0.5, bc=W.DIRICHLET, bc_left=(0.4, 0, 0),
                        bc_right=(-0.2, 0, 0)), W.fourier_ic(4096, 45)), 1024, 64),
    (lambda: (W.sod_problem(4096, 1200), W.sod_ic(4096)), 256, 64),
    (lambda: (W.sod_problem(1 << 14), W.sod_ic(1 << 14)), 0, 0),                           # to t = 0.2
]


@pytest.mark.parametrize("case", range(len(HYBRID)))
def test_hybrid_equals_swept_and_oracle(oracle_mod, case):
    """Hybrid variant (Sec. 5.1): the straddling tile on the host, the rest on the GPU;
    bit-identical to the all-GPU swept solve and to the oracle."""
    factory, width, threads = HYBRID[case]
    prob, ic = factory()
    got = gpu_solve(prob, ic, "swept", width, threads, flags=sw.SW_TUNE_HYBRID)
    assert np.array_equal(got, gpu_solve(prob, ic, "swept", width, threads))
    assert np.array_equal(got.reshape(prob.nvars, prob.n), oracle_mod.solve(prob, ic))


def test_hybrid_repeated_solves_on_one_plan():
    """Two hybrid solves in a row on one plan (the second waits for the first's host work)."""
    prob, ic = W.heat_problem(8192, 1500, bc=W.REFLECTIVE), W.fourier_ic(8192, 46)
    with sw.Plan(prob, 512, 64, sw.SW_TUNE_HYBRID) as plan:
        a = torch.tensor(ic, dtype=torch.float64, device=DEV)
        b = a.clone()
        plan.swept(a)
        plan.swept(b)
        torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert np.array_equal(a.cpu().numpy(), gpu_solve(prob, ic, "swept", 512, 64))


# ---------------------------------------------------------------- Shared variant (rows in LDS)

LDS_CASES = [  # (problem factory, width, threads): remainders, walls, and widths near 160 KB of LDS
    (lambda: (W.heat_problem(4096, 1777), W.fourier_ic(4096, 31)), 1024, 256),
    (lambda: (W.heat_problem(3072, 1201, bc=W.DIRICHLET, bc_left=0.3, bc_right=-0.7),
              W.fourier_ic(3072, 32)), 512, 128),
    (lambda: (W.heat_problem(2048, 1313, bc=W.REFLECTIVE), W.fourier_ic(2048, 33)), 1024, 1024),
    (lambda: (W.heat_problem(20352, 9000), W.fourier_ic(20352, 34)), 10176, 192),      # 162,848 B of LDS
    (lambda: (W.ks_problem(8192, 555), W.fourier_ic(8192, 35)), 2048, 512),
    (lambda: (W.Problem(W.KS, 3072, 421, 2.0 ** -8, 0.5, bc=W.DIRICHLET, bc_left=(0.4, 0, 0),
                        bc_right=(-0.2, 0, 0)), W.fourier_ic(3072, 36)), 1024, 64),
    (lambda: (W.sod_problem(2048, 777), W.sod_ic(2048)), 1024, 256),
    (lambda: (W.sod_problem(6656, 1500), W.sod_ic(6656)), 3328, 256),                  # 159,936 B of LDS
]


@pytest.mark.parametrize("case", range(len(LDS_CASES)))
def test_lds_variant_matches_classic_bitwise_and_oracle(oracle_mod, case):
    """The Shared variant (SW_TUNE_LDS: each tile's two rows in LDS, threads striding over
    the points, one barrier per level) gives the register kernel's and classic's bits."""
    factory, width, threads = LDS_CASES[case]
    prob, ic = factory()
    lds = gpu_solve(prob, ic, "swept", width, threads, flags=sw.SW_TUNE_LDS)
    classic = gpu_solve(prob, ic, "classic")   # (the register kernel cannot take every LDS width)
    assert np.array_equal(lds, classic)
    assert relerr(lds, oracle_mod.solve(prob, ic)) <= TOL
