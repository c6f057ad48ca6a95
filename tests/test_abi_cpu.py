"""The C interface on the CPU: the library loads, exports every symbol declared
in include/swept.h, and its host logic (validation, plan geometry, error
reporting) works without a GPU.  No kernel is launched here."""
import ctypes
import json
import os
import re

import pytest

import workloads as W
from paper_1705_03162_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swept.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(N.LIB_PATH):
        from paper_1705_03162_amd import build
        build.build(verbose=False)
    return N.lib()


def test_header_declares_the_interface():
    names = declared_functions()
    for n in ["swept_plan", "swept_plan_info", "swept_solve", "classic_solve", "swept_plan_destroy",
              "batch_create", "batch_submit", "batch_run", "batch_poll", "batch_wait",
              "batch_cancel", "batch_destroy", "sw_strerror", "sw_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(N.LIB_PATH)
    for name in declared_functions():
        assert hasattr(raw, name), name
    assert set(declared_functions()) <= set(N.SIGNATURES)


def _plan(lib, prob, width=0, threads=0, flags=0):
    p = N.problem_struct(prob)
    t = N.SwTuning(width, threads, flags)
    h = ctypes.c_void_p()
    rc = lib.swept_plan(ctypes.byref(p), ctypes.byref(t), ctypes.byref(h))
    return rc, h


def _info(lib, h):
    i = N.SwPlanInfo()
    assert lib.swept_plan_info(h, ctypes.byref(i)) == 0
    return i


def test_plan_geometry_heat_cfg1(lib):
    prob, _ = W.cfg_heat_small()
    rc, h = _plan(lib, prob, 64, 64)
    assert rc == 0
    i = _info(lib, h)
    assert (i.width, i.threads, i.points_per_lane, i.radius, i.substeps, i.nvars) == (64, 64, 1, 1, 1, 1)
    assert (i.nodes, i.levels_per_phase, i.full_phases, i.remainder) == (16, 32, 312, 16)
    assert i.swept_launches == 1 + 311 + 1 + 2 and i.classic_launches == 10_000
    lib.swept_plan_destroy(h)


def test_plan_geometry_ks_large(lib):
    rc, h = _plan(lib, W.ks_problem(1 << 20, 50_000), 1024, 128)
    assert rc == 0
    i = _info(lib, h)
    assert (i.points_per_lane, i.levels_per_phase, i.full_phases, i.remainder) == (8, 256, 390, 160)
    assert i.nodes == 1024 and i.classic_launches == 100_000 and i.swept_launches == 393
    lib.swept_plan_destroy(h)


GOLDEN = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_geometry.json")))


def _phase_levels(width, radius):
    """Levels per swept phase for a node of `width` points: H = w / (2 r)."""
    return width // (2 * radius)


def test_paper_geometry_pins():
    """Printed geometry of Sec. 4.2 and Sec. 6 follows from H = w/(2r) and two rows of
    w + k - 1 values (k = 2r + 1)."""
    n = 512
    assert sum(2 * j for j in range(1, n // 2 + 1)) == GOLDEN["full_triangle_values_n512_radius1"]["value"]
    assert 2 * (n + 3 - 1) == GOLDEN["two_row_working_array_values_n512_width3"]["value"]
    w32 = GOLDEN["register_ks_node_points"]["value"]
    h32 = _phase_levels(w32, 2)                      # KS: r = 2, two sub-steps per step
    assert h32 // 2 == GOLDEN["register_ks_timesteps_per_cycle"]["value"]
    assert h32 == GOLDEN["register_ks_launch_ratio_vs_classic"]["value"]
    assert _phase_levels(128, 2) // h32 == GOLDEN["shared_n128_vs_register_n32_launch_ratio"]["value"]


@pytest.mark.parametrize("width,threads", [(128, 64), (256, 64), (1024, 128)])
def test_plan_levels_per_phase_matches_formula(lib, width, threads):
    rc, h = _plan(lib, W.ks_problem(1 << 14, 1000), width, threads)
    assert rc == 0
    i = _info(lib, h)
    assert i.levels_per_phase == _phase_levels(width, 2)
    # one phase advances H levels = H/2 timesteps; classic takes 2 launches per timestep
    assert i.full_phases == (2 * 1000) // i.levels_per_phase
    lib.swept_plan_destroy(h)


def test_default_shape_divides_n(lib):
    for prob in (W.heat_problem(1 << 20, 10), W.ks_problem(1 << 16, 10), W.sod_problem(1 << 14, 10),
                 W.heat_problem(1024, 10), W.ks_problem(3 * 1024, 5)):
        rc, h = _plan(lib, prob)
        assert rc == 0
        i = _info(lib, h)
        assert i.swept_ok == 1 and prob.n % i.width == 0
        lib.swept_plan_destroy(h)


def _table(kind="swept"):
    """Rows of the tuning table: swept (scheme, log2n) -> (width, threads), or classic
    (scheme, log2n) -> threads."""
    out = {}
    with open(os.path.join(ROOT, "paper_1705_03162_amd", "tune_gfx950.txt")) as f:
        for line in f:
            parts = line.split()
            if not parts or parts[0].startswith("#"):
                continue
            if parts[0] == "classic":
                if kind == "classic":
                    out[(int(parts[1]), int(parts[2]))] = int(parts[3])
            elif parts[0] == "batch":
                continue
            elif kind == "swept":
                s, lg, w, t = (int(x) for x in parts[:4])
                out[(s, lg)] = (w, t)
    return out


def test_classic_threads_from_the_table_or_the_tuning(lib):
    """The classic work-group size comes from the table's classic row for the size
    class, or from sw_tuning.classic_threads when given; illegal sizes are rejected."""
    table = _table("classic")
    assert table, "the tuning table holds classic rows"
    for (scheme, lg), t in sorted(table.items())[:6]:
        n = 1 << lg
        prob = (W.heat_problem(n, 10) if scheme == W.HEAT else
                W.ks_problem(n, 10) if scheme == W.KS else W.sod_problem(n, 10))
        rc, h = _plan(lib, prob)
        assert rc == 0
        assert _info(lib, h).classic_threads == t, (scheme, lg)
        lib.swept_plan_destroy(h)
    p = N.problem_struct(W.heat_problem(4096, 10))
    for ct, ok in ((128, True), (1024, True), (96, False), (2048, False)):
        tun = N.SwTuning(0, 0, 0, ct)
        h = ctypes.c_void_p()
        rc = lib.swept_plan(ctypes.byref(p), ctypes.byref(tun), ctypes.byref(h))
        assert (rc == 0) == ok, ct
        if ok:
            assert _info(lib, h).classic_threads == ct
            lib.swept_plan_destroy(h)


def test_hybrid_flag_accepted_and_unknown_flags_rejected(lib):
    rc, h = _plan(lib, W.sod_problem(4096, 10), flags=N.SW_TUNE_HYBRID)
    assert rc == 0
    lib.swept_plan_destroy(h)
    rc, _ = _plan(lib, W.sod_problem(4096, 10), flags=64)
    assert rc == N.SW_EINVAL


def test_lds_variant_shapes(lib):
    """SW_TUNE_LDS (the Shared variant) takes widths the register kernel cannot (any number
    of points per thread up to 64) as long as the two rows fit in 160 KB of LDS, and it
    excludes the Hybrid variant and the allocation-free solve."""
    heat = W.heat_problem(1 << 16, 10)
    rc, h = _plan(lib, heat, 8192, 1024, flags=N.SW_TUNE_LDS)
    assert rc == 0
    i = _info(lib, h)
    assert (i.width, i.threads, i.points_per_lane) == (8192, 1024, 8)
    lib.swept_plan_destroy(h)
    assert _plan(lib, heat, 8192, 1024)[0] == N.SW_EINVAL                   # register budget
    assert _plan(lib, heat, 16384, 1024, flags=N.SW_TUNE_LDS)[0] == N.SW_EINVAL   # 262 KB of rows
    assert b"160 KB" in lib.sw_last_error()
    assert _plan(lib, heat, 8192, 64, flags=N.SW_TUNE_LDS)[0] == N.SW_EINVAL      # 128 points per thread
    sod = W.sod_problem(1 << 14, 10)
    assert _plan(lib, sod, 4096, 1024, flags=N.SW_TUNE_LDS)[0] == N.SW_EINVAL     # 3 variables: 197 KB
    rc, h = _plan(lib, sod, 2048, 1024, flags=N.SW_TUNE_LDS)
    assert rc == 0
    lib.swept_plan_destroy(h)
    assert _plan(lib, sod, 2048, 1024, flags=N.SW_TUNE_LDS | N.SW_TUNE_HYBRID)[0] == N.SW_EINVAL
    ok = N.problem_struct(W.ks_problem(1 << 20, 10))
    t = N.SwTuning(1024, 64, N.SW_TUNE_LDS)
    assert lib.swept_solve_noalloc(ctypes.byref(ok), ctypes.byref(t), None, None) == N.SW_EINVAL


def test_tuned_shapes_from_nearest_measured_class(lib):
    """Sizes the table measured take their row; larger sizes take the largest measured
    class, smaller ones the smallest, as long as that width divides n."""
    table = _table()
    for scheme in (W.HEAT, W.KS, W.EULER):
        classes = sorted(lg for s, lg in table if s == scheme)
        for lg, cls in ((classes[-1], classes[-1]), (classes[-1] + 4, classes[-1]),
                        (classes[0] - 1, classes[0])):
            n = 1 << lg
            prob = (W.heat_problem(n, 10) if scheme == W.HEAT else
                    W.ks_problem(n, 10) if scheme == W.KS else W.sod_problem(n, 10))
            w, t = table[(scheme, cls)]
            if n % w:
                continue
            rc, h = _plan(lib, prob)
            assert rc == 0
            i = _info(lib, h)
            assert (i.width, i.threads) == (w, t), (scheme, lg)
            lib.swept_plan_destroy(h)


def test_no_legal_width_still_plans_for_classic(lib):
    rc, h = _plan(lib, W.heat_problem(1000, 10))
    assert rc == 0
    assert _info(lib, h).swept_ok == 0
    lib.swept_plan_destroy(h)


@pytest.mark.parametrize("mutate,code", [
    (lambda p: setattr(p, "scheme", 7), N.SW_EINVAL),
    (lambda p: setattr(p, "bc", 3), N.SW_EINVAL),
    (lambda p: setattr(p, "n", 0), N.SW_EINVAL),
    (lambda p: setattr(p, "nsteps", -1), N.SW_EINVAL),
    (lambda p: setattr(p, "dt", 0.0), N.SW_EINVAL),
    (lambda p: setattr(p, "dx", float("nan")), N.SW_EINVAL),
    (lambda p: setattr(p, "flags", 8), N.SW_EINVAL),
])
def test_invalid_problems_rejected(lib, mutate, code):
    p = N.problem_struct(W.heat_problem(256, 10))
    mutate(p)
    h = ctypes.c_void_p()
    assert lib.swept_plan(ctypes.byref(p), None, ctypes.byref(h)) == code
    assert not h.value
    assert len(lib.sw_last_error()) > 0


@pytest.mark.parametrize("width,threads", [(96, 64), (64, 32), (64 * 32, 64), (128, 128 + 64),
                                           (256, 64 * 2)])
def test_invalid_shapes_rejected(lib, width, threads):
    rc, h = _plan(lib, W.ks_problem(1 << 12, 10), width, threads)
    # KS needs >= 2 points per lane: (256, 128) has P = 2 and is legal
    if (width, threads) == (256, 128):
        assert rc == 0
        lib.swept_plan_destroy(h)
    else:
        assert rc == N.SW_EINVAL


def test_eight_points_per_lane_caps_work_group_at_512(lib):
    """With P >= 8 the rows take 2 P doubles per lane; the kernels are compiled for at
    most 512 lanes (two waves per SIMD), so 16-wave tiles of 8 points per lane are refused."""
    prob = W.ks_problem(1 << 14, 10)
    rc, h = _plan(lib, prob, 4096, 512)
    assert rc == 0
    lib.swept_plan_destroy(h)
    rc, _ = _plan(lib, prob, 8192, 1024)
    assert rc == N.SW_EINVAL
    rc, h = _plan(lib, prob, 1024, 1024)          # P = 1: 16 waves allowed
    assert rc == 0
    lib.swept_plan_destroy(h)


def test_width_must_divide_n(lib):
    rc, _ = _plan(lib, W.heat_problem(1000, 10), 64, 64)
    assert rc == N.SW_EINVAL


def test_strerror_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, -6, -7, 99):
        assert lib.sw_strerror(code)


def test_destroy_null_is_noop(lib):
    lib.swept_plan_destroy(None)
    lib.batch_destroy(None)


def test_binding_rejects_bad_state_before_the_library(lib):
    """The C interface takes a bare pointer, so the binding checks the tensor first:
    type, dtype, device, contiguity and size (no kernel can run on a wrong buffer)."""
    torch = pytest.importorskip("torch")
    import paper_1705_03162_amd as sw
    prob = W.heat_problem(1024, 10)
    with sw.Plan(prob, 64, 64) as plan:
        with pytest.raises(TypeError):
            plan.swept([0.0] * 1024)
        with pytest.raises(ValueError):
            plan.swept(torch.zeros(1024, dtype=torch.float64))          # host tensor
        with pytest.raises(ValueError):
            plan.classic(torch.zeros(1024, dtype=torch.float32))        # wrong dtype


def test_noalloc_rejects_before_touching_the_device(lib):
    """The allocation-free solve checks its static scratch limit (32 MiB of edges)
    and its flags before it looks at the state pointer or the device."""
    big = N.problem_struct(W.sod_problem(1 << 20, 10))     # Euler at 2^20: ~50 MB of edges
    rc = lib.swept_solve_noalloc(ctypes.byref(big), None, None, None)
    assert rc == N.SW_EINVAL
    assert b"static scratch" in lib.sw_last_error()
    ok = N.problem_struct(W.ks_problem(1 << 20, 10))      # KS at 2^20 fits (~16.8 MB)
    t = N.SwTuning(1024, 64, N.SW_TUNE_CHECK_NAN)
    assert lib.swept_solve_noalloc(ctypes.byref(ok), ctypes.byref(t), None, None) == N.SW_EINVAL
    assert b"flags" in lib.sw_last_error()
    t = N.SwTuning(1024, 64, 0)
    assert lib.swept_solve_noalloc(ctypes.byref(ok), ctypes.byref(t), None, None) == N.SW_EINVAL
    assert b"NULL" in lib.sw_last_error()                  # got past the size check to the state
