"""GPU: the allocation-free swept solve equals the plan-based swept solve.

swept_solve_noalloc keeps its edge slots in the library's static device scratch
and enqueues its phases directly; on the same problem and tile shape it must
return exactly what swept_solve on a plan returns (bit for bit), on two calls in
a row with the second on a smaller input (the scratch keeps the first call's
contents), and both must equal the CPU oracle.  Called through the C interface.
"""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
import paper_1705_03162_amd as sw  # noqa: E402
from paper_1705_03162_amd import _native as N  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _noalloc(prob, ic, width, threads):
    x = torch.tensor(ic, dtype=torch.float64, device=DEV)
    p = N.problem_struct(prob)
    tun = N.SwTuning(width, threads, 0)
    stream = torch.cuda.current_stream().cuda_stream
    N.check(N.lib().swept_solve_noalloc(ctypes.byref(p), ctypes.byref(tun), x.data_ptr(), stream),
            "swept_solve_noalloc")
    torch.cuda.synchronize()
    return x.cpu().numpy()


def _plan(prob, ic, width, threads):
    with sw.Plan(prob, width, threads) as plan:
        x = torch.tensor(ic, dtype=torch.float64, device=DEV)
        plan.swept(x)
        torch.cuda.synchronize()
    return x.cpu().numpy()


# (first call, second smaller call) per scheme; shapes with remainders and
# several tiles; the KS pair puts the large call at the full n = 2^20 width
PAIRS = [
    ((W.heat_problem(1 << 16, 777), W.fourier_ic(1 << 16, 21), 1024, 64),
     (W.heat_problem(4096, 333), W.fourier_ic(4096, 22), 256, 64)),
    ((W.ks_problem(1 << 20, 40), W.fourier_ic(1 << 20, 23), 1024, 64),
     (W.ks_problem(2048, 301), W.fourier_ic(2048, 24), 512, 128)),
    ((W.sod_problem(8192, 700), W.sod_ic(8192), 256, 64),
     (W.sod_problem(1024, 500), W.sod_ic(1024), 128, 64)),
    ((W.heat_problem(8192, 901, bc=W.REFLECTIVE), W.fourier_ic(8192, 25), 512, 64),
     (W.heat_problem(1024, 455, bc=W.DIRICHLET, bc_left=0.5, bc_right=-0.25), W.fourier_ic(1024, 26),
      128, 64)),
]


@pytest.mark.parametrize("pair", range(len(PAIRS)))
def test_noalloc_equals_plan_on_two_calls(pair):
    for prob, ic, width, threads in PAIRS[pair]:
        print(f"[gpu] noalloc scheme={prob.scheme} bc={prob.bc} n={prob.n} steps={prob.nsteps} "
              f"w={width} T={threads}", flush=True)
        got = _noalloc(prob, ic, width, threads)
        want = _plan(prob, ic, width, threads)
        assert np.array_equal(got, want)
        if prob.n <= 8192:
            assert np.array_equal(got.reshape(prob.nvars, prob.n), oracle.solve(prob, ic))


def test_noalloc_tuned_shape_matches_plan():
    prob, ic = W.cfg_sweep(W.KS, 14, nsteps=500)
    print(f"[gpu] noalloc tuned shape n={prob.n}", flush=True)
    assert np.array_equal(_noalloc(prob, ic, 0, 0), _plan(prob, ic, 0, 0))


def test_noalloc_rejects_oversized_problem():
    prob, ic = W.cfg_sod(20, nsteps=10)   # Euler at 2^20 needs 50 MB of edges
    x = torch.tensor(ic, dtype=torch.float64, device=DEV)
    p = N.problem_struct(prob)
    rc = N.lib().swept_solve_noalloc(ctypes.byref(p), None, x.data_ptr(), None)
    assert rc == N.SW_EINVAL
    assert b"static scratch" in N.lib().sw_last_error()
