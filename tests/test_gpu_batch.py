"""Batched and served solves on the GPU: each result equals the same problem
solved alone (swept_solve) and the oracle, bit for bit."""
import threading
import time

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
import paper_1705_03162_amd as sw  # noqa: E402
from paper_1705_03162_amd import _native as N  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def alone(prob, ic):
    with sw.Plan(prob) as plan:
        x = torch.tensor(ic, dtype=torch.float64, device=DEV)
        if plan.info()["swept_ok"]:
            plan.swept(x)
        else:
            plan.classic(x)
        torch.cuda.synchronize()
    return x.cpu().numpy()


def charged_bytes(prob, x):
    """Device bytes a batch charges this solve, read back from the library (a probe
    batch that is never run)."""
    with sw.Batch(budget_bytes=1 << 40) as b:
        return b.info(b.submit(prob, x))["resident_bytes"]


def mixed_problems(count, seed, schemes=(W.HEAT, W.KS), nmax=8192, smax=900):
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        scheme = schemes[int(rng.integers(0, len(schemes)))]
        n = 64 * int(rng.integers(1, nmax // 64 + 1))
        steps = int(rng.integers(1, smax))
        if scheme == W.HEAT:
            prob, ic = W.heat_problem(n, steps), W.fourier_ic(n, seed=j)
        elif scheme == W.KS:
            prob, ic = W.ks_problem(n, steps), W.fourier_ic(n, seed=j)
        else:
            prob, ic = W.sod_problem(n, steps), W.sod_ic(n)
        out.append((prob, ic))
    return out


def test_ensemble_each_result_equals_alone(oracle_mod):
    probs = mixed_problems(48, seed=1)
    probs.append((W.heat_problem(1000, 77), W.fourier_ic(1000, 5)))   # no swept width: classic
    probs.append((W.ks_problem(4096, 0), W.fourier_ic(4096, 6)))      # zero steps
    probs.append((W.heat_problem(2048, 613, bc=W.REFLECTIVE), W.fourier_ic(2048, 7)))
    probs.append((W.heat_problem(1024, 420, bc=W.DIRICHLET, bc_left=0.5, bc_right=-0.5),
                  W.fourier_ic(1024, 8)))
    print(f"[gpu] ensemble of {len(probs)} solves", flush=True)
    states = [torch.tensor(ic, dtype=torch.float64, device=DEV) for _, ic in probs]
    with sw.Batch(budget_bytes=1 << 34) as b:
        tickets = [b.submit(p, x) for (p, _), x in zip(probs, states)]
        b.run()
        for t in tickets:
            assert b.poll(t) == N.SW_TICKET_DONE
        infos = [b.info(t) for t in tickets]
    torch.cuda.synchronize()
    assert infos[-4]["swept"] == 0
    for (prob, ic), x in zip(probs, states):
        got = x.cpu().numpy()
        assert np.array_equal(got, alone(prob, ic))
        assert np.array_equal(got.reshape(prob.nvars, prob.n), oracle_mod.solve(prob, ic)), (prob.n, prob.nsteps)


@pytest.mark.parametrize("ppl", [0, 1, 4])
def test_persistent_ensemble_equals_oracle(oracle_mod, ppl):
    """The persistent ensemble launch (work-groups take tiles from a device queue and wait
    on the completion counters of the tiles they depend on): mixed heat, KS and Sod with
    every boundary type, default and forced tile shapes; every result equals the oracle
    bit for bit and the lock-step launch's."""
    probs = mixed_problems(40, seed=12, schemes=(W.HEAT, W.KS, W.EULER), nmax=8192, smax=700)
    probs.append((W.heat_problem(2048, 613, bc=W.REFLECTIVE), W.fourier_ic(2048, 7)))
    probs.append((W.heat_problem(1024, 420, bc=W.DIRICHLET, bc_left=0.5, bc_right=-0.5),
                  W.fourier_ic(1024, 8)))
    probs.append((W.ks_problem(512, 3), W.fourier_ic(512, 9)))          # fewer levels than one phase
    print(f"[gpu] persistent ensemble of {len(probs)} solves, points per lane {ppl}", flush=True)
    runs = []
    for persistent in (True, False):
        states = [torch.tensor(ic, dtype=torch.float64, device=DEV) for _, ic in probs]
        with sw.Batch(budget_bytes=1 << 34, persistent=persistent, points_per_lane=ppl) as b:
            tickets = [b.submit(p, x) for (p, _), x in zip(probs, states)]
            b.run()
            assert all(b.poll(t) == N.SW_TICKET_DONE for t in tickets)
            infos = [b.info(t) for t in tickets]
        torch.cuda.synchronize()
        assert all(i["end_s"] >= i["start_s"] for i in infos)
        runs.append([x.cpu().numpy() for x in states])
    for (prob, ic), a, b_ in zip(probs, runs[0], runs[1]):
        assert np.array_equal(a, b_)
        assert np.array_equal(a.reshape(prob.nvars, prob.n), oracle_mod.solve(prob, ic)), (prob.n, prob.nsteps)


def test_ensemble_with_euler_and_budget_waves(oracle_mod):
    """Mixed ensemble in budget-limited waves; each result equals the solve alone, and the
    Sod solves (batched one-wave tiles, pressures, ratios and fluxes exchanged between
    lanes) equal the oracle bit for bit."""
    probs = mixed_problems(20, seed=2, schemes=(W.HEAT, W.KS, W.EULER), nmax=4096, smax=400)
    states = [torch.tensor(ic, dtype=torch.float64, device=DEV) for _, ic in probs]
    budget = max(charged_bytes(p, x) for (p, _), x in zip(probs, states)) * 3   # a few solves per wave
    with sw.Batch(budget_bytes=budget, max_slots=5) as b:
        tickets = [b.submit(p, x) for (p, _), x in zip(probs, states)]
        b.run()
        assert all(b.poll(t) == N.SW_TICKET_DONE for t in tickets)
    for (prob, ic), x in zip(probs, states):
        got = x.cpu().numpy()
        assert np.array_equal(got, alone(prob, ic))
        if prob.scheme == W.EULER:
            assert np.array_equal(got, oracle_mod.solve(prob, ic)), (prob.n, prob.nsteps)


def test_served_mix_equals_alone(oracle_mod):
    """Continuous batching: solves arrive while others run; each result is the
    same as alone and equals the oracle bit for bit."""
    probs = mixed_problems(30, seed=3, schemes=(W.HEAT, W.KS, W.EULER), nmax=4096, smax=600)
    states = [torch.tensor(ic, dtype=torch.float64, device=DEV) for _, ic in probs]
    torch.cuda.synchronize()
    tickets = []
    with sw.Batch(budget_bytes=1 << 33, max_slots=8, serve=True) as b:
        def producer():
            for (p, _), x in zip(probs, states):
                tickets.append(b.submit(p, x))
                time.sleep(0.002)
        th = threading.Thread(target=producer)
        th.start()
        th.join()
        for t in tickets:
            b.wait(t, timeout_us=60_000_000)
        infos = [b.info(t) for t in tickets]
    assert all(i["status"] == N.SW_TICKET_DONE for i in infos)
    assert all(i["end_s"] >= i["start_s"] >= i["submit_s"] for i in infos)
    for (prob, ic), x in zip(probs, states):
        got = x.cpu().numpy()
        assert np.array_equal(got, alone(prob, ic))
        assert np.array_equal(got.reshape(prob.nvars, prob.n), oracle_mod.solve(prob, ic)), (prob.n, prob.nsteps)


def test_served_group_appends_and_compaction():
    """One (scheme, points per lane) group: 24 heat solves whose n are multiples of 512
    (eight points per lane for all), uneven step counts, submitted in three bursts.  Later
    solves join a group that is already ticking (appended to its table) and most solves
    finish while others still run (the table is rebuilt once half of it is finished);
    every result equals the solve alone."""
    rng = np.random.default_rng(11)
    probs = []
    for j in range(24):
        n = 512 * int(rng.integers(1, 9))
        probs.append((W.heat_problem(n, int(rng.integers(50, 3000))), W.fourier_ic(n, 100 + j)))
    states = [torch.tensor(ic, dtype=torch.float64, device=DEV) for _, ic in probs]
    torch.cuda.synchronize()
    print(f"[gpu] served group of {len(probs)} heat solves in three bursts", flush=True)
    with sw.Batch(budget_bytes=1 << 33, serve=True) as b:
        tickets = []
        for burst in range(3):
            for (p, _), x in list(zip(probs, states))[8 * burst:8 * burst + 8]:
                tickets.append(b.submit(p, x))
            time.sleep(0.02)
        for t in tickets:
            b.wait(t, timeout_us=60_000_000)
        infos = [b.info(t) for t in tickets]
    assert all(i["status"] == N.SW_TICKET_DONE and i["width"] == 512 for i in infos)
    for (prob, ic), x in zip(probs, states):
        assert np.array_equal(x.cpu().numpy(), alone(prob, ic))


def test_served_budget_never_exceeded():
    """A served batch whose budget holds only a few solves at a time: from every ticket's
    residency interval [start, end) and the bytes the library charged it (state plus edge
    slots, checked against the geometry), the bytes resident at once never exceed the
    budget, and every result equals the solve alone."""
    probs = mixed_problems(24, seed=9, schemes=(W.HEAT, W.KS, W.EULER), nmax=4096, smax=500)
    states = [torch.tensor(ic, dtype=torch.float64, device=DEV) for _, ic in probs]
    budget = 3 * max(charged_bytes(p, x) for (p, _), x in zip(probs, states))
    torch.cuda.synchronize()
    with sw.Batch(budget_bytes=budget, serve=True) as b:
        tickets = [b.submit(p, x) for (p, _), x in zip(probs, states)]
        for t in tickets:
            b.wait(t, timeout_us=60_000_000)
        infos = [b.info(t) for t in tickets]
    assert all(i["status"] == N.SW_TICKET_DONE for i in infos)
    sizes = [i["resident_bytes"] for i in infos]            # what the library charged
    for i, sz, (p, _) in zip(infos, sizes, probs):
        # its state plus 2K edge slots of nvars x 2 rows x (w/2 + r) doubles, rounded to 256 B
        w, r = i["width"], (1 if p.scheme == W.HEAT else 2)
        edges = 2 * (p.n // w) * p.nvars * 2 * (w // 2 + r) * 8
        assert sz == p.n * p.nvars * 8 + (edges + 255) // 256 * 256, (p.scheme, p.n)
    events = sorted([(i["start_s"], +sz) for i, sz in zip(infos, sizes)] +
                    [(i["end_s"], -sz) for i, sz in zip(infos, sizes)], key=lambda e: (e[0], e[1]))
    held = peak = 0
    for _, d in events:
        held += d
        peak = max(peak, held)
    assert peak <= budget
    assert peak > max(sizes)                     # the budget was actually shared
    for (prob, ic), x in zip(probs, states):
        assert np.array_equal(x.cpu().numpy(), alone(prob, ic))


def test_served_budget_queues_and_cancel():
    big = (W.ks_problem(1 << 16, 3000), W.fourier_ic(1 << 16, 1))
    small = [(W.heat_problem(1024, 200 + j), W.fourier_ic(1024, j)) for j in range(4)]
    xs = [torch.tensor(ic, dtype=torch.float64, device=DEV) for _, ic in [big] + small]
    budget = charged_bytes(big[0], xs[0]) + 10    # the big solve alone fills the budget
    with sw.Batch(budget_bytes=budget, serve=True) as b:
        tb = b.submit(big[0], xs[0])
        ts = [b.submit(p, x) for (p, _), x in zip(small, xs[1:])]
        b.cancel(ts[1])               # still queued behind the big solve
        assert b.poll(ts[1]) == N.SW_TICKET_CANCELLED
        for t in [tb] + ts:
            b.wait(t, timeout_us=60_000_000)
        assert b.poll(tb) == N.SW_TICKET_DONE
        for j, t in enumerate(ts):
            assert b.poll(t) == (N.SW_TICKET_CANCELLED if j == 1 else N.SW_TICKET_DONE)
    for j, ((prob, ic), x) in enumerate(zip([big] + small, xs)):
        if j == 2:
            assert np.array_equal(x.cpu().numpy(), ic)   # cancelled: untouched
        else:
            assert np.array_equal(x.cpu().numpy(), alone(prob, ic))


def test_oversized_solve_rejected():
    with sw.Batch(budget_bytes=1 << 20) as b:
        x = torch.zeros((1, 1 << 16), dtype=torch.float64, device=DEV)
        with pytest.raises(sw.SweptError) as e:
            b.submit(W.heat_problem(1 << 16, 10), x)
        assert e.value.status == N.SW_EBUSY
