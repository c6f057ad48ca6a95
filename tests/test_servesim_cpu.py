"""The batched and served solve scheduler on the CPU.

batch.hip is compiled unchanged against a stand-in runtime (tests/hostsim/fakehip)
whose streams run lazily -- enqueued work runs only when the host waits for it, so
ticks are in flight while the scheduler admits, appends and retires -- and whose batch
kernel runs every (solve, tile) item through the tile emulator.  Every result must equal
the oracle bit for bit, and the admission rules (memory budget, slot limit, first come
first served, cancellation) must hold.
"""
import ctypes
import os
import subprocess
import sys
import time

import numpy as np
import pytest

import workloads as W
from paper_1705_03162_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HS = os.path.join(ROOT, "tests", "hostsim")
LIB = os.path.join(HS, "libservesim.so")


def _build():
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", "-pthread", "-Wno-unknown-pragmas", "-Wno-subobject-linkage",
                    "-I", os.path.join(HS, "fakehip"), "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_1705_03162_amd", "csrc"),
                    os.path.join(HS, "servesim.cpp"), "-o", LIB], check=True)


@pytest.fixture(scope="module")
def sim():
    if not os.path.exists(LIB):
        _build()
    L = ctypes.CDLL(LIB)
    for name in ("batch_create", "batch_submit", "batch_run", "batch_poll", "batch_wait",
                 "batch_cancel", "batch_ticket_info", "batch_destroy"):
        fn = getattr(L, name)
        fn.restype, fn.argtypes = N.SIGNATURES[name]
    L.servesim_ticks.restype = ctypes.c_int64
    L.servesim_ticks.argtypes = [ctypes.c_void_p]
    fn = L.batch_submit_async
    fn.restype, fn.argtypes = N.SIGNATURES["batch_submit_async"]
    L.servesim_stream_create.restype = ctypes.c_void_p
    L.servesim_stream_create.argtypes = []
    L.servesim_enqueue_copy.restype = None
    L.servesim_enqueue_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
    L.servesim_stream_destroy.restype = None
    L.servesim_stream_destroy.argtypes = [ctypes.c_void_p]
    return L


class SimBatch:
    """Host arrays stand in for device memory; the caller keeps them alive."""

    def __init__(self, L, budget, slots=0, serve=False, persistent=False, points_per_lane=0):
        self.L = L
        flags = (N.SW_BATCH_SERVE if serve else 0) | (N.SW_BATCH_PERSISTENT if persistent else 0)
        cfg = N.SwBatchConfig(int(budget), int(slots), flags, int(points_per_lane), 0)
        h = ctypes.c_void_p()
        assert L.batch_create(ctypes.byref(cfg), ctypes.byref(h)) == 0
        self.h = h
        self.keep = []

    def submit(self, prob, state):
        p = N.problem_struct(prob)
        t = ctypes.c_uint64()
        rc = self.L.batch_submit(self.h, ctypes.byref(p), state.ctypes.data, ctypes.byref(t))
        self.keep.append(p)
        assert rc == 0, rc
        return t.value

    def wait(self, t):
        assert self.L.batch_wait(self.h, t, 120_000_000) == 0

    def wait_all(self, tickets, states):
        """Wait for each ticket in turn and copy its state the moment it reports done:
        a finished solve's state must be final then, not only once the batch drains."""
        snaps = []
        for t, x in zip(tickets, states):
            self.wait(t)
            snaps.append(x.copy())
        return snaps

    def poll(self, t):
        s = ctypes.c_int32()
        assert self.L.batch_poll(self.h, t, ctypes.byref(s)) == 0
        return s.value

    def info(self, t):
        i = N.SwTicketInfo()
        assert self.L.batch_ticket_info(self.h, t, ctypes.byref(i)) == 0
        return {k: getattr(i, k) for k, _ in N.SwTicketInfo._fields_}

    def close(self):
        self.L.batch_destroy(self.h)


def mixed(count, seed, schemes=(W.HEAT, W.KS, W.EULER), nmax=512, smax=120, bcs=True):
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        scheme = schemes[int(rng.integers(0, len(schemes)))]
        n = 64 * int(rng.integers(1, nmax // 64 + 1))
        steps = int(rng.integers(1, smax))
        if scheme == W.EULER:
            prob, ic = W.sod_problem(n, steps), W.sod_ic(n)
        else:
            bc = int(rng.integers(0, 3 if scheme == W.HEAT else 2)) if bcs else W.PERIODIC
            if scheme == W.HEAT:
                prob = W.heat_problem(n, steps, bc=bc, bc_left=0.25, bc_right=-0.5)
            else:
                prob = W.ks_problem(n, steps, bc=bc)
                if bc == W.DIRICHLET:
                    prob = W.Problem(W.KS, n, steps, prob.dt, prob.dx, bc=bc, bc_left=(0.3, 0, 0),
                                     bc_right=(-0.1, 0, 0))
            ic = W.fourier_ic(n, seed=1000 + j)
        out.append((prob, np.ascontiguousarray(ic, dtype=np.float64)))
    return out


def nbytes(prob):
    """Device bytes the batch charges a swept solve: its state plus its edge slots
    (2 K slots of nvars x 2 rows x (w/2 + r) doubles) rounded up to 256 bytes, for the
    widest one-wave tile (at most 8 points per lane) that divides n."""
    P = 8
    while (prob.n // 64) % P:
        P //= 2
    w, r = 64 * P, (1 if prob.scheme == W.HEAT else 2)
    edges = 2 * (prob.n // w) * prob.nvars * 2 * (w // 2 + r) * 8
    return prob.n * prob.nvars * 8 + (edges + 255) // 256 * 256


def peak_resident(infos, sizes):
    ev = sorted([(i["start_s"], s) for i, s in zip(infos, sizes)] +
                [(i["end_s"], -s) for i, s in zip(infos, sizes)], key=lambda e: (e[0], e[1]))
    held = peak = 0
    for _, d in ev:
        held += d
        peak = max(peak, held)
    return peak


def test_ensemble_equals_oracle(sim, oracle_mod):
    """Ensemble mode (one captured graph per wave of admitted solves, each tile group's
    launches on a branch of its own): mixed schemes, sizes and boundaries, each result
    equal to the oracle; within a group a solve of more phases completes later (its
    stamp is a later one of the same branch) and solves of as many phases together."""
    probs = mixed(14, seed=21)
    states = [ic.copy() for _, ic in probs]
    b = SimBatch(sim, budget=1 << 30)
    tickets = [b.submit(p, x) for (p, _), x in zip(probs, states)]
    assert sim.batch_run(b.h, None) == 0
    infos = [b.info(t) for t in tickets]
    assert all(i["status"] == N.SW_TICKET_DONE for i in infos)
    assert all(i["end_s"] >= i["start_s"] for i in infos)
    groups = {}
    for (p, _), i in zip(probs, infos):
        if i["swept"]:
            groups.setdefault((p.scheme, i["width"]), []).append((i["phases"], i["end_s"]))
    assert any(len(v) > 1 for v in groups.values())
    for v in groups.values():
        v.sort()
        for (pa, ea), (pb, eb) in zip(v, v[1:]):
            assert eb > ea if pb > pa else eb == ea, v
    b.close()
    for (prob, ic), x in zip(probs, states):
        assert np.array_equal(x, oracle_mod.solve(prob, ic)), (prob.scheme, prob.n, prob.nsteps, prob.bc)


@pytest.mark.parametrize("ppl", [0, 2])
def test_ensemble_persistent_equals_oracle(sim, oracle_mod, ppl):
    """Persistent ensemble (one launch per tile group taking tiles from a queue in
    phase-major order and checking the tiles it depends on): mixed schemes, sizes and
    boundaries, default and forced tile shapes, each result equal to the oracle, and
    every solve's charged bytes as the library reports them."""
    probs = mixed(14, seed=24)
    states = [ic.copy() for _, ic in probs]
    b = SimBatch(sim, budget=1 << 30, persistent=True, points_per_lane=ppl)
    tickets = [b.submit(p, x) for (p, _), x in zip(probs, states)]
    assert sim.batch_run(b.h, None) == 0
    infos = [b.info(t) for t in tickets]
    assert all(i["status"] == N.SW_TICKET_DONE for i in infos)
    assert all(i["end_s"] >= i["start_s"] for i in infos)
    if ppl == 0:
        assert [i["resident_bytes"] for i in infos] == [nbytes(p) for p, _ in probs]
    b.close()
    for (prob, ic), x in zip(probs, states):
        assert np.array_equal(x, oracle_mod.solve(prob, ic)), (prob.scheme, prob.n, prob.nsteps, prob.bc)


def test_ensemble_budget_waves(sim, oracle_mod):
    """A budget of two solves: the ensemble runs in waves, results unchanged."""
    probs = mixed(8, seed=22, schemes=(W.HEAT, W.KS))
    states = [ic.copy() for _, ic in probs]
    b = SimBatch(sim, budget=2 * max(nbytes(p) for p, _ in probs), slots=2)
    tickets = [b.submit(p, x) for (p, _), x in zip(probs, states)]
    assert sim.batch_run(b.h, None) == 0
    assert all(b.poll(t) == N.SW_TICKET_DONE for t in tickets)
    b.close()
    for (prob, ic), x in zip(probs, states):
        assert np.array_equal(x, oracle_mod.solve(prob, ic))


def test_served_equals_oracle_under_budget(sim, oracle_mod):
    """Served mode with room for about three solves: admissions wait for retirements,
    the resident bytes never exceed the budget, every result equals the oracle."""
    probs = mixed(16, seed=23)
    sizes = [nbytes(p) for p, _ in probs]
    budget = 3 * max(sizes)
    states = [ic.copy() for _, ic in probs]
    b = SimBatch(sim, budget=budget, serve=True)
    tickets = [b.submit(p, x) for (p, _), x in zip(probs, states)]
    snaps = b.wait_all(tickets, states)
    infos = [b.info(t) for t in tickets]
    ticks = sim.servesim_ticks(b.h)
    b.close()
    assert all(i["status"] == N.SW_TICKET_DONE for i in infos)
    assert ticks > 0
    # the library charges each solve its state plus its rounded edge slots
    assert [i["resident_bytes"] for i in infos] == sizes
    assert max(sizes) < peak_resident(infos, sizes) <= budget
    for (prob, ic), x in zip(probs, snaps):
        assert np.array_equal(x, oracle_mod.solve(prob, ic)), (prob.scheme, prob.n, prob.nsteps, prob.bc)


def test_served_bursts_into_running_groups(sim, oracle_mod):
    """Solves of one group (heat, n a multiple of 512: eight points per lane) arrive in
    bursts while earlier ones tick: later solves are appended to a table that in-flight
    ticks still read, and finished solves are dropped once they fill half of it."""
    rng = np.random.default_rng(24)
    probs = [(W.heat_problem(512 * int(rng.integers(1, 3)), int(rng.integers(20, 400))),) for _ in range(18)]
    probs = [(p, np.ascontiguousarray(W.fourier_ic(p.n, 2000 + j))) for j, (p,) in enumerate(probs)]
    states = [ic.copy() for _, ic in probs]
    b = SimBatch(sim, budget=1 << 30, serve=True)
    tickets = []
    for burst in range(3):
        for (p, _), x in list(zip(probs, states))[6 * burst:6 * burst + 6]:
            tickets.append(b.submit(p, x))
        time.sleep(0.05)
    snaps = b.wait_all(tickets, states)
    infos = [b.info(t) for t in tickets]
    b.close()
    assert all(i["status"] == N.SW_TICKET_DONE and i["width"] == 512 for i in infos)
    for (prob, ic), x in zip(probs, snaps):
        assert np.array_equal(x, oracle_mod.solve(prob, ic))


def test_served_one_slot_is_first_come_first_served(sim, oracle_mod):
    """With one slot, solves run one after another in submission order."""
    probs = mixed(6, seed=25, schemes=(W.HEAT, W.KS), smax=60)
    states = [ic.copy() for _, ic in probs]
    b = SimBatch(sim, budget=1 << 30, slots=1, serve=True)
    tickets = [b.submit(p, x) for (p, _), x in zip(probs, states)]
    snaps = b.wait_all(tickets, states)
    infos = [b.info(t) for t in tickets]
    b.close()
    for prev, cur in zip(infos, infos[1:]):
        assert cur["start_s"] >= prev["end_s"]
    for (prob, ic), x in zip(probs, snaps):
        assert np.array_equal(x, oracle_mod.solve(prob, ic))


def test_served_cancel_while_queued(sim, oracle_mod):
    """A budget of one solve: a queued solve can be cancelled and stays untouched; the
    others complete."""
    probs = [(W.ks_problem(256, 300 + 50 * j), np.ascontiguousarray(W.fourier_ic(256, 3000 + j)))
             for j in range(3)]
    states = [ic.copy() for _, ic in probs]
    b = SimBatch(sim, budget=nbytes(probs[0][0]), serve=True)   # exactly one resident solve
    tickets = [b.submit(p, x) for (p, _), x in zip(probs, states)]
    assert sim.batch_cancel(b.h, tickets[2]) == 0
    snaps = b.wait_all(tickets[:2], states[:2])
    b.wait(tickets[2])
    status = [b.poll(t) for t in tickets]
    b.close()
    assert status == [N.SW_TICKET_DONE, N.SW_TICKET_DONE, N.SW_TICKET_CANCELLED]
    assert np.array_equal(states[2], probs[2][1])
    for (prob, ic), x in zip(probs[:2], snaps):
        assert np.array_equal(x, oracle_mod.solve(prob, ic))


def test_served_done_means_final(sim, oracle_mod):
    """Solves whose ticks take long on the emulator: when a ticket reports done, its
    state already holds the final level (not only after the batch drains)."""
    probs = [(W.ks_problem(4096, 150 + 20 * j), np.ascontiguousarray(W.fourier_ic(4096, 4000 + j)))
             for j in range(3)]
    states = [ic.copy() for _, ic in probs]
    b = SimBatch(sim, budget=1 << 30, serve=True)
    tickets = [b.submit(p, x) for (p, _), x in zip(probs, states)]
    snaps = b.wait_all(tickets, states)
    b.close()
    for (prob, ic), x in zip(probs, snaps):
        assert np.array_equal(x, oracle_mod.solve(prob, ic))


@pytest.mark.parametrize("serve", [False, True])
def test_async_submit_waits_for_the_submitting_stream(sim, oracle_mod, serve):
    """batch_submit_async: the initial state is still being written by work queued on the
    caller's stream (a copy that runs only when something waits for that stream); the
    batch's first launch for the solve waits for it, so every result equals the oracle.
    The same solves submitted with plain batch_submit start from the unwritten (zero)
    state, which shows the wait is what orders them."""
    probs = mixed(6, seed=31, schemes=(W.HEAT, W.KS))
    for use_async in (True, False):
        states = [np.zeros_like(ic) for _, ic in probs]
        stream = sim.servesim_stream_create()
        b = SimBatch(sim, budget=1 << 30, serve=serve)
        tickets = []
        for (p, ic), x in zip(probs, states):
            sim.servesim_enqueue_copy(stream, x.ctypes.data, ic.ctypes.data, ic.nbytes)
            s = N.problem_struct(p)
            t = ctypes.c_uint64()
            if use_async:
                assert sim.batch_submit_async(b.h, ctypes.byref(s), x.ctypes.data, stream, ctypes.byref(t)) == 0
            else:
                assert sim.batch_submit(b.h, ctypes.byref(s), x.ctypes.data, ctypes.byref(t)) == 0
            b.keep.append(s)
            tickets.append(t.value)
        if serve:
            snaps = b.wait_all(tickets, states)
        else:
            assert sim.batch_run(b.h, None) == 0
            snaps = [x.copy() for x in states]
        b.close()
        sim.servesim_stream_destroy(stream)
        same = [np.array_equal(x, oracle_mod.solve(p, ic)) for (p, ic), x in zip(probs, snaps)]
        assert all(same) if use_async else not any(same)


def test_batch_shape_from_the_tuning_table(tmp_path):
    """Batched tiles take the points per lane of the table's "batch" row for the size
    class (the most that divide n/64 up to it), else the most up to 8."""
    table = tmp_path / "tune.txt"
    table.write_text("batch 0 12 2\nbatch 1 12 4\nbatch 0 14 8\n")
    code = f"""
import ctypes, os, sys
sys.path.insert(0, {ROOT!r})
os.environ["SWEPT_TUNE_FILE"] = {str(table)!r}
import numpy as np
import workloads as W
from paper_1705_03162_amd import _native as N
L = ctypes.CDLL({LIB!r})
for name in ("batch_create", "batch_submit", "batch_ticket_info", "batch_destroy"):
    fn = getattr(L, name); fn.restype, fn.argtypes = N.SIGNATURES[name]
cfg = N.SwBatchConfig(1 << 30, 0, 0, 0, 0)
h = ctypes.c_void_p(); assert L.batch_create(ctypes.byref(cfg), ctypes.byref(h)) == 0
x = np.zeros(1 << 16)
out = []
for prob in (W.heat_problem(4096, 10), W.ks_problem(4096, 10), W.heat_problem(1 << 14, 10),
             W.heat_problem(8192, 10), W.ks_problem(3 * 64, 10), W.sod_problem(4096, 10)):
    p = N.problem_struct(prob); t = ctypes.c_uint64()
    assert L.batch_submit(h, ctypes.byref(p), x.ctypes.data, ctypes.byref(t)) == 0
    i = N.SwTicketInfo(); assert L.batch_ticket_info(h, t, ctypes.byref(i)) == 0
    out.append(i.width)
L.batch_destroy(h)
print(out)
"""
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    # heat 2^12 -> table 2; KS 2^12 -> 4; heat 2^14 -> 8; heat 2^13 -> nearest smaller class (12): 2;
    # KS n = 192 (n/64 = 3) -> 1 (the table's cap, but only 1 divides); Sod: no row -> most up to 8
    assert r.stdout.strip() == str([128, 256, 512, 128, 64, 512])
