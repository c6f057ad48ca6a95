#!/usr/bin/env python3
"""Benchmark: FP64 point-updates/s of the swept decomposition on one MI355X.

One step = one swept solve of the heat equation (FTCS) and one of the
Kuramoto-Sivashinsky equation (central differences + RK2), each on N = 2^20
periodic points for 50,000 timesteps, initial states resident in HBM.  value =
2 * N * 50,000 / (seconds per step).  The same line reports the classic
decomposition (one launch per sub-step; replayed HIP graphs and plain stream
launches), the live roofline figure of the dominant kernel (the swept Diamond
kernel, timed with HIP events on its own stream) and the CPU oracle timed on
the host's cores on a bounded sample.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

LOG2N = 20
NSTEPS = 50_000
METRIC = "FP64 point-updates/s (swept vs classic, 1 GPU) + batched p50/p99 solve latency"
PEAK_FP64_TFLOPS = 78.6   # MI355X published FP64 vector peak
N_SW_ENOTREADY = -6       # include/swept.h: ticket still running
PEAK_HBM_GBS = 8000.0
# Algorithmic FP64 operations per point per sub-step level: each add, subtract,
# multiply, divide and square root of the update as the paper writes it, each
# counted once, independent of how the kernel fuses or regroups them.  Heat (Eq.
# Heatdisc): 2 adds, 2 multiplies.  KS (Eq. KSDisc with the four-point terms in
# symmetric pairs, plus the RK stage): 16 in f, 2 in u + c f.  Euler (Appendix D,
# per cell and sub-step with each interface flux evaluated once): pressure 6,
# pressure ratio 3, interface flux 80 (reciprocal ratio and two reconstructions 21,
# two physical fluxes 22, Roe average 13, P_sp 5, spectral radius 4, flux 15),
# stage 9 = 98, of them 8 divisions and 4 square roots, each counted as one
# operation although gfx950 evaluates a binary64 division or root as a sequence.
FLOPS_PER_POINT_LEVEL = {W.HEAT: 4, W.KS: 18, W.EULER: 98}
SUBSTEPS = {W.HEAT: 1, W.KS: 2, W.EULER: 2}
# Algorithmic HBM bytes per point-update of the classic decomposition (state read
# and written once per sub-step: heat 8r+8w; KS predictor 8r+8w, final 16r+8w;
# Euler 3 variables over two sub-steps).
CLASSIC_BYTES_PER_UPDATE = {W.HEAT: 16, W.KS: 40, W.EULER: 120}

# Sources that determine the swept tile kernel's machine code, and the committed
# hardware-counter summary of its KS Diamond launch at N = 2^20.
KERNEL_SOURCES = ("paper_1705_03162_amd/csrc/swept_tile.hpp", "paper_1705_03162_amd/csrc/tiles_ks.hip",
                  "paper_1705_03162_amd/csrc/tile.hpp", "paper_1705_03162_amd/csrc/schemes.hpp",
                  "paper_1705_03162_amd/build.py")
TRAFFIC_SUMMARY = "profiles/swept_tile_ks_diamond_n2p20_pmc.txt"


def kernel_digest() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(width: int, threads: int):
    """HBM bytes per launch of the KS Diamond from the committed counter summary
    (lines '@key value'), or None when the kernel sources or the tile shape differ
    from those the counters were taken on."""
    try:
        with open(os.path.join(ROOT, TRAFFIC_SUMMARY)) as f:
            kv = dict(line[1:].split(None, 1) for line in f.read().splitlines()
                      if line.startswith("@") and len(line.split()) >= 2)
    except OSError:
        return None
    kv = {k: v.strip() for k, v in kv.items()}
    if kv.get("kernel_digest") != kernel_digest():
        return None
    if int(kv.get("width", -1)) != width or int(kv.get("threads", -1)) != threads:
        return None
    return float(kv["hbm_bytes_per_launch"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed_solves(plans, states, kind, reps, torch):
    """Mean seconds of `reps` rounds of solving every (plan, state) pair."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for plan, st in zip(plans, states):
            getattr(plan, kind)(st)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def cpu_baseline(budget_s: float = 12.0):
    import oracle
    oracle.build(force=False)
    cores = oracle.threads(0)
    n = 1 << LOG2N
    samples = []
    total_upd, total_s = 0, 0.0
    for scheme in (W.HEAT, W.KS):
        prob, ic = W.cfg_sweep(scheme, LOG2N)
        probe = 20 if scheme == W.HEAT else 10
        _, s = oracle.solve(prob.with_steps(probe), ic, timed=True)
        steps = max(probe, int((budget_s / 2) / max(s / probe, 1e-9)))
        steps = min(steps, NSTEPS)
        _, s = oracle.solve(prob.with_steps(steps), ic, timed=True)
        total_upd += n * steps
        total_s += s
        samples.append(f"{W.SCHEME_NAMES[scheme]} N=2^{LOG2N} x {steps} steps ({s:.1f} s)")
    return {"value": total_upd / total_s, "unit": "point-updates/s", "cores": cores,
            "kind": "oracle", "sample": "; ".join(samples) + f" of the {NSTEPS}-step workload"}


def rate_of(sw, torch, prob, ic, kind, flags=0, reps=2, width=0, threads=0, stat=min):
    """Point-updates/s of one solve (state resident, graph captured), from the best
    (or, with stat=np.median, the median) of `reps` timed runs after one warm run."""
    with sw.Plan(prob, width, threads, flags) as plan:
        x0 = torch.tensor(ic, dtype=torch.float64, device="cuda")
        x = x0.clone()
        getattr(plan, kind)(x)
        times = []
        for _ in range(reps):
            x.copy_(x0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            getattr(plan, kind)(x)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        best = float(stat(times))
        info = plan.info()
    return prob.n * prob.nsteps / best, best, info, x


def pct(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def batched_ensemble(sw, torch, members, ics, persistent):
    """One batch_run over every member (one graph launch), timed by the host clock;
    completion latency per solve from the library's device stamps."""
    upd = sum(m.problem.point_updates for m in members)
    states = [torch.tensor(ic, dtype=torch.float64, device="cuda") for ic in ics]
    torch.cuda.synchronize()
    with sw.Batch(budget_bytes=200 << 30, persistent=persistent) as b:
        tickets = [b.submit(m.problem, x) for m, x in zip(members, states)]
        t0 = time.perf_counter()
        b.run()
        torch.cuda.synchronize()
        makespan = time.perf_counter() - t0
        infos = [b.info(t) for t in tickets]
    start = min(i["start_s"] for i in infos)
    lat = [i["end_s"] - start for i in infos]
    return {"solves": len(members), "point_updates": upd, "seconds": makespan, "rate": upd / makespan,
            "p50_s": pct(lat, 50), "p99_s": pct(lat, 99)}, states


def ensemble_run(count=4096, nsteps=10_000, one_at_a_time_sample=512):
    """4096 independent heat/KS solves of uneven N: one batched graph launch (one launch
    per phase index, and the persistent variant with device-side dependency counters)
    vs the same solves one after another (each its own tuned plan), on the same GPU."""
    import torch
    import paper_1705_03162_amd as sw
    members = W.ensemble(count=count, nsteps=nsteps)
    ics = [W.ensemble_ic(m) for m in members]
    upd = sum(m.problem.point_updates for m in members)
    batched, out_l = batched_ensemble(sw, torch, members, ics, persistent=False)
    persist, out_p = batched_ensemble(sw, torch, members, ics, persistent=True)
    same = all(torch.equal(a, b) for a, b in zip(out_l, out_p))
    del out_l, out_p
    # one solve at a time: a seeded sample, extrapolated by point-updates
    rng = np.random.default_rng(7)
    idx = rng.choice(count, size=min(one_at_a_time_sample, count), replace=False)
    t_alone, upd_alone, lat_alone = 0.0, 0, []
    for j in idx:
        m = members[j]
        with sw.Plan(m.problem) as plan:
            x = torch.tensor(ics[j], dtype=torch.float64, device="cuda")
            plan.swept(x)                 # capture the graph outside the timing
            x.copy_(torch.tensor(ics[j], dtype=torch.float64, device="cuda"))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.swept(x)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        t_alone += dt
        upd_alone += m.problem.point_updates
        lat_alone.append(dt)
    alone_rate = upd_alone / t_alone
    # FIFO completion times if every solve ran alone, back to back from t = 0
    est = upd / alone_rate
    best = max(batched["rate"], persist["rate"])
    return {"batched": batched, "batched_persistent": persist, "persistent_equals_lockstep": bool(same),
            "faster": "persistent" if persist["rate"] > batched["rate"] else "lockstep",
            "one_at_a_time": {"sampled_solves": len(idx), "rate": alone_rate,
                              "estimated_seconds": est, "solve_p50_s": pct(lat_alone, 50),
                              "solve_p99_s": pct(lat_alone, 99)},
            "speedup": best / alone_rate}


# Shared-variant widths searched per scheme (two rows of nvars (w + 2 r) doubles within 160 KB)
LDS_WIDTHS = {W.HEAT: (256, 1024, 2048, 4096, 8192), W.KS: (256, 1024, 2048, 4096, 8192),
              W.EULER: (256, 1024, 2048)}


def legal_p(scheme):
    return (1, 2, 4, 8) if scheme == W.EULER else (1, 2, 4, 8, 16)


def search_shapes(sw, torch, prob, ic, shapes, flags=0):
    """Best (rate, width, threads) of the swept solve over the given tile shapes."""
    best = None
    for w, t in shapes:
        if prob.n % w:
            continue
        try:
            r, _, _, _ = rate_of(sw, torch, prob, ic, "swept", flags=flags, reps=1, width=w, threads=t)
        except sw.SweptError:
            continue
        if best is None or r > best[0]:
            best = (r, w, t)
    return best


def e2e_seconds(sw, torch, prob, ic, kind):
    """Paper-style end-to-end time: plan and device allocation, host-to-device copy of
    the initial state, the solve, device-to-host copy of the result."""
    host = np.ascontiguousarray(ic)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with sw.Plan(prob) as plan:
        x = torch.from_numpy(host).to("cuda")
        getattr(plan, kind)(x)
        out = x.cpu()
    dt = time.perf_counter() - t0
    del out
    return dt


def suite_sweep(schemes, log2ns, max_steps):
    """One JSON line per (scheme, N): the tuned swept solve (median of 5), the best
    one-wave "register" tile, the best one-point-per-thread tile (w = T, the paper's
    layout), classic through replayed graphs and through stream launches, the
    end-to-end times of both, and the swept rate against the classic HBM roofline and
    the FP64 VALU ceiling."""
    import torch
    import paper_1705_03162_amd as sw
    for scheme in schemes:
        for lg in log2ns:
            if scheme == W.EULER:
                prob, ic = W.cfg_sod(lg)
            else:
                prob, ic = W.cfg_sweep(scheme, lg)
            full = prob.nsteps
            prob = prob.with_steps(min(full, max_steps))
            rs, ts, info, xs = rate_of(sw, torch, prob, ic, "swept", reps=5, stat=np.median)
            rg, tg, _, xg = rate_of(sw, torch, prob, ic, "classic", reps=3, stat=np.median)
            rst, tst, _, _ = rate_of(sw, torch, prob, ic, "classic", flags=sw.SW_TUNE_NO_GRAPH, reps=1)
            same = bool(torch.equal(xs, xg))
            reg = search_shapes(sw, torch, prob, ic, [(64 * p, 64) for p in legal_p(scheme)])
            p1 = search_shapes(sw, torch, prob, ic, [(t, t) for t in (64, 128, 256, 512, 1024)])
            # the Shared variant (rows in LDS), up to the widest tile 160 KB of LDS holds
            lds = search_shapes(sw, torch, prob, ic, [(w, t) for w in LDS_WIDTHS[scheme] for t in (256, 1024)
                                                      if w % t == 0], flags=sw.SW_TUNE_LDS)
            e2e_s = e2e_seconds(sw, torch, prob, ic, "swept")
            e2e_c = e2e_seconds(sw, torch, prob, ic, "classic")
            upd = prob.n * prob.nsteps
            roof = PEAK_HBM_GBS * 1e9 / CLASSIC_BYTES_PER_UPDATE[scheme]
            line = {"scheme": W.SCHEME_NAMES[scheme], "n": prob.n, "steps": prob.nsteps,
                    "full_steps": full, "swept": rs, "classic_graph": rg, "classic_stream": rst,
                    "swept_over_classic_graph": rs / rg, "swept_over_classic_stream": rs / rst,
                    "swept_ms": ts * 1e3, "classic_graph_ms": tg * 1e3,
                    "width": info["width"], "threads": info["threads"], "bitwise_equal": same,
                    "register_best": None if reg is None else {"rate": reg[0], "width": reg[1], "threads": reg[2]},
                    "one_point_per_thread_best": None if p1 is None else {"rate": p1[0], "width": p1[1], "threads": p1[2]},
                    "lds_best": None if lds is None else {"rate": lds[0], "width": lds[1], "threads": lds[2]},
                    "e2e_swept": upd / e2e_s, "e2e_classic": upd / e2e_c,
                    "classic_hbm_roofline": roof, "swept_over_classic_roofline": rs / roof}
            if scheme in FLOPS_PER_POINT_LEVEL:
                ops = rs * FLOPS_PER_POINT_LEVEL[scheme] * SUBSTEPS[scheme]
                line["swept_fp64_tflops"] = ops / 1e12
                line["swept_frac_fp64_peak"] = ops / (PEAK_FP64_TFLOPS * 1e12)
            print(json.dumps(line), flush=True)
            log(f"{W.SCHEME_NAMES[scheme]} 2^{lg}: swept {rs:.3e} classic graph {rg:.3e} "
                f"stream {rst:.3e} e2e swept {upd / e2e_s:.3e}")


def suite_hybrid(log2ns=range(12, 21), max_steps=20_000):
    """Hybrid variant (the host CPU computes the straddling tile of every shifted phase)
    against the all-GPU swept solve on the same tile shape: the paper's insulated heat
    case (50,000 steps) and the Sod tube (to t = 0.2, at most max_steps steps), one JSON
    line per (scheme, N), median of 3 timed solves each; results compared bit for bit."""
    import torch
    import paper_1705_03162_amd as sw
    for scheme in (W.HEAT, W.EULER):
        for lg in log2ns:
            n = 1 << lg
            if scheme == W.HEAT:
                prob, ic = W.heat_problem(n, 50_000, bc=W.REFLECTIVE), W.fourier_ic(n, seed=2 + lg)
            else:
                prob, ic = W.cfg_sod(lg)
                prob = prob.with_steps(min(prob.nsteps, max_steps))
            rs, ts, info, xs = rate_of(sw, torch, prob, ic, "swept", reps=3, stat=np.median)
            w, t = info["width"], info["threads"]
            rh, th, _, xh = rate_of(sw, torch, prob, ic, "swept", flags=sw.SW_TUNE_HYBRID, reps=3,
                                    width=w, threads=t, stat=np.median)
            line = {"suite": "hybrid", "scheme": W.SCHEME_NAMES[scheme], "bc": prob.bc, "n": n,
                    "steps": prob.nsteps, "width": w, "threads": t, "shared": rs, "hybrid": rh,
                    "hybrid_over_shared": rh / rs, "shared_ms": ts * 1e3, "hybrid_ms": th * 1e3,
                    "bitwise_equal": bool(torch.equal(xs, xh))}
            print(json.dumps(line), flush=True)
            log(f"hybrid {W.SCHEME_NAMES[scheme]} 2^{lg}: shared {rs:.3e} hybrid {rh:.3e} ({rh / rs:.2f}x)")


def suite_euler_full(log2n=20):
    """Sod at N = 2^20 for the whole run to t = 0.2 (about 1.15M steps), swept and
    classic: times, and whether the two final states are bit-identical."""
    import torch
    import paper_1705_03162_amd as sw
    prob, ic = W.cfg_sod(log2n)
    x0 = torch.tensor(ic, dtype=torch.float64, device="cuda")
    out = {"suite": "euler-full", "n": prob.n, "steps": prob.nsteps}
    res = {}
    for kind in ("swept", "classic"):
        with sw.Plan(prob) as plan:
            x = x0.clone()
            torch.cuda.synchronize()
            log(f"sod 2^{log2n} full length, {kind} ...")
            t0 = time.perf_counter()
            getattr(plan, kind)(x)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if kind == "swept":
                out["width"], out["threads"] = plan.info()["width"], plan.info()["threads"]
        res[kind] = x
        out[f"{kind}_s"] = dt
        out[kind] = prob.n * prob.nsteps / dt
        log(f"  {kind}: {dt:.1f} s, {out[kind]:.3e} point-updates/s")
    out["bitwise_equal"] = bool(torch.equal(res["swept"], res["classic"]))
    out["swept_over_classic"] = out["swept"] / out["classic"]
    rho = res["swept"][0]
    out["min_density"] = float(rho.min())
    print(json.dumps(out), flush=True)


def device_fourier_ic(torch, n, seed, kmax=16):
    """Smooth periodic field built on the device (same modes as the host generator,
    for sizes where evaluating it on the host would dominate the run)."""
    rng = np.random.default_rng(seed)
    kmax = max(1, min(kmax, n // 8)) if n >= 8 else 1
    a = rng.uniform(-1.0, 1.0, kmax)
    b = rng.uniform(-1.0, 1.0, kmax)
    i = torch.arange(n, dtype=torch.float64, device="cuda")
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    for k in range(kmax):
        th = i * (2.0 * math.pi * (k + 1) / n)
        x += float(a[k]) * torch.cos(th) + float(b[k]) * torch.sin(th)
    return x.reshape(1, n)


def device_ic(torch, prob, seed):
    if prob.scheme == W.EULER:
        return torch.tensor(W.sod_ic(prob.n), dtype=torch.float64, device="cuda")
    return device_fourier_ic(torch, prob.n, seed)


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Achievable HBM bandwidth: a plain device copy of `nbytes` (read + write)."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    return 2 * nbytes / dt / 1e9


def suite_anchors(steps=200):
    """Out-of-cache anchors: classic and swept at sizes whose state exceeds the
    on-chip caches (heat, KS at 2^26; Euler at 2^24), against a plain copy."""
    import torch
    import paper_1705_03162_amd as sw
    bw = copy_bandwidth(torch)
    print(json.dumps({"anchor": "copy", "bytes": 1 << 30, "gb_per_s": bw,
                      "frac_of_peak": bw / PEAK_HBM_GBS}), flush=True)
    for scheme, lg in ((W.HEAT, 26), (W.KS, 26), (W.EULER, 24)):
        n = 1 << lg
        prob = {W.HEAT: W.heat_problem, W.KS: W.ks_problem}[scheme](n, steps) if scheme != W.EULER \
            else W.sod_problem(n, steps // 2)
        x0 = device_ic(torch, prob, seed=lg)
        out = {"anchor": W.SCHEME_NAMES[scheme], "n": n, "steps": prob.nsteps}
        for kind, flags in (("classic", 0), ("swept", 0)):
            with sw.Plan(prob, flags=flags) as plan:
                x = x0.clone()
                getattr(plan, kind)(x)
                x.copy_(x0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                getattr(plan, kind)(x)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                out[kind] = n * prob.nsteps / dt
                if kind == "swept":
                    out["width"], out["threads"] = plan.info()["width"], plan.info()["threads"]
        gbs = out["classic"] * CLASSIC_BYTES_PER_UPDATE[scheme] / 1e9
        out.update({"classic_algorithmic_gb_per_s": gbs, "classic_frac_of_copy": gbs / bw,
                    "classic_frac_of_peak_hbm": gbs / PEAK_HBM_GBS,
                    "swept_over_classic": out["swept"] / out["classic"]})
        print(json.dumps(out), flush=True)
        log(f"anchor {W.SCHEME_NAMES[scheme]} 2^{lg}: classic {out['classic']:.3e} ({gbs:.0f} GB/s) "
            f"swept {out['swept']:.3e}")
        del x0


def served(torch, sw, trace, warmup_s=0.0, max_slots=0):
    """Feed a Poisson trace into a served batch in real time; latency = completion -
    submission, over requests that arrived after the warm-up."""
    states = [device_ic(torch, r.problem, r.ic_seed) for r in trace]
    torch.cuda.synchronize()
    upd = sum(r.problem.point_updates for r in trace)
    with sw.Batch(budget_bytes=200 << 30, max_slots=max_slots, serve=True) as b:
        t0 = time.perf_counter()
        tickets = []
        for j, (r, x) in enumerate(zip(trace, states)):
            delay = r.arrival_s - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets.append(b.submit(r.problem, x))
            if (j + 1) % 2000 == 0:
                log(f"  submitted {j + 1}/{len(trace)} at {time.perf_counter() - t0:.1f} s")
        for j, t in enumerate(tickets):
            while True:   # bounded waits, so a long drain still reports progress
                try:
                    b.wait(t, 20_000_000)
                    break
                except sw.SweptError as e:
                    if e.status != N_SW_ENOTREADY:
                        raise
                    log(f"  waiting for request {j} at {time.perf_counter() - t0:.1f} s")
            if (j + 1) % 2000 == 0:
                log(f"  completed {j + 1}/{len(trace)} at {time.perf_counter() - t0:.1f} s")
        wall = time.perf_counter() - t0
        infos = [b.info(t) for t in tickets]
    keep = [(r, i) for r, i in zip(trace, infos) if r.arrival_s >= warmup_s]
    lat = [i["end_s"] - i["submit_s"] for _, i in keep]
    window = max(r.arrival_s for r in trace) - warmup_s if keep else 0.0
    thirds = []
    if keep:
        span = max(r.arrival_s for r, _ in keep) - warmup_s
        for q in range(3):
            lo, hi = warmup_s + span * q / 3, warmup_s + span * (q + 1) / 3
            sel = [i["end_s"] - i["submit_s"] for r, i in keep if lo <= r.arrival_s <= hi]
            thirds.append(float(np.mean(sel)) if sel else None)
    return {"requests": len(keep), "point_updates": upd, "wall_s": wall,
            "throughput_point_updates_s": upd / wall, "p50_latency_s": pct(lat, 50),
            "p99_latency_s": pct(lat, 99), "mean_latency_by_arrival_third_s": thirds,
            "arrival_window_s": window}


def serve_configured(rate=2000.0, duration_s=10.0, warmup_s=1.0, fifo_prefix=300,
                     rates=(100.0, 150.0, 200.0, 250.0, 300.0, 400.0), window=5.0, emit=None):
    """The configured serving run (Poisson arrivals at `rate` for `duration_s` after
    `warmup_s`, then drain), the highest rate with a stable queue, and one solve at a
    time, first come first served, on a prefix of the configured trace.  Returns one
    dict; `emit`, if given, receives each partial result as it is measured."""
    import torch
    import paper_1705_03162_amd as sw
    emit = emit or (lambda d: None)
    trace = W.poisson_trace(rate=rate, duration_s=warmup_s + duration_s, seed=5)
    log(f"serve: configured {rate}/s, {len(trace)} requests ...")
    conf = served(torch, sw, trace, warmup_s=warmup_s)
    conf.update({"run": "configured", "offered_rate_per_s": rate, "warmup_s": warmup_s})
    emit(conf)

    # sustainable rate: ascending offered rates on short traces.  With a budget this
    # large every request is resident at once, so an overloaded server shows up as
    # a long drain after the last arrival, not as a queue: a rate is sustainable
    # when the drain takes at most max(2 s, half the window).
    stable, searched = None, []
    for r in rates:
        tr = W.poisson_trace(rate=r, duration_s=window, seed=6)
        x = served(torch, sw, tr)
        drain = x["wall_s"] - max(q.arrival_s for q in tr)
        x["drain_s"] = drain
        ok = drain <= max(2.0, 0.5 * window)
        x.update({"run": "rate_search", "offered_rate_per_s": r, "stable": ok})
        searched.append({"rate_per_s": r, "stable": ok, "drain_s": drain, "p50_latency_s": x["p50_latency_s"],
                         "p99_latency_s": x["p99_latency_s"]})
        emit(x)
        log(f"serve rate {r}/s: stable={ok} p50 {x['p50_latency_s']:.3f} s p99 {x['p99_latency_s']:.3f} s")
        if not ok:
            break
        stable = x
    sustainable = {"rate_per_s": None if stable is None else stable["offered_rate_per_s"],
                   "p50_latency_s": None if stable is None else stable["p50_latency_s"],
                   "p99_latency_s": None if stable is None else stable["p99_latency_s"],
                   "throughput_point_updates_s": None if stable is None else stable["throughput_point_updates_s"],
                   "window_s": window, "searched": searched}

    # one solve at a time, FIFO, on the configured trace's first requests
    pre = trace[:fifo_prefix]
    lat = []
    upd = sum(r.problem.point_updates for r in pre)
    t0 = time.perf_counter()
    for r in pre:
        now = time.perf_counter() - t0
        if now < r.arrival_s:
            time.sleep(r.arrival_s - now)
        x = device_ic(torch, r.problem, r.ic_seed)
        with sw.Plan(r.problem, flags=sw.SW_TUNE_NO_GRAPH) as plan:
            if plan.info()["swept_ok"]:
                plan.swept(x)
            else:
                plan.classic(x)
            torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0 - r.arrival_s)
    wall = time.perf_counter() - t0
    fifo = {"run": "fifo_one_at_a_time", "requests": len(pre), "offered_rate_per_s": rate,
            "wall_s": wall, "throughput_point_updates_s": upd / wall,
            "p50_latency_s": pct(lat, 50), "p99_latency_s": pct(lat, 99)}
    emit(fifo)
    # the same prefix through the served batch, for a like-for-like comparison
    pre_served = served(torch, sw, pre)
    return {"configured": conf, "sustainable": sustainable, "fifo_prefix_one_at_a_time": fifo,
            "fifo_prefix_served": {"requests": pre_served["requests"], "wall_s": pre_served["wall_s"],
                                   "throughput_point_updates_s": pre_served["throughput_point_updates_s"],
                                   "p50_latency_s": pre_served["p50_latency_s"],
                                   "p99_latency_s": pre_served["p99_latency_s"]}}


def suite_serve(rate=2000.0, duration_s=10.0, warmup_s=1.0, fifo_prefix=300):
    """One JSON line per serving measurement (see serve_configured), then a summary."""
    res = serve_configured(rate, duration_s, warmup_s, fifo_prefix, emit=lambda d: print(json.dumps(d), flush=True))
    print(json.dumps({"run": "summary", "sustainable": res["sustainable"],
                      "fifo_prefix_served": res["fifo_prefix_served"]}), flush=True)


def suite_oracle(budget_s=6.0):
    """The CPU oracle on all host cores and on one core, bounded samples."""
    import oracle
    oracle.build(force=False)
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    for scheme, lg in ((W.HEAT, 20), (W.KS, 20), (W.EULER, 18)):
        prob, ic = (W.cfg_sod(lg) if scheme == W.EULER else W.cfg_sweep(scheme, lg))
        for nth in (0, 1):
            probe = 4
            _, s = oracle.solve(prob.with_steps(probe), ic, nthreads=nth, timed=True)
            steps = max(probe, min(prob.nsteps, int(budget_s / max(s / probe, 1e-9))))
            _, s = oracle.solve(prob.with_steps(steps), ic, nthreads=nth, timed=True)
            print(json.dumps({"oracle": W.SCHEME_NAMES[scheme], "n": prob.n, "steps": steps,
                              "threads": oracle.threads(nth), "affinity_cpus": affinity,
                              "cpu_model": model, "seconds": s,
                              "point_updates_s": prob.n * steps / s}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the ensemble and serving runs")
    ap.add_argument("--profile-reps", type=int, default=30)
    ap.add_argument("--serve-window", type=float, default=10.0,
                    help="arrival window (s, after a 1 s warm-up) of the configured serving run")
    ap.add_argument("--suite", default="main",
                    choices=["main", "sweep", "euler", "euler-full", "ensemble", "serve", "kernel",
                             "classic-kernel", "anchors", "oracle", "hybrid"],
                    help="main: the one-line benchmark; sweep/euler: per-N swept vs classic lines; "
                         "anchors: out-of-cache sizes and a copy; serve: configured and sustainable "
                         "serving; oracle: CPU oracle on all cores and one; kernel, classic-kernel: counter runs")
    ap.add_argument("--max-steps", type=int, default=50_000)
    ap.add_argument("--kernel-scheme", default="ks", choices=["ks", "heat", "euler"],
                    help="kernel suite: scheme of the profiled Diamond (N = 2^20; euler: the Sod tube)")
    ap.add_argument("--kernel-width", type=int, default=0, help="kernel suite: tile width (0 = tuned)")
    ap.add_argument("--kernel-threads", type=int, default=0, help="kernel suite: work-group size (0 = tuned)")
    ap.add_argument("--kernel-lds", action="store_true",
                    help="kernel suite: the Shared variant (rows in LDS; give --kernel-width/--kernel-threads)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the multi-GPU "
              "decomposition is not implemented.", file=sys.stderr)
        sys.exit(2)
    if args.suite == "kernel":
        # for hardware-counter runs: a known-size device copy (calibrates FETCH/WRITE)
        # and a few launches of the dominant kernel (KS Diamond at N = 2^20)
        if args.kernel_lds and (args.kernel_width <= 0 or args.kernel_threads <= 0):
            print("--kernel-lds needs --kernel-width and --kernel-threads", file=sys.stderr)
            sys.exit(2)
        import torch
        import paper_1705_03162_amd as sw
        src = torch.ones(1 << 25, dtype=torch.float64, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        if args.kernel_scheme == "euler":
            prob, ic = W.cfg_sod(LOG2N, nsteps=2000)
        else:
            prob, ic = W.cfg_sweep({"ks": W.KS, "heat": W.HEAT}[args.kernel_scheme], LOG2N)
        flags = sw.SW_TUNE_LDS if args.kernel_lds else 0
        with sw.Plan(prob, args.kernel_width, args.kernel_threads, flags=flags) as plan:
            x = torch.tensor(ic, dtype=torch.float64, device="cuda")
            if args.kernel_scheme == "euler":
                plan.swept(x)   # the Diamonds then read edges of a developed Sod state
            us = plan.profile_phase(x, kind=1, reps=args.profile_reps)
            info = plan.info()
        flops = prob.n * info["levels_per_phase"] * FLOPS_PER_POINT_LEVEL[prob.scheme]
        print(json.dumps({"copy_bytes": 2 * src.numel() * 8, "diamond_avg_us": us, "scheme": args.kernel_scheme,
                          "variant": "lds" if args.kernel_lds else "register",
                          "width": info["width"], "threads": info["threads"],
                          "levels_per_phase": info["levels_per_phase"], "n": prob.n,
                          "flops_per_launch": flops, "tflops": flops / (us * 1e-6) / 1e12,
                          "frac_fp64_peak": flops / (us * 1e-6) / 1e12 / PEAK_FP64_TFLOPS,
                          "kernel_digest": kernel_digest()}), flush=True)
        return
    if args.suite == "classic-kernel":
        # for hardware-counter runs of the classic kernel: a known-size device copy, then
        # classic solves at an out-of-cache size with one launch per sub-step
        import torch
        import paper_1705_03162_amd as sw
        src = torch.ones(1 << 25, dtype=torch.float64, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        n, steps = 1 << 26, 20
        for scheme in (W.HEAT, W.KS):
            prob = (W.heat_problem if scheme == W.HEAT else W.ks_problem)(n, steps)
            x = device_ic(torch, prob, seed=26)
            with sw.Plan(prob, flags=sw.SW_TUNE_NO_GRAPH) as plan:
                plan.classic(x)
            torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 2 * src.numel() * 8, "n": n, "steps": steps}), flush=True)
        return
    if args.suite == "euler-full":
        suite_euler_full()
        return
    if args.suite == "hybrid":
        suite_hybrid(max_steps=args.max_steps)
        return
    if args.suite == "anchors":
        suite_anchors()
        return
    if args.suite == "oracle":
        suite_oracle()
        return
    if args.suite == "ensemble":
        print(json.dumps(ensemble_run()), flush=True)
        return
    if args.suite == "serve":
        suite_serve()
        return
    if args.suite != "main":
        if args.suite == "euler":
            suite_sweep([W.EULER], range(12, 21), args.max_steps)
        else:
            suite_sweep([W.HEAT, W.KS], range(12, 21, 2), args.max_steps)
        return

    import torch
    import paper_1705_03162_amd as sw

    dev = torch.device("cuda:0")
    n = 1 << LOG2N
    probs, ics = [], []
    for scheme in (W.HEAT, W.KS):
        p, ic = W.cfg_sweep(scheme, LOG2N, NSTEPS)
        probs.append(p)
        ics.append(ic)
    plans = [sw.Plan(p) for p in probs]
    infos = [pl.info() for pl in plans]
    for p, i in zip(probs, infos):
        log(f"plan {W.SCHEME_NAMES[p.scheme]}: w={i['width']} T={i['threads']} P={i['points_per_lane']} "
            f"H={i['levels_per_phase']} Q={i['full_phases']} rem={i['remainder']} "
            f"launches swept={i['swept_launches']} classic={i['classic_launches']}")
    fresh = lambda ic: torch.tensor(ic, dtype=torch.float64, device=dev)
    states = [fresh(ic) for ic in ics]

    # ---- swept: warmup + timed steps (each step starts again from the initial state,
    # copied device-to-device outside the timed region)
    init = [fresh(ic) for ic in ics]
    for _ in range(args.warmup):
        for st, i0 in zip(states, init):
            st.copy_(i0)
        timed_solves(plans, states, "swept", 1, torch)
    step_times = []
    for _ in range(args.steps):
        for st, i0 in zip(states, init):
            st.copy_(i0)
        torch.cuda.synchronize()
        step_times.append(timed_solves(plans, states, "swept", 1, torch))
    swept_out = [st.cpu().numpy() for st in states]
    t_step = float(np.mean(step_times))
    updates = 2 * n * NSTEPS
    value = updates / t_step
    log(f"swept: {t_step * 1e3:.2f} ms/step -> {value:.3e} point-updates/s")

    # per-scheme swept rates (one solve each)
    per_scheme = {}
    for p, pl, st, i0 in zip(probs, plans, states, init):
        st.copy_(i0)
        s = timed_solves([pl], [st], "swept", 1, torch)
        per_scheme[W.SCHEME_NAMES[p.scheme]] = {"swept_s": s, "swept": n * NSTEPS / s}

    # ---- classic: graph replays and stream launches
    classic = {}
    for flags, label in ((0, "graph"), (sw.SW_TUNE_NO_GRAPH, "stream")):
        cp = [sw.Plan(p, flags=flags) for p in probs]
        tot = 0.0
        outs = []
        for p, pl, i0 in zip(probs, cp, init):
            st = i0.clone()
            pl.classic(st)            # warm (graph capture)
            st.copy_(i0)
            s = timed_solves([pl], [st], "classic", 1, torch)
            tot += s
            outs.append(st.cpu().numpy())
            per_scheme[W.SCHEME_NAMES[p.scheme]][f"classic_{label}"] = n * NSTEPS / s
        classic[label] = updates / tot
        if label == "graph":
            bitwise = all(np.array_equal(a, b) for a, b in zip(swept_out, outs))
        for pl in cp:
            pl.close()
        log(f"classic ({label}): {tot * 1e3:.2f} ms/step -> {classic[label]:.3e} point-updates/s")

    # ---- roofline of the dominant kernel (swept Diamond), timed with HIP events
    kern = []
    for p, pl, i0, info in zip(probs, plans, init, infos):
        scratch = i0.clone()
        pl.swept(scratch)
        us = pl.profile_phase(scratch, kind=1, reps=args.profile_reps)
        launches = info["swept_launches"] - 3
        flops = n * info["levels_per_phase"] * FLOPS_PER_POINT_LEVEL[p.scheme]
        # edge slots read and written by a Diamond: per tile 2 slots x nv x 2 rows x E doubles each way
        edge_bytes = 2 * info["nodes"] * 2 * info["nvars"] * 2 * (info["width"] // 2 + info["radius"]) * 8
        kern.append({"scheme": W.SCHEME_NAMES[p.scheme], "avg_us": us, "flops_per_launch": flops,
                     "launches_per_solve": launches, "share_s": us * 1e-6 * launches,
                     "edge_bytes": edge_bytes, "width": info["width"], "threads": info["threads"]})
        log(f"diamond {W.SCHEME_NAMES[p.scheme]}: {us:.1f} us/launch, {flops / us * 1e-6:.2f} TFLOP/s")
    dom = max(kern, key=lambda k: k["share_s"])
    achieved = dom["flops_per_launch"] / (dom["avg_us"] * 1e-6) / 1e12
    traffic = measured_traffic(dom["width"], dom["threads"]) if dom["scheme"] == "ks" else None
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                "kernel": f"swept_tile<{dom['scheme']}> diamond", "avg_us": dom["avg_us"],
                "flops_per_launch": dom["flops_per_launch"],
                "algorithmic_bytes_per_launch": dom["edge_bytes"],
                "traffic_source": TRAFFIC_SUMMARY if traffic is not None else None,
                "kernel_digest": kernel_digest()}

    # ---- the paper's insulated heat case with end-to-end times (plan, allocation, copies in
    # and out), and the Euler/Sod verdict, swept against classic at the same size
    log("insulated heat and Sod at 2^20 ...")
    extra = {}
    hp = W.heat_problem(n, NSTEPS, bc=W.REFLECTIVE)
    hic = W.fourier_ic(n, seed=2 + LOG2N)
    rs, _, _, _ = rate_of(sw, torch, hp, hic, "swept", reps=2)
    rc, _, _, _ = rate_of(sw, torch, hp, hic, "classic", reps=1)
    upd_h = hp.n * hp.nsteps
    extra["heat_insulated"] = {"n": hp.n, "steps": hp.nsteps, "swept": rs, "classic_graph": rc,
                               "swept_e2e": upd_h / e2e_seconds(sw, torch, hp, hic, "swept"),
                               "classic_e2e": upd_h / e2e_seconds(sw, torch, hp, hic, "classic")}
    sp, sic = W.cfg_sod(LOG2N, nsteps=20_000)
    rs, _, _, xs = rate_of(sw, torch, sp, sic, "swept", reps=1)
    rc, _, _, xc = rate_of(sw, torch, sp, sic, "classic", reps=1)
    extra["sod"] = {"n": sp.n, "steps": sp.nsteps, "swept": rs, "classic_graph": rc,
                    "swept_over_classic": rs / rc, "bitwise_equal": bool(torch.equal(xs, xc)),
                    "verdict": "swept faster" if rs > rc else "classic faster"}

    result = {
        "metric": METRIC, "value": value, "unit": "point-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_step * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"heat FTCS + Kuramoto-Sivashinsky RK2, periodic, N=2^{LOG2N}, "
                               f"{NSTEPS} steps each, one swept solve per scheme per step",
                   "n": n, "nsteps": NSTEPS,
                   "tiles": {W.SCHEME_NAMES[p.scheme]: {"width": i["width"], "threads": i["threads"]}
                             for p, i in zip(probs, infos)}},
        "classic": {"graph": classic["graph"], "stream": classic["stream"],
                    "speedup_swept_vs_graph": value / classic["graph"],
                    "speedup_swept_vs_stream": value / classic["stream"]},
        "per_scheme": per_scheme,
        "swept_equals_classic_bitwise": bool(bitwise),
        "roofline": roofline,
        "variants": extra,
    }
    for pl in plans:
        pl.close()
    if not args.no_batch:
        log("ensemble (4096 solves) ...")
        result["batch"] = {"ensemble": ensemble_run()}
        log("served Poisson traces (configured 2000/s for 10 s after 1 s, sustainable rate, FIFO) ...")
        result["batch"]["serve"] = serve_configured(duration_s=args.serve_window)
        e = result["batch"]["ensemble"]
        log(f"ensemble: batched {e['batched']['rate']:.3e} pt-upd/s in {e['batched']['seconds']:.2f} s "
            f"(persistent {e['batched_persistent']['rate']:.3e} in {e['batched_persistent']['seconds']:.2f} s), "
            f"one-at-a-time {e['one_at_a_time']['rate']:.3e}; serve p50 "
            f"{result['batch']['serve']['configured']['p50_latency_s']:.3f} s p99 "
            f"{result['batch']['serve']['configured']['p99_latency_s']:.3f} s")
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
