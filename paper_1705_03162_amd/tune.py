"""Autotuner for the swept tile shape and the classic work-group size.

For each (scheme, floor(log2 n)) it times swept solves over every legal
(width, threads) pair that divides n, and classic solves over work-group sizes
64..1024, and writes the fastest to tune_gfx950.txt next to libswept.so;
swept_plan() reads that table whenever the caller does not fix a shape.  The
choice never changes results: the decomposition is bitwise identical for every
shape (the GPU tests check it).  The paper likewise takes the best time over
block sizes per grid size (Sec. 4.1, experimental method; Sec. 6).

    python -m paper_1705_03162_amd.tune [--schemes heat,ks,euler] [--log2n 12-20] [--what swept,classic]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tune_gfx950.txt")

POINTS_PER_LANE = (1, 2, 4, 8, 16)
WAVES = (1, 2, 4, 8, 16)


def legal(scheme: int, P: int, threads: int) -> bool:
    if scheme == 2 and P > 8:
        return False
    max_t = (256 if P >= 8 else 512) if scheme == 2 else (512 if P >= 8 else 1024)
    return threads <= max_t


def candidate_shapes(scheme: int, n: int):
    out = []
    for P in POINTS_PER_LANE:
        for nw in WAVES:
            t = 64 * nw
            w = P * t
            if legal(scheme, P, t) and n % w == 0:
                out.append((w, t))
    return out


def _problem(scheme: int, log2n: int, nsteps: int):
    import workloads as W
    n = 1 << log2n
    if scheme == W.HEAT:
        return W.heat_problem(n, nsteps), W.fourier_ic(n, seed=log2n)
    if scheme == W.KS:
        return W.ks_problem(n, nsteps), W.fourier_ic(n, seed=log2n)
    return W.sod_problem(n, nsteps), W.sod_ic(n)


def time_shape(sw, torch, prob, ic, width, threads, reps):
    with sw.Plan(prob, width=width, threads=threads) as plan:
        x0 = torch.tensor(ic, dtype=torch.float64, device="cuda")
        x = x0.clone()
        plan.swept(x)                # warm: graph capture
        best = float("inf")
        for _ in range(reps):
            x.copy_(x0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.swept(x)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
    return best


CLASSIC_THREADS = (64, 128, 256, 512, 1024)


def read_table(table: str = TABLE):
    """(swept rows {(scheme, lg): line}, classic rows {(scheme, lg): line}) of a table file."""
    swept, classic = {}, {}
    if os.path.exists(table):
        with open(table) as f:
            for line in f:
                parts = line.split()
                if not parts or parts[0].startswith("#"):
                    continue
                if parts[0] == "classic" and len(parts) >= 4:
                    classic[(int(parts[1]), int(parts[2]))] = line.rstrip("\n")
                elif parts[0] == "batch":
                    continue
                elif len(parts) >= 4:
                    swept[(int(parts[0]), int(parts[1]))] = line.rstrip("\n")
    return swept, classic


def write_table(swept, classic, table: str = TABLE, batch=None):
    batch = read_batch_rows(table) if batch is None else batch
    with open(table + ".tmp", "w") as f:
        f.write("# scheme log2n width threads  (point-updates/s, steps timed)\n")
        for k in sorted(swept):
            f.write(swept[k] + "\n")
        f.write("# classic scheme log2n threads  (point-updates/s, steps timed)\n")
        for k in sorted(classic):
            f.write(classic[k] + "\n")
        if batch:
            f.write("# batch scheme log2n points-per-lane  (point-updates/s, steps timed, solves)\n")
            for k in sorted(batch):
                f.write(batch[k] + "\n")
    os.replace(table + ".tmp", table)


def time_classic(sw, torch, prob, ic, threads, reps):
    with sw.Plan(prob, classic_threads=threads) as plan:
        x0 = torch.tensor(ic, dtype=torch.float64, device="cuda")
        x = x0.clone()
        plan.classic(x)              # warm: graph capture
        best = float("inf")
        for _ in range(reps):
            x.copy_(x0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.classic(x)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
    return best


BATCH_POINTS = (1, 2, 4, 8)


def time_batch(sw, torch, prob, ic, count, points, reps):
    """Best seconds of running `count` copies of one problem as a batched ensemble with
    one-wave tiles of `points` points per lane."""
    best = float("inf")
    x0 = torch.tensor(ic, dtype=torch.float64, device="cuda")
    for _ in range(reps + 1):   # the first run warms up
        xs = [x0.clone() for _ in range(count)]
        torch.cuda.synchronize()
        with sw.Batch(budget_bytes=64 << 30, points_per_lane=points) as b:
            for x in xs:
                b.submit(prob, x)
            t0 = time.perf_counter()
            b.run()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0) if _ else best
    return best


def tune_batch(schemes=(0, 1, 2), log2ns=range(8, 19), target_s: float = 0.05, reps: int = 2,
               table: str = TABLE, log=print):
    """Points per lane of batched one-wave tiles per (scheme, size class): ensembles of
    identical solves (enough to fill the GPU) timed for each legal shape, merged into the
    table as lines "batch scheme log2n points"."""
    import torch

    import paper_1705_03162_amd as sw
    swept, classic = read_table(table)
    batch = read_batch_rows(table)
    for scheme in schemes:
        for lg in log2ns:
            n = 1 << lg
            count = max(8, (1 << 22) // n)
            legal = [P for P in BATCH_POINTS if (n // 64) % P == 0 and (scheme != 2 or P <= 8)]
            prob, ic = _problem(scheme, lg, 64)
            t = time_batch(sw, torch, prob, ic, count, legal[-1], reps=1)
            steps = int(min(20_000, max(64, 64 * target_s / max(t, 1e-6))))
            prob, ic = _problem(scheme, lg, steps)
            res = sorted((time_batch(sw, torch, prob, ic, count, P, reps), P) for P in legal)
            t, P = res[0]
            rate = count * n * steps / t
            log(f"batch scheme={scheme} log2n={lg} x{count} steps={steps} best P={P} {rate:.3e} pt-upd/s; "
                + ", ".join(f"P={pp}: {count * n * steps / x:.3e}" for x, pp in sorted(res, key=lambda r: r[1])))
            batch[(scheme, lg)] = f"batch {scheme} {lg} {P}  # {rate:.4e} {steps} x{count}"
    write_table(swept, classic, table, batch)


def read_batch_rows(table: str = TABLE):
    rows = {}
    if os.path.exists(table):
        with open(table) as f:
            for line in f:
                parts = line.split()
                if len(parts) >= 4 and parts[0] == "batch":
                    rows[(int(parts[1]), int(parts[2]))] = line.rstrip("\n")
    return rows


def tune_classic(schemes=(0, 1, 2), log2ns=range(12, 21), target_s: float = 0.02, reps: int = 3,
                 table: str = TABLE, log=print):
    """Best classic work-group size per (scheme, size class), merged into the table."""
    import torch

    import paper_1705_03162_amd as sw
    swept, classic = read_table(table)
    for scheme in schemes:
        for lg in log2ns:
            n = 1 << lg
            prob, ic = _problem(scheme, lg, 256)
            t = time_classic(sw, torch, prob, ic, 256, reps=1)
            steps = int(min(20_000, max(256, 256 * target_s / max(t, 1e-6))))
            prob, ic = _problem(scheme, lg, steps)
            results = sorted((time_classic(sw, torch, prob, ic, T, reps), T) for T in CLASSIC_THREADS)
            t, T = results[0]
            rate = n * steps / t
            log(f"classic scheme={scheme} log2n={lg} steps={steps} best T={T} {rate:.3e} pt-upd/s; "
                + ", ".join(f"T={tt}: {n * steps / x:.3e}" for x, tt in sorted(results, key=lambda r: r[1])))
            classic[(scheme, lg)] = f"classic {scheme} {lg} {T}  # {rate:.4e} {steps}"
    write_table(swept, classic, table)


def tune(schemes=(0, 1, 2), log2ns=range(12, 21), target_s: float = 0.02, reps: int = 3,
         table: str = TABLE, log=print, verbose: bool = False):
    import torch

    import paper_1705_03162_amd as sw
    rows = []
    for scheme in schemes:
        for lg in log2ns:
            n = 1 << lg
            shapes = candidate_shapes(scheme, n)
            if not shapes:
                continue
            # choose a step count that takes ~target_s with the default shape
            steps = 200
            prob, ic = _problem(scheme, lg, steps)
            t = time_shape(sw, torch, prob, ic, *shapes[len(shapes) // 2], reps=1)
            steps = int(min(50_000, max(200, steps * target_s / max(t, 1e-6))))
            prob, ic = _problem(scheme, lg, steps)
            results = []
            for w, th in shapes:
                t = time_shape(sw, torch, prob, ic, w, th, reps)
                results.append((t, w, th))
            if verbose:
                for tt, ww, tth in results:
                    log(f"  shape w={ww} T={tth} P={ww // tth} waves={tth // 64}: "
                        f"{n * steps / tt:.3e} pt-upd/s")
            results.sort()
            t, w, th = results[0]
            rate = n * steps / t
            log(f"scheme={scheme} log2n={lg} steps={steps} best w={w} T={th} "
                f"{rate:.3e} pt-upd/s; worst {n * steps / results[-1][0]:.3e}")
            rows.append((scheme, lg, w, th, rate, steps))
    swept, classic = read_table(table)
    for scheme, lg, w, th, rate, steps in rows:
        swept[(scheme, lg)] = f"{scheme} {lg} {w} {th}  # {rate:.4e} {steps}"
    write_table(swept, classic, table)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--schemes", default="heat,ks,euler")
    ap.add_argument("--log2n", default="12-20")
    ap.add_argument("--table", default=TABLE)
    ap.add_argument("--target-ms", type=float, default=20.0)
    ap.add_argument("--verbose", action="store_true", help="log every shape timed")
    ap.add_argument("--what", default="swept,classic", help="comma list of swept, classic, batch")
    args = ap.parse_args()
    names = {"heat": 0, "ks": 1, "euler": 2}
    schemes = [names[s] for s in args.schemes.split(",")]
    a, b = (int(x) for x in args.log2n.split("-"))
    sys.path.insert(0, os.path.dirname(HERE))
    what = args.what.split(",")
    log = lambda m: print(m, flush=True)  # noqa: E731
    if "swept" in what:
        tune(schemes, range(a, b + 1), target_s=args.target_ms / 1000.0, table=args.table, log=log,
             verbose=args.verbose)
    if "classic" in what:
        tune_classic(schemes, range(a, b + 1), target_s=args.target_ms / 1000.0, table=args.table, log=log)
    if "batch" in what:
        tune_batch(schemes, range(max(a, 8), min(b, 18) + 1), table=args.table, log=log)


if __name__ == "__main__":
    main()
