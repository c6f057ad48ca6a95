"""Write the oracle's results at the benchmark configurations' full sizes.

    python tests/golden/make_full_size.py [--only NAME ...] [--jobs 8]

Calls only the CPU oracle (oracle/) and the seeded input generators
(workloads/); nothing here touches the GPU library.  For every configuration at
its stated step count it stores the SHA-256 of the oracle's final state (float64,
[nvars][n], little-endian, C order), the per-variable infinity norm, and a few
sampled values (hex floats), in tests/golden/full_size_oracle.json:

  * heat FTCS and KS RK2, periodic, N = 2^12, 2^14, 2^16, 2^18, 2^20, 50,000 steps,
    Fourier-mode initial states (the per-N sweep configuration);
  * Sod shock tube, N = 2^12 .. 2^18 to t = 0.2, and the first 20,000 steps at
    N = 2^19 and 2^20 (the whole run there is ~1e12 point-updates);
  * the 4096-solve ensemble (heat and KS, N log-uniform in [256, 65536], 10,000
    steps): one truncated digest (16 hex digits) per solve.

The GPU tests recompute each case and compare digests, i.e. bit for bit.  The
oracle does no reductions, so its results do not depend on the thread count.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "full_size_oracle.json")
NSAMPLES = 16


def digest(x: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(x, dtype="<f8").tobytes()).hexdigest()


def cases():
    out = []
    for lg in (12, 14, 16, 18, 20):
        for scheme in (W.HEAT, W.KS):
            out.append((f"{W.SCHEME_NAMES[scheme]}-2^{lg}-50000", "sweep", scheme, lg, 50_000))
    for lg in range(12, 19):
        prob, _ = W.cfg_sod(lg)
        out.append((f"sod-2^{lg}-{prob.nsteps}", "sod", W.EULER, lg, prob.nsteps))
    for lg in (19, 20):
        out.append((f"sod-2^{lg}-20000", "sod", W.EULER, lg, 20_000))
    return out


def problem_of(kind, scheme, lg, nsteps):
    if kind == "sweep":
        return W.cfg_sweep(scheme, lg, nsteps=nsteps)
    return W.cfg_sod(lg, nsteps=nsteps)


def run_case(case):
    name, kind, scheme, lg, nsteps = case
    prob, ic = problem_of(kind, scheme, lg, nsteps)
    t0 = time.time()
    y = oracle.solve(prob, ic)
    rng = np.random.default_rng(lg)
    idx = sorted(set(int(i) for i in rng.integers(0, prob.n, size=NSAMPLES)))
    return name, {
        "kind": kind, "scheme": int(scheme), "log2n": lg, "n": prob.n, "nsteps": nsteps,
        "sha256": digest(y),
        "inf_norm": [float(np.abs(y[v]).max()) for v in range(y.shape[0])],
        "samples": [[i] + [float(y[v, i]).hex() for v in range(y.shape[0])] for i in idx],
        "oracle_seconds": round(time.time() - t0, 1),
    }


def ensemble_digest(j):
    member = W.ensemble()[j]
    y = oracle.solve(member.problem, W.ensemble_ic(member), nthreads=1)
    return j, digest(y)[:16]


def save(data):
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, OUT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=None, help="case names (or 'ensemble') to (re)compute")
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 8)
    args = ap.parse_args()
    data = {"cases": {}, "ensemble": None}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data["_generator"] = "tests/golden/make_full_size.py (CPU oracle only)"
    want = set(args.only) if args.only else None
    oracle.build(force=False)
    oracle.threads(args.jobs)
    for case in cases():
        if want is not None and case[0] not in want:
            continue
        name, rec = run_case(case)
        data["cases"][name] = rec
        print(f"{name}: {rec['oracle_seconds']} s", flush=True)
        save(data)
    if want is None or "ensemble" in want:
        members = W.ensemble()
        order = sorted(range(len(members)), key=lambda j: -members[j].problem.point_updates)
        digests = [None] * len(members)
        t0 = time.time()
        with cf.ProcessPoolExecutor(max_workers=args.jobs) as ex:
            for j, d in ex.map(ensemble_digest, order, chunksize=4):
                digests[j] = d
        data["ensemble"] = {"count": len(members), "seed": 4, "nsteps": 10_000, "digest_hex_digits": 16,
                            "digests": digests, "oracle_seconds": round(time.time() - t0, 1)}
        print(f"ensemble: {time.time() - t0:.0f} s", flush=True)
        save(data)


if __name__ == "__main__":
    main()
