"""GPU parity at the benchmark configurations' full sizes and stated step counts.

The expected results are the CPU oracle's, computed once by the committed script
tests/golden/make_full_size.py (it calls only oracle/ and workloads/) and stored
as SHA-256 digests of the final states with sampled values and norms in
tests/golden/full_size_oracle.json.  Each case is solved here with the tuned
swept plan (the launch configuration bench.py times) and compared digest for
digest: the bar is bit-for-bit equality with the oracle, which implies the
1e-12 relative bound.  On a mismatch the message reports the relative error at
the stored samples.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
import paper_1705_03162_amd as sw  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size_oracle.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _digest(x: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(x, dtype="<f8").tobytes()).hexdigest()


def _problem(rec):
    if rec["kind"] == "sweep":
        return W.cfg_sweep(rec["scheme"], rec["log2n"], nsteps=rec["nsteps"])
    return W.cfg_sod(rec["log2n"], nsteps=rec["nsteps"])


def _sample_report(got, rec):
    worst = 0.0
    for row in rec["samples"]:
        i = row[0]
        for v, hx in enumerate(row[1:]):
            want = float.fromhex(hx)
            worst = max(worst, abs(got[v, i] - want) / rec["inf_norm"][v])
    return worst


CASES = sorted(_golden()["cases"]) if os.path.exists(GOLDEN) else []


@pytest.mark.parametrize("name", CASES)
def test_full_size_swept_equals_oracle(name):
    rec = _golden()["cases"][name]
    prob, ic = _problem(rec)
    print(f"[gpu] full-size {name}: n={prob.n} steps={prob.nsteps}", flush=True)
    with sw.Plan(prob) as plan:
        x = torch.tensor(ic, dtype=torch.float64, device=DEV)
        plan.swept(x)
        torch.cuda.synchronize()
    got = x.cpu().numpy().reshape(prob.nvars, prob.n)
    assert _digest(got) == rec["sha256"], (
        f"{name}: GPU result differs from the oracle; max relative error at the stored samples "
        f"{_sample_report(got, rec):.3e}")


@pytest.mark.parametrize("persistent", [False, True])
def test_ensemble_every_result_equals_oracle(persistent):
    """The 4096-solve ensemble (heat and KS, N log-uniform in [256, 65536], 10,000 steps)
    in one batched graph launch (one launch per phase index, or the persistent launch):
    every one of the 4096 results equals the oracle's."""
    g = _golden()["ensemble"]
    members = W.ensemble()
    assert len(members) == g["count"]
    print(f"[gpu] ensemble of {len(members)} solves (persistent={persistent}) against the oracle digests",
          flush=True)
    states = [torch.tensor(W.ensemble_ic(m), dtype=torch.float64, device=DEV) for m in members]
    with sw.Batch(budget_bytes=64 << 30, persistent=persistent) as b:
        tickets = [b.submit(m.problem, x) for m, x in zip(members, states)]
        b.run()
    torch.cuda.synchronize()
    bad = [j for j, x in enumerate(states) if _digest(x.cpu().numpy())[:16] != g["digests"][j]]
    assert not bad, f"{len(bad)} of {len(members)} ensemble results differ from the oracle, e.g. {bad[:5]}"
