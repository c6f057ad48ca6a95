"""The benchmark's host logic on the CPU: it refuses more than one GPU, and the HBM
traffic figure it reports beside the roofline is taken from the committed counter
summary only while the kernel sources and the tile shape are those the counters
were measured on (otherwise it is null)."""
import importlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    return importlib.import_module("bench")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _summary(tmp_path, digest, width=1024, threads=64, hbm=34_600_000):
    p = tmp_path / "pmc.txt"
    p.write_text("header line\n"
                 f"@kernel_digest {digest}\n@width {width}\n@threads {threads}\n@n 1048576\n"
                 f"@hbm_bytes_per_launch {hbm}\n@algorithmic_bytes_per_launch 33685504\n")
    return str(p)


def test_traffic_only_for_the_profiled_kernel_and_shape(bench, tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", _summary(tmp_path, bench.kernel_digest()))
    assert bench.measured_traffic(1024, 64) == 34_600_000.0
    assert bench.measured_traffic(512, 64) is None          # other tile shape
    assert bench.measured_traffic(1024, 128) is None
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", _summary(tmp_path, "0123456789abcdef"))
    assert bench.measured_traffic(1024, 64) is None         # counters of other kernel sources
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic(1024, 64) is None


def test_digest_follows_every_kernel_source(bench, tmp_path, monkeypatch):
    files = []
    for i, rel in enumerate(bench.KERNEL_SOURCES):
        p = tmp_path / f"src{i}"
        with open(os.path.join(ROOT, rel), "rb") as src:
            p.write_bytes(src.read())
        files.append(p)
    monkeypatch.setattr(bench, "KERNEL_SOURCES", tuple(str(p) for p in files))
    base = bench.kernel_digest()
    for p in files:
        original = p.read_bytes()
        p.write_bytes(original + b"\n")
        assert bench.kernel_digest() != base, p
        p.write_bytes(original)
    assert bench.kernel_digest() == base


def test_algorithmic_flop_counts(bench):
    """Guard on the operation counts the roofline is priced with (each add, subtract and
    multiply of the update as the paper writes it): heat 2 adds and 2 multiplies; KS 16 in
    f with the four-point terms of Eq. KSDisc in symmetric pairs, 2 in the stage."""
    assert bench.FLOPS_PER_POINT_LEVEL[bench.W.HEAT] == 4
    assert bench.FLOPS_PER_POINT_LEVEL[bench.W.KS] == 18
