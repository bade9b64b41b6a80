"""bench.py's host-side contract, on the CPU: argument checks that must fail
before any device work, and the consistency of the recorded HBM traffic of
the current kernel sources (when none is recorded the bench reports traffic
as null, and the check is skipped)."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_unknown_variant_is_refused():
    r = _run("--variants", "fp16,no_such_variant")
    assert r.returncode == 2
    assert "no_such_variant" in r.stderr


def test_variant_names_are_unique():
    assert len(set(bench.VARIANTS)) == len(bench.VARIANTS)


def test_recorded_traffic_matches_kernel_sources():
    h = bench.kernel_sources_hash()
    if h not in bench.MEASURED_TRAFFIC:
        pytest.skip(f"no HBM counters recorded for kernel sources {h}; bench reports traffic null")
    rec = bench.MEASURED_TRAFFIC[h]
    algorithmic = 2 * 512 ** 3 * 8
    assert 0.99 * algorithmic <= rec["bytes"] <= 1.5 * algorithmic
    assert os.path.exists(os.path.join(ROOT, rec["profile"]))
    with open(os.path.join(ROOT, rec["profile"])) as f:
        assert h in f.read()
