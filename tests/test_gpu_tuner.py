"""Autotuner: every compiled launch variant of the hot lengths matches the FP64
oracle, tuning records its choices in the cache, and later plans reuse them."""
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import c16_to_c128, c16_to_dev, need_gpu, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

SHAPES = [(512, 64, 32), (256, 1024, 4), (128, 64, 512), (4096, 8, 2), (64, 2048, 1)]


@pytest.fixture(scope="module")
def ws():
    return need_gpu()


@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_forced_variants_match_oracle(ws, shape, variant, monkeypatch):
    monkeypatch.setenv("WSFFT_TUNE_FORCE", str(variant))
    nx, ny, nz = shape
    a = synth.normal_c((nz, ny, nx), seed=31).astype(np.complex64)
    p = ws.Plan(nx, ny, nz, "c64", -1)
    y = to_host(p.execute(to_dev(a)))
    assert rel_l2(y, oracle.fftn(a.astype(np.complex128), -1)) <= 1e-6, p.describe()
    r = to_host(p.execute_inverse(p.execute(to_dev(a))))
    assert rel_l2(r, a) <= 2e-6


@pytest.mark.parametrize("flags", [0, 4], ids=["fp32-math", "fp16-math"])   # 4: WSFFT_FLAG_FP16_MATH
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_forced_variants_fp16(ws, variant, flags, monkeypatch):
    monkeypatch.setenv("WSFFT_TUNE_FORCE", str(variant))
    nx, ny, nz = 512, 256, 16
    pairs = synth.to_fp16_pairs(synth.normal_c((nz, ny, nx), seed=32, scale=0.5))
    p = ws.Plan(nx, ny, nz, "fp16", -1, flags)
    got = c16_to_c128(p.execute(c16_to_dev(pairs, "fp16")), "fp16") * 2.0 ** p.scale_log2
    want = oracle.fftn(synth.pairs_to_c128(pairs, "fp16"), -1)
    assert rel_l2(got, want) <= 3e-3


def test_tuning_writes_and_reuses_cache(ws, tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("WSFFT_TUNE_CACHE", str(cache))
    monkeypatch.delenv("WSFFT_TUNE_FORCE", raising=False)
    nx, ny, nz = 256, 256, 64
    a = synth.normal_c((nz, ny, nx), seed=33).astype(np.complex64)
    p = ws.Plan(nx, ny, nz, "c64", -1, ws.FLAG_TUNE)
    assert rel_l2(to_host(p.execute(to_dev(a))), oracle.fftn(a.astype(np.complex128), -1)) <= 1e-6
    lines = cache.read_text().splitlines()
    assert len(lines) == 3                # one tuned entry per pass
    for ln in lines:
        key, v, us = ln.split()
        assert int(v) in (0, 1, 2) and float(us) > 0
    # a second plan of the same geometry reads the cache instead of timing
    p2 = ws.Plan(nx, ny, nz, "c64", -1, ws.FLAG_TUNE)
    assert len(cache.read_text().splitlines()) == 3
    assert p2.describe() == p.describe()
