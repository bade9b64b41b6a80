"""16-bit storage (FP16, BF16) with FP32 arithmetic and per-pass power-of-two
scaling, against the FP64 oracle applied to the same rounded input.

Bound: relative L2 <= 3e-3 for the three-pass 512^3 workload.  Every stored
pass rounds once to the storage type, and the transform is unitary up to
scale, so the error grows like sqrt(passes) times the one-rounding floor; for
schedules with more passes (split axes) the bound is scaled by
sqrt(passes / 3).  Twiddles rounded to the storage type are the literal
workload recipe; for BF16 that recipe's error sits above 3e-3 (the
one-rounding floor of BF16 alone is ~1.7e-3), so it is reported and held to
6e-3, while BF16 with FP32 twiddles is held to 3e-3.  Each test also prints
the ratio to the single-rounding floor."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import c16_to_c128, c16_to_dev, need_gpu, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    return need_gpu()


def round_pairs(z, kind):
    return synth.to_fp16_pairs(z) if kind == "fp16" else synth.to_bf16_pairs(z)


def floor_error(X, S, kind):
    """Error of rounding the exact scaled result once to the storage type."""
    r = synth.pairs_to_c128(round_pairs(X * 2.0 ** -S, kind), kind) * 2.0 ** S
    return rel_l2(r, X)


def run_case(ws, shape, kind, flags, seed=2):
    nx, ny, nz = shape
    z = synth.normal_c((nz, ny, nx), seed=seed, scale=0.5)
    pairs = round_pairs(z, kind)
    a = synth.pairs_to_c128(pairs, kind)        # the exact stored input
    p = ws.Plan(nx, ny, nz, kind, -1, flags)
    y = p.execute(c16_to_dev(pairs, kind))
    got = c16_to_c128(y, kind) * 2.0 ** p.scale_log2
    X = oracle.fftn(a, -1)
    return rel_l2(got, X), floor_error(X, p.scale_log2, kind), p


FP16_MATH = 4   # WSFFT_FLAG_FP16_MATH: packed FP16 butterflies, FP16 values in registers and LDS
CASES = [("fp16", 0, 3e-3), ("bf16", 0, 6e-3), ("bf16", 1, 3e-3), ("fp16", FP16_MATH, 3e-3)]
CASE_IDS = ["fp16", "bf16", "bf16-fp32tw", "fp16-math"]


@pytest.mark.parametrize("kind,flags,bound", CASES, ids=CASE_IDS)
# (54, 36, 8) and (48, 54, 24): strided tiles of 32 columns with a ragged
# last tile of an even column count (y: 22, 16; z of the first: 24);
# (27, 16, 8): odd y column count and stride, where adjacent columns do not
# pair, then an even z pass that does
@pytest.mark.parametrize("shape", [(64, 64, 64), (96, 32, 128), (32, 1, 1), (256, 256, 1), (8, 2048, 2),
                                   (54, 36, 8), (48, 54, 24), (27, 16, 8)],
                         ids=lambda s: "x".join(map(str, s)))
def test_small(ws, shape, kind, flags, bound):
    e, fl, p = run_case(ws, shape, kind, flags)
    b = bound * max(1.0, (p.num_passes / 3) ** 0.5)
    print(f"{kind} flags={flags} {shape}: rel_l2 {e:.3e}, floor {fl:.3e}, ratio {e / fl:.2f}, "
          f"S={p.scale_log2}, passes {p.num_passes}, bound {b:.2e}")
    assert e <= b


@pytest.mark.parametrize("kind,flags,bound", CASES, ids=CASE_IDS)
def test_512cubed(ws, kind, flags, bound):
    """512^3 forward, re/im 0.5*N(0,1) seed 2 rounded to storage, every output
    element against the oracle."""
    e, fl, p = run_case(ws, (512, 512, 512), kind, flags)
    print(f"512^3 {kind} flags={flags}: rel_l2 {e:.3e}, floor {fl:.3e}, ratio {e / fl:.2f}, S={p.scale_log2} "
          f"[{p.describe()}]")
    assert e <= bound


def test_scale_log2_values(ws):
    assert ws.Plan(512, 512, 512, "fp16").scale_log2 == 15      # 5 per 512-point pass
    assert ws.Plan(96, 32, 256, "bf16").scale_log2 == 4 + 3 + 4
    assert ws.Plan(512, 512, 512, "c64").scale_log2 == 0


@pytest.mark.parametrize("flags", [0, FP16_MATH], ids=["fp16", "fp16-math"])
def test_constant_input_stays_finite(ws, flags):
    """A constant input puts all energy in one bin (N times larger): the
    per-pass scaling keeps it in FP16 range (with FP16 arithmetic also the
    partial sums inside each pass)."""
    n = 256
    pairs = np.zeros((n, n, n, 2), np.float16)
    pairs[..., 0] = 1.0
    p = ws.Plan(n, n, n, "fp16", -1, flags)
    y = c16_to_c128(p.execute(c16_to_dev(pairs, "fp16")), "fp16")
    assert np.isfinite(y).all()
    assert abs(y[0, 0, 0] * 2.0 ** p.scale_log2 - n ** 3) <= 1e-3 * n ** 3


@pytest.mark.parametrize("kind,flags", [("fp16", 0), ("bf16", 0), ("fp16", FP16_MATH)],
                         ids=["fp16", "bf16", "fp16-math"])
@pytest.mark.parametrize("shape", [(64, 32, 16), (96, 27, 8), (8192, 1, 4)], ids=lambda s: "x".join(map(str, s)))
def test_adjoint_and_inverse_16bit(ws, kind, flags, shape):
    """The adjoint (opposite sign, 2^-S times the exact sum) and the inverse
    (2^S/N times the opposite-sign sum, the exact inverse of the forward
    transform) with 16-bit storage, against the oracle on the same rounded
    input."""
    nx, ny, nz = shape
    z = synth.normal_c((nz, ny, nx), seed=13, scale=0.5)
    pairs = round_pairs(z, kind)
    a = synth.pairs_to_c128(pairs, kind)
    p = ws.Plan(nx, ny, nz, kind, -1, flags)
    bound = (3e-3 if kind == "fp16" else 6e-3) * max(1.0, (p.num_passes / 3) ** 0.5)
    x = c16_to_dev(pairs, kind)
    adj = c16_to_c128(p.execute_adjoint(x), kind) * 2.0 ** p.scale_log2
    assert rel_l2(adj, oracle.fftn(a, +1)) <= bound
    inv = c16_to_c128(p.execute_inverse(x), kind) * 2.0 ** -p.scale_log2
    assert rel_l2(inv, oracle.fftn(a, +1) / a.size) <= bound


@pytest.mark.parametrize("kind,flags", [("fp16", 0), ("bf16", 0), ("fp16", FP16_MATH)],
                         ids=["fp16", "bf16", "fp16-math"])
def test_round_trip_16bit_512cubed(ws, kind, flags):
    """inverse(forward(a)) = a at 512^3: the inverse undoes the forward
    scaling, so no stored value leaves the 16-bit range on the way back."""
    n = 512
    z = synth.normal_c((n, n, n), seed=14, scale=0.5)
    pairs = round_pairs(z, kind)
    a = synth.pairs_to_c128(pairs, kind)
    del z
    p = ws.Plan(n, n, n, kind, -1, flags)
    y = p.execute(c16_to_dev(pairs, kind))
    back = c16_to_c128(p.execute_inverse(y), kind)
    e = rel_l2(back, a)
    print(f"512^3 {kind} flags={flags} round trip: rel_l2 {e:.3e}")
    assert e <= 2 * 3e-3 * (1.0 if kind == "fp16" else 2.0)


@pytest.mark.parametrize("flags", [0, FP16_MATH], ids=["fp16", "fp16-math"])
def test_batched_16bit_matches_single_calls(ws, flags):
    shapes = [(32, 64, 16), (64, 32, 32), (128, 16, 8)]
    plans = [ws.Plan(*s, "fp16", -1, flags) for s in shapes]
    xs = [c16_to_dev(synth.to_fp16_pairs(synth.normal_c((s[2], s[1], s[0]), seed=50 + i, scale=0.5)), "fp16")
          for i, s in enumerate(shapes)]
    ys = [torch.empty_like(x) for x in xs]
    ws.execute_batched(plans, xs, ys)
    for p, x, y in zip(plans, xs, ys):
        single = p.execute(x)
        torch.cuda.synchronize()
        assert torch.equal(single, y)
