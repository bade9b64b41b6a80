"""16-bit storage (FP16, BF16) with FP32 arithmetic and per-pass power-of-two
scaling, against the FP64 oracle applied to the same rounded input.

Bound: relative L2 <= 3e-3 for the three-pass 512^3 workload.  Every stored
pass rounds once to the storage type, and the transform is unitary up to
scale, so the error grows like sqrt(passes) times the one-rounding floor; for
schedules with more passes (split axes) the bound is scaled by
sqrt(passes / 3).

Twiddles rounded to the storage type are the literal workload recipe.  For
BF16 that recipe cannot meet 3e-3: the one-rounding floor of BF16 alone is
~1.7e-3, three stored passes give ~sqrt(3) floors and the BF16-rounded
twiddles add about one more rounding per twiddled stage (measured 3.8e-3 at
512^3).  That variant is reported as over the 3e-3 target and held to a bound
derived from the arithmetic instead, 3 one-rounding floors (scaled like the
others for longer schedules); BF16 with FP32 twiddles is held to 3e-3.

A whole-array relative L2 cannot see one wrong pencil among 2^18, so the
512^3 tests also bound every pencil: each pass alone, every pencil of the
array against the oracle's 1D transform, and the whole transform, every
pencil along each axis, both as a multiple of the one-rounding floor.  Each
test prints its ratios to that floor."""
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
TARGET = 3e-3   # relative L2 target of the 16-bit workloads
# (kind, flags, bound): a number is an absolute bound; "floors" means a
# multiple of the one-rounding floor (BF16 with BF16 twiddles, see above)
CASES = [("fp16", 0, TARGET), ("bf16", 0, "3 floors"), ("bf16", 1, TARGET), ("fp16", FP16_MATH, TARGET)]
CASE_IDS = ["fp16", "bf16", "bf16-fp32tw", "fp16-math"]
# per-pencil bounds, in one-rounding floors: one pass alone, and the whole
# transform (FP16 arithmetic rounds every butterfly stage as well)
PENCIL_FLOORS_PASS = 10.0
PENCIL_FLOORS_WHOLE = {0: 10.0, FP16_MATH: 15.0}


def bound_of(bound, floor, passes):
    b = 3.0 * floor if bound == "3 floors" else bound
    return b * max(1.0, (passes / 3) ** 0.5)


@pytest.mark.parametrize("kind,flags,bound", CASES, ids=CASE_IDS)
# (54, 36, 8) and (48, 54, 24): strided tiles of 32 columns with a ragged
# last tile of an even column count (y: 22, 16; z of the first: 24);
# (27, 16, 8): odd y column count and stride, where adjacent columns do not
# pair, then an even z pass that does; (16, 512, 512): 512-point strided y
# and z passes (the 512^3 kernels) on an array small enough (2^22 elements)
# that one wrong pencil moves the whole-array error past the bound
@pytest.mark.parametrize("shape", [(64, 64, 64), (96, 32, 128), (32, 1, 1), (256, 256, 1), (8, 2048, 2),
                                   (54, 36, 8), (48, 54, 24), (27, 16, 8), (16, 512, 512)],
                         ids=lambda s: "x".join(map(str, s)))
def test_small(ws, shape, kind, flags, bound):
    e, fl, p = run_case(ws, shape, kind, flags)
    b = bound_of(bound, fl, p.num_passes)
    print(f"{kind} flags={flags} {shape}: rel_l2 {e:.3e}, floor {fl:.3e}, ratio {e / fl:.2f}, "
          f"S={p.scale_log2}, passes {p.num_passes}, bound {b:.2e}"
          + ("  [over the 3e-3 target]" if e > TARGET else ""))
    assert e <= b


def pencil_errors(got, want, axis):
    """Relative L2 error of every pencil along `axis` of (nz, ny, nx) arrays
    (axis 0 = x, the last array axis)."""
    ax = 2 - axis
    d = np.moveaxis(got - want, ax, -1)
    w = np.moveaxis(want, ax, -1)
    return np.sqrt((np.abs(d) ** 2).sum(-1) / (np.abs(w) ** 2).sum(-1)).ravel()


@pytest.mark.parametrize("kind,flags,bound", CASES, ids=CASE_IDS)
def test_512cubed(ws, kind, flags, bound):
    """512^3 forward, re/im 0.5*N(0,1) seed 2 rounded to storage, every output
    element against the oracle; then every pencil along each axis."""
    n = 512
    z = synth.normal_c((n, n, n), seed=2, scale=0.5)
    pairs = round_pairs(z, kind)
    del z
    a = synth.pairs_to_c128(pairs, kind)
    p = ws.Plan(n, n, n, kind, -1, flags)
    x = c16_to_dev(pairs, kind)
    del pairs
    got = c16_to_c128(p.execute(x), kind) * 2.0 ** p.scale_log2
    del x
    torch.cuda.empty_cache()
    X = oracle.fftn(a, -1)
    del a
    e, fl = rel_l2(got, X), floor_error(X, p.scale_log2, kind)
    b = bound_of(bound, fl, 3)
    worst = [float(pencil_errors(got, X, ax).max()) for ax in range(3)]
    pb = PENCIL_FLOORS_WHOLE[flags & FP16_MATH] * fl
    print(f"512^3 {kind} flags={flags}: rel_l2 {e:.3e}, floor {fl:.3e}, ratio {e / fl:.2f}, bound {b:.2e}"
          + ("  [over the 3e-3 target]" if e > TARGET else "")
          + f"; worst pencil along x/y/z {worst[0]:.2e}/{worst[1]:.2e}/{worst[2]:.2e} "
          f"({max(worst) / fl:.2f} floors, bound {pb / fl:.0f}) S={p.scale_log2} [{p.describe()}]")
    assert e <= b
    assert max(worst) <= pb


@pytest.mark.parametrize("kind,flags,bound", CASES, ids=CASE_IDS)
@pytest.mark.parametrize("axis", [0, 1, 2], ids=["x", "y", "z"])
def test_512cubed_each_pass_every_pencil(ws, kind, flags, bound, axis):
    """One pass of the 512^3 plan alone (the kernel the whole transform runs
    for that axis) on a random 16-bit input: all 2^18 pencils against the
    oracle's 1D transform, each within PENCIL_FLOORS_PASS one-rounding
    floors, so a single wrong pencil fails."""
    n = 512
    z = synth.normal_c((n, n, n), seed=20 + axis, scale=0.5)
    pairs = round_pairs(z, kind)
    del z
    p = ws.Plan(n, n, n, kind, -1, flags)
    assert p.num_passes == 3
    x = c16_to_dev(pairs, kind)
    y = torch.empty_like(x) if axis == 0 else x.clone()   # the y and z passes run in place on the output
    p.execute_pass(axis, x, y)
    s_p = 5                                               # 2^-5 per 512-point pass
    got = c16_to_c128(y, kind) * 2.0 ** s_p
    del x, y
    torch.cuda.empty_cache()
    a = synth.pairs_to_c128(pairs, kind)
    del pairs
    ax = 2 - axis
    want = np.moveaxis(oracle.fft1d_batch(np.ascontiguousarray(np.moveaxis(a, ax, -1)).reshape(-1, n), -1)
                       .reshape(np.moveaxis(a, ax, -1).shape), -1, ax)
    del a
    fl = floor_error(want, s_p, kind)
    errs = pencil_errors(got, want, axis)
    print(f"512^3 {kind} flags={flags} pass {'xyz'[axis]} alone: rel_l2 {rel_l2(got, want):.3e}, "
          f"floor {fl:.3e}, worst pencil {errs.max():.3e} ({errs.max() / fl:.2f} floors), "
          f"median {np.median(errs):.3e}")
    assert errs.size == n * n
    assert errs.max() <= PENCIL_FLOORS_PASS * fl


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
    x = c16_to_dev(pairs, kind)
    ref = oracle.fftn(a, +1)
    fl = floor_error(ref, p.scale_log2, kind)
    # BF16 here has BF16 twiddles: the derived 3-floor bound (module docstring)
    bound = bound_of(TARGET if kind == "fp16" else "3 floors", fl, p.num_passes)
    adj = c16_to_c128(p.execute_adjoint(x), kind) * 2.0 ** p.scale_log2
    assert rel_l2(adj, ref) <= bound
    inv = c16_to_c128(p.execute_inverse(x), kind) * 2.0 ** -p.scale_log2
    assert rel_l2(inv, ref / a.size) <= bound


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
    del y
    torch.cuda.empty_cache()
    e = rel_l2(back, a)
    # six stored passes: sqrt(2) times the forward bound (BF16 with BF16 twiddles: the derived one)
    fl = floor_error(oracle.fftn(a, -1), p.scale_log2, kind)
    b = 2 ** 0.5 * bound_of(TARGET if kind == "fp16" else "3 floors", fl, 3)
    print(f"512^3 {kind} flags={flags} round trip: rel_l2 {e:.3e}, floor {fl:.3e}, bound {b:.2e}")
    assert e <= b


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
