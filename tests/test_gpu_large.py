"""Large arrays: past the 32-bit lane-offset limit of the split addressing,
and the 1024^3 cube.

16384 x 16384 x 2 complex64 (4 GiB): the z pass has a 2 GiB element stride,
so its per-lane offsets no longer fit 32 bits and it runs the 64-bit
element-index form of the same kernel.  Checked two ways:
* the z pass alone on a random input, against the oracle on sampled pencils;
* the whole transform of a separable input f(x) g(y) h(z), whose DFT is
  exactly F(kx) G(ky) H(kz) (each factor from the oracle's 1D transform), at
  sampled outputs, plus Parseval over the whole output.
1024^3 complex64 (8 GiB per array; pencils of 1024 in every pass, z stride
8 MiB) is checked the same two ways: each pass alone on a random input at
sampled pencils, and the separable whole transform.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import need_gpu, rel_l2

pytestmark = pytest.mark.gpu
NX, NY, NZ = 16384, 16384, 2
SAMPLES = 200_000


@pytest.fixture(scope="module")
def ws():
    b = need_gpu()
    free, _ = torch.cuda.mem_get_info()
    if free < 20 * 2 ** 30:
        pytest.skip("needs 20 GiB of free device memory")
    return b


def _plan(ws):
    p = ws.Plan(NX, NY, NZ, "c64", -1)
    desc = p.describe()
    assert "z[strided n=2" in desc, desc
    return p


def test_z_pass_alone_random_input(ws):
    p = _plan(ws)
    gen = torch.Generator(device="cuda").manual_seed(34)
    x = torch.randn((NZ, NY, NX), dtype=torch.complex64, device="cuda", generator=gen)
    y = x.clone()
    p.execute_pass(p.num_passes - 1, x, y)     # the z pass runs in place on the output
    torch.cuda.synchronize()
    rng = np.random.default_rng(35)
    ky = torch.from_numpy(rng.integers(0, NY, SAMPLES)).cuda()
    kx = torch.from_numpy(rng.integers(0, NX, SAMPLES)).cuda()
    a = x[:, ky, kx].cpu().numpy().T.astype(np.complex128)        # (SAMPLES, 2) pencils along z
    got = y[:, ky, kx].cpu().numpy().T
    want = oracle.fft1d_batch(np.ascontiguousarray(a), -1)
    e = rel_l2(got, want)
    print(f"z pass, 2 GiB stride: {SAMPLES} pencils, rel_l2 {e:.3e}")
    assert e <= 1e-6


def test_whole_transform_separable_input(ws):
    p = _plan(ws)
    f = synth.normal_c((NX,), seed=31).astype(np.complex64)
    g = synth.normal_c((NY,), seed=32).astype(np.complex64)
    h = synth.normal_c((NZ,), seed=33).astype(np.complex64)
    x = (torch.from_numpy(h).cuda()[:, None, None] * torch.from_numpy(g).cuda()[None, :, None]) * \
        torch.from_numpy(f).cuda()[None, None, :]
    y = torch.empty_like(x)
    p.execute(x, y)
    torch.cuda.synchronize()
    F = oracle.fft1d_batch(f.astype(np.complex128)[None], -1)[0]
    G = oracle.fft1d_batch(g.astype(np.complex128)[None], -1)[0]
    H = oracle.fft1d_batch(h.astype(np.complex128)[None], -1)[0]
    rng = np.random.default_rng(36)
    kz = rng.integers(0, NZ, SAMPLES)
    ky = rng.integers(0, NY, SAMPLES)
    kx = rng.integers(0, NX, SAMPLES)
    got = y[torch.from_numpy(kz).cuda(), torch.from_numpy(ky).cuda(), torch.from_numpy(kx).cuda()].cpu().numpy()
    want = H[kz] * G[ky] * F[kx]
    e = rel_l2(got, want)
    # Parseval: ||Y||^2 = N ||x||^2, both accumulated in FP64 plane by plane
    sx = sum(float((x[z].abs().double() ** 2).sum()) for z in range(NZ))
    sy = sum(float((y[z].abs().double() ** 2).sum()) for z in range(NZ))
    parseval = abs(sy / (NX * NY * NZ * sx) - 1.0)
    print(f"16384x16384x2 separable: sampled rel_l2 {e:.3e}, Parseval deviation {parseval:.2e} [{p.describe()}]")
    assert e <= 1e-6
    assert parseval <= 1e-6


CUBE = 1024
CUBE_SAMPLES = 20_000


def _cube_plan(ws):
    free, _ = torch.cuda.mem_get_info()
    if free < 20 * 2 ** 30:
        pytest.skip("needs 20 GiB of free device memory")
    return ws.Plan(CUBE, CUBE, CUBE, "c64", -1)


@pytest.mark.parametrize("axis", [0, 1, 2], ids=["x", "y", "z"])
def test_1024cubed_each_pass_random_input(ws, axis):
    """Pass `axis` of the 1024^3 plan alone: CUBE_SAMPLES random pencils along
    that axis against the oracle's 1D transform."""
    p = _cube_plan(ws)
    assert p.num_passes == 3, p.describe()
    gen = torch.Generator(device="cuda").manual_seed(40 + axis)
    x = torch.randn((CUBE, CUBE, CUBE), dtype=torch.complex64, device="cuda", generator=gen)
    y = torch.empty_like(x) if axis == 0 else x.clone()   # the y and z passes run in place on the output
    p.execute_pass(axis, x, y)
    torch.cuda.synchronize()
    rng = np.random.default_rng(41 + axis)
    i = torch.from_numpy(rng.integers(0, CUBE, CUBE_SAMPLES)).cuda()
    k = torch.from_numpy(rng.integers(0, CUBE, CUBE_SAMPLES)).cuda()
    if axis == 0:
        a, got = x[i, k, :], y[i, k, :]                  # (z, y) fixed, pencils along x
    elif axis == 1:
        a, got = x[i, :, k], y[i, :, k]                  # (z, x) fixed, along y
    else:
        a, got = x[:, i, k].T, y[:, i, k].T              # (y, x) fixed, along z
    a = a.cpu().numpy().astype(np.complex128)
    got = got.cpu().numpy()
    del x, y
    torch.cuda.empty_cache()
    want = oracle.fft1d_batch(np.ascontiguousarray(a), -1)
    e = rel_l2(got, want)
    print(f"1024^3 pass {axis}: {CUBE_SAMPLES} pencils, rel_l2 {e:.3e} [{p.describe()}]")
    assert e <= 1e-6


def test_1024cubed_separable(ws):
    p = _cube_plan(ws)
    f = synth.normal_c((CUBE,), seed=43).astype(np.complex64)
    g = synth.normal_c((CUBE,), seed=44).astype(np.complex64)
    h = synth.normal_c((CUBE,), seed=45).astype(np.complex64)
    x = (torch.from_numpy(h).cuda()[:, None, None] * torch.from_numpy(g).cuda()[None, :, None]) * \
        torch.from_numpy(f).cuda()[None, None, :]
    y = torch.empty_like(x)
    p.execute(x, y)
    torch.cuda.synchronize()
    F, G, H = (oracle.fft1d_batch(v.astype(np.complex128)[None], -1)[0] for v in (f, g, h))
    rng = np.random.default_rng(46)
    kz, ky, kx = (rng.integers(0, CUBE, SAMPLES) for _ in range(3))
    got = y[torch.from_numpy(kz).cuda(), torch.from_numpy(ky).cuda(), torch.from_numpy(kx).cuda()].cpu().numpy()
    want = H[kz] * G[ky] * F[kx]
    e = rel_l2(got, want)
    sx = sum(float((x[z].abs().double() ** 2).sum()) for z in range(CUBE))
    sy = sum(float((y[z].abs().double() ** 2).sum()) for z in range(CUBE))
    parseval = abs(sy / (CUBE ** 3 * sx) - 1.0)
    print(f"1024^3 separable: sampled rel_l2 {e:.3e}, Parseval deviation {parseval:.2e}")
    assert e <= 1e-6
    assert parseval <= 1e-6
