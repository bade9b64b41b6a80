"""Real input and output (half spectrum) on the GPU, through the C-ABI,
against the FP64 oracle's rfftn / irfftn.  Bounds as for complex64: relative
L2 <= 1e-6, round trip <= 2e-6."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import need_gpu, rel_l2, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-6
TOL_RT = 2e-6


@pytest.fixture(scope="module")
def ws():
    return need_gpu()


def real_input(shape, seed):
    return synth.normal_c(shape, seed=seed).real.astype(np.float32)


# (nz, ny, nx): even real axes from 4 up to the longest x pass (16384 complex
# points), odd half lengths (6, 18, 54: radix-3 pencils of 3, 9, 27 points),
# 2D and 1D, y pass ragged (half spectrum of 17, 33, 257 columns) and flattened
# over z, and split y and z axes (2048 points: two passes through the work buffer)
SHAPES = [(1, 1, 4), (1, 1, 6), (1, 3, 8), (2, 4, 18), (32, 32, 32), (24, 48, 64), (16, 27, 54),
          (8, 6, 512), (1, 1, 32768), (3, 6, 2048), (1, 64, 256), (4, 2048, 16), (2048, 2, 8),
          (64, 64, 64), (12, 24, 96), (9, 9, 12)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_r2c_c2r(ws, shape):
    nz, ny, nx = shape
    a = real_input(shape, seed=nx + 7 * ny + 31 * nz)
    p = ws.RealPlan(nx, ny, nz)
    x = torch.from_numpy(a).cuda()
    H = p.r2c(x)
    Hh = to_host(H)
    want = oracle.rfftn(a.astype(np.float64))
    e = rel_l2(Hh, want)
    assert np.array_equal(to_host(x), a), "r2c wrote its input"
    # C2R of the exact half spectrum, unnormalised, against the oracle
    Hx = torch.from_numpy(want.astype(np.complex64)).cuda()
    back = to_host(p.c2r(Hx.clone()))
    e_c2r = rel_l2(back, oracle.irfftn(want.astype(np.complex64).astype(np.complex128), nx))
    # round trip through the inverse (1/N)
    rt = to_host(p.c2r(H, inverse=True))
    e_rt = rel_l2(rt, a)
    print(f"{shape}: r2c {e:.2e} c2r {e_c2r:.2e} round trip {e_rt:.2e} [{p.describe()}]")
    assert e <= TOL and e_c2r <= TOL and e_rt <= TOL_RT


@pytest.mark.parametrize("shape", [(4, 6, 8), (16, 16, 64), (2, 2048, 6)], ids=lambda s: "x".join(map(str, s)))
def test_c2r_of_a_non_hermitian_half_spectrum(ws, shape):
    """A random half spectrum (not the transform of a real array): the y and z
    transforms are taken as given and along x only the real parts of bins 0
    and nx/2 count, as the oracle defines."""
    nz, ny, nx = shape
    H = synth.normal_c((nz, ny, nx // 2 + 1), seed=5 * nx).astype(np.complex64)
    p = ws.RealPlan(nx, ny, nz)
    got = to_host(p.c2r(torch.from_numpy(H).cuda()))
    assert rel_l2(got, oracle.irfftn(H.astype(np.complex128), nx)) <= TOL


@pytest.mark.parametrize("n", [256, 512])
def test_cube_r2c_and_round_trip(ws, n):
    """n^3 real N(0,1) (the real part of the seed-1 draw of the complex
    workload): every half-spectrum bin against the oracle, and the round
    trip; the launch configuration the bench times."""
    a = synth.normal_c64((n, n, n), seed=1).real.copy()
    p = ws.RealPlan(n, n, n)
    x = torch.from_numpy(a).cuda()
    H = p.r2c(x)
    Hh = to_host(H)
    rt = to_host(p.c2r(H, inverse=True))
    del H, x
    torch.cuda.empty_cache()
    want = oracle.rfftn(a.astype(np.float64))
    e = rel_l2(Hh, want)
    del want, Hh
    e_rt = rel_l2(rt, a)
    print(f"{n}^3 real: r2c rel_l2 {e:.3e}, round trip {e_rt:.3e} [{p.describe()}]")
    assert e <= TOL and e_rt <= TOL_RT


def test_real_plan_argument_checks(ws):
    p = ws.RealPlan(16, 8, 4)
    x = torch.zeros((4, 8, 16), dtype=torch.float32, device="cuda")
    H = torch.zeros((4, 8, 9), dtype=torch.complex64, device="cuda")
    # complex calls on a real plan, and in == out on the real calls
    assert ws._execute(p.handle, H.data_ptr(), H.data_ptr(), ws._stream(None)) == 1
    assert ws._execute_r2c(p.handle, x.data_ptr(), x.data_ptr(), ws._stream(None)) == 1
    assert ws._execute_c2r(p.handle, H.data_ptr(), H.data_ptr(), ws._stream(None)) == 1
    # real calls on a complex plan
    c = ws.Plan(16, 8, 4, "c64", -1)
    assert ws._execute_r2c(c.handle, x.data_ptr(), H.data_ptr(), ws._stream(None)) == 1
    assert ws._plan_is_real(p.handle) == 1 and ws._plan_is_real(c.handle) == 0
    # misaligned complex output
    assert ws._execute_r2c(p.handle, x.data_ptr(), H.data_ptr() + 4, ws._stream(None)) == 4
    assert p.work_bytes == 0
    assert ws.RealPlan(16, 2048, 2).work_bytes == 9 * 2048 * 2 * 8


def test_rfftn_irfftn_functions(ws):
    a = real_input((6, 12, 24), seed=77)
    x = torch.from_numpy(a).cuda()
    H = ws.rfftn(x)
    assert H.shape == (6, 12, 13)
    assert rel_l2(to_host(H), oracle.rfftn(a.astype(np.float64))) <= TOL
    Hc = H.clone()
    back = ws.irfftn(H, 24)
    assert torch.equal(H, Hc), "irfftn modified its input"
    assert rel_l2(to_host(back), a) <= TOL_RT


# Padded half spectrum (wsfft_plan_create_real_ex): rows `pitch` complex
# values apart.  The padded plan runs the same arithmetic as the compact one
# on every spectrum column (aligned rows only change the cache policy of its
# passes, and its y and z passes also transform the padding columns), so the
# spectrum part is compared bitwise with the compact plan's, and C2R from
# padded input with C2R from compact input.
PADDED = [((8, 6, 512), 272), ((32, 32, 32), 32), ((32, 32, 32), 20), ((1, 1, 32768), 16400),
          ((4, 2048, 16), 16), ((3, 18, 64), 48), ((2, 3, 4), 8)]


@pytest.mark.parametrize("shape,pitch", PADDED, ids=lambda v: "x".join(map(str, v)) if isinstance(v, tuple) else str(v))
def test_padded_half_spectrum_matches_compact(ws, shape, pitch):
    nz, ny, nx = shape
    nxh = nx // 2 + 1
    a = real_input(shape, seed=5 + nx + ny + nz)
    x = torch.from_numpy(a).cuda()
    pc = ws.RealPlan(nx, ny, nz)
    pp = ws.RealPlan(nx, ny, nz, pitch=pitch)
    print(pp.describe())
    Hc = pc.r2c(x)
    Hp = torch.view_as_complex(torch.full((nz, ny, pitch, 2), float("nan"), device="cuda"))
    pp.r2c(x, out=Hp)
    torch.cuda.synchronize()
    # NaN in the padding (transformed along by the y and z passes) must not
    # reach the spectrum
    assert torch.equal(torch.view_as_real(Hp[..., :nxh]), torch.view_as_real(Hc))
    for inverse in (False, True):
        Hp2 = torch.zeros((nz, ny, pitch), dtype=torch.complex64, device="cuda")
        Hp2[..., :nxh] = Hc
        got = pp.c2r(Hp2, inverse=inverse)
        want = pc.c2r(Hc.clone(), inverse=inverse)
        torch.cuda.synchronize()
        assert torch.equal(got, want), inverse
    rt = to_host(pp.c2r(Hp, inverse=True))
    assert rel_l2(rt, a) <= TOL_RT


def test_padded_plan_against_oracle(ws):
    nz, ny, nx = 16, 24, 96
    a = real_input((nz, ny, nx), seed=77)
    p = ws.RealPlan(nx, ny, nz, pitch=64)
    H = p.r2c(torch.from_numpy(a).cuda())
    assert rel_l2(to_host(H)[..., :nx // 2 + 1], oracle.rfftn(a.astype(np.float64))) <= TOL


def test_poisson_solve_rejects_padded_real_plans(ws):
    p = ws.RealPlan(32, 32, 32, pitch=32)
    f = torch.zeros((32, 32, 32), device="cuda")
    u = torch.empty_like(f)
    w = torch.empty((32, 32, 32), dtype=torch.complex64, device="cuda")
    st = ws._poisson_solve(p.handle, f.data_ptr(), u.data_ptr(), w.data_ptr(), None)
    assert st == 1   # WSFFT_ERROR_INVALID_VALUE
