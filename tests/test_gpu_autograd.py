"""Differentiation through the adjoint kernels: torch.autograd Functions whose
backward runs wsfft_execute_adjoint / the inverse kernels, checked against the
FP64 oracle, finite differences, and the spectral Poisson solve's closed-form
gradient."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import need_gpu, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    return need_gpu()


@pytest.mark.parametrize("sign", [-1, 1])
def test_fftn_backward_is_adjoint(ws, sign):
    shape = (24, 32, 48)
    x = to_dev(synth.normal_c(shape, seed=1)).requires_grad_(True)
    w = synth.normal_c(shape, seed=2)
    loss = (ws.FFTn.apply(x, sign) * to_dev(w).conj()).real.sum()
    loss.backward()
    assert rel_l2(to_host(x.grad), oracle.fftn(w, -sign)) <= 1e-6


def test_ifftn_backward(ws):
    shape = (16, 32, 64)
    x = to_dev(synth.normal_c(shape, seed=3)).requires_grad_(True)
    w = synth.normal_c(shape, seed=4)
    loss = (ws.IFFTn.apply(x, -1) * to_dev(w).conj()).real.sum()
    loss.backward()
    # y = (1/N) F_{+1} x  =>  grad = (1/N) F_{-1} w
    assert rel_l2(to_host(x.grad), oracle.fftn(w, -1) / w.size) <= 1e-6


def test_fftn_directional_finite_difference(ws):
    """L(x) = Re<w, F x> is linear, so a central difference equals the
    directional derivative for any step; a unit step keeps the FP32 rounding
    of L (~1e-3 here) from being amplified by 1/(2h).  Random directions."""
    shape = (16, 16, 16)
    x0 = to_dev(synth.normal_c(shape, seed=5))
    w = to_dev(synth.normal_c(shape, seed=6))
    xg = x0.clone().requires_grad_(True)
    (ws.FFTn.apply(xg, -1) * w.conj()).real.sum().backward()

    def L(x):
        y = ws.FFTn.apply(x, -1)
        return float(np.sum((to_host(y).astype(np.complex128) * np.conj(to_host(w).astype(np.complex128))).real))

    h = 1.0
    for s in range(4):
        v = to_dev(synth.normal_c(shape, seed=100 + s))
        fd = (L(x0 + h * v) - L(x0 - h * v)) / (2 * h)
        an = float(np.sum((np.conj(to_host(xg.grad).astype(np.complex128)) * to_host(v).astype(np.complex128)).real))
        assert abs(fd - an) <= 1e-3 * abs(an) + 1e-3


def test_pointwise_kernels(ws):
    f = torch.from_numpy(synth.normal_c((6, 10, 12), seed=7).real.astype(np.float32)).cuda()
    z = ws.RealToComplex.apply(f)
    assert torch.equal(z.real, f) and torch.count_nonzero(z.imag) == 0
    assert torch.equal(ws.ComplexRealPart.apply(z * (1 + 2j)), f)
    X = to_dev(synth.normal_c((6, 10, 12), seed=8))
    got = to_host(ws.PoissonSymbol.apply(X))
    want = to_host(X) * oracle.poisson_symbol(12, 10, 6)
    assert np.max(np.abs(got - want)) <= 1e-6 * np.max(np.abs(want))


def _poisson_inputs(n, seed):
    f = synth.gaussian_bumps(n, 64, 0.05, seed=seed)
    w = synth.poisson_weights(n, seed=seed)
    return f, w


@pytest.mark.parametrize("path", ["real", "complex", "composed"])
def test_poisson_256_forward_and_gradient(ws, path):
    """Poisson solve on 256^3: u vs the FP64 operator, and d(sum u*w)/df vs the
    closed form (the operator is self-adjoint, so the gradient is the operator
    applied to w); the half-spectrum solve (the default), the complex one
    and the composed one."""
    n = 256
    f, w = _poisson_inputs(n, 4)
    fg = torch.from_numpy(f.astype(np.float32)).cuda().requires_grad_(True)
    wt = torch.from_numpy(w.astype(np.float32)).cuda()
    u = ws.poisson_solve(fg, path=path)
    (u * wt).sum().backward()
    u_ref = oracle.poisson_apply(f.astype(np.float32).astype(np.float64))
    g_ref = oracle.poisson_loss_grad(w.astype(np.float32).astype(np.float64))
    eu = rel_l2(to_host(u), u_ref)
    eg = rel_l2(to_host(fg.grad), g_ref)
    print(f"poisson 256^3 ({path}): u rel_l2 {eu:.3e}, grad rel_l2 {eg:.3e}")
    assert eu <= 1e-6 and eg <= 1e-6


def test_poisson_directional_fd(ws):
    """Directional central differences of the loss, accumulated in FP64, along
    smooth bump-field directions.  The solve is linear, so the difference is
    exact for any step; a unit step keeps FP32 rounding from being amplified."""
    n = 64
    f, w = _poisson_inputs(n, 11)
    ft = torch.from_numpy(f.astype(np.float32)).cuda()
    wt = torch.from_numpy(w.astype(np.float32)).cuda()
    fg = ft.clone().requires_grad_(True)
    (ws.poisson_solve(fg) * wt).sum().backward()
    g = to_host(fg.grad).astype(np.float64)

    def L(x):
        return float(np.sum(to_host(ws.poisson_solve(x)).astype(np.float64) * w.astype(np.float32)))

    h = 1.0
    for s in range(4):
        v = synth.gaussian_bumps(n, 8, 0.1, seed=200 + s)
        v /= np.abs(v).max()
        vt = torch.from_numpy(v.astype(np.float32)).cuda()
        fd = (L(ft + h * vt) - L(ft - h * vt)) / (2 * h)
        an = float(np.sum(g * v.astype(np.float32)))
        print(f"direction {s}: fd {fd:.6e} analytic {an:.6e}")
        assert abs(fd - an) <= 1e-3 * abs(an) + 1e-6


def test_poisson_256_directional_fd_h1e3(ws):
    """The workload's own check: central differences with h = 1e-3 on the
    256^3 grid (64 bumps, seed 4) along four smooth bump-field directions,
    the loss accumulated in FP64 on the host, against <grad, v> from the
    backward pass.  The loss is linear in f, so the difference has no
    truncation error; what remains is FP32 rounding of f +- h v and of u."""
    n = 256
    f, w = _poisson_inputs(n, 4)
    ft = torch.from_numpy(f.astype(np.float32)).cuda()
    w32 = w.astype(np.float32)
    wt = torch.from_numpy(w32).cuda()
    fg = ft.clone().requires_grad_(True)
    (ws.poisson_solve(fg) * wt).sum().backward()
    g = to_host(fg.grad).astype(np.float64)

    def L(x):
        return float(np.sum(to_host(ws.poisson_solve(x)).astype(np.float64) * w32))

    h = 1e-3
    for s in range(4):
        v = synth.gaussian_bumps(n, 8, 0.1, seed=300 + s)
        v /= np.abs(v).max()
        v32 = v.astype(np.float32)
        vt = torch.from_numpy(v32).cuda()
        fd = (L(ft + h * vt) - L(ft - h * vt)) / (2 * h)
        an = float(np.sum(g * v32))
        print(f"256^3 h=1e-3 direction {s}: fd {fd:.6e} analytic {an:.6e} rel {abs(fd - an) / abs(an):.2e}")
        assert abs(fd - an) <= 1e-3 * abs(an)


def test_poisson_per_coordinate_fd_small(ws):
    n = 16
    f, w = _poisson_inputs(n, 12)
    ft = torch.from_numpy(f.astype(np.float32)).cuda()
    fg = ft.clone().requires_grad_(True)
    wt = torch.from_numpy(w.astype(np.float32)).cuda()
    (ws.poisson_solve(fg) * wt).sum().backward()
    g = to_host(fg.grad)
    rng = np.random.default_rng(0)
    h = 1.0   # linear map: exact for any step
    for _ in range(8):
        idx = tuple(int(i) for i in rng.integers(0, n, 3))
        e = torch.zeros_like(ft)
        e[idx] = h
        lp = float(np.sum(to_host(ws.poisson_solve(ft + e)).astype(np.float64) * w.astype(np.float32)))
        lm = float(np.sum(to_host(ws.poisson_solve(ft - e)).astype(np.float64) * w.astype(np.float32)))
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[idx]) <= 2e-3 * max(1.0, abs(g[idx]))


# --- the fused solve (wsfft_poisson_solve: six passes, no elementwise passes) --------

@pytest.mark.parametrize("path", ["real", "complex"])
@pytest.mark.parametrize("shape", [(64, 64, 64), (32, 64, 128), (256, 32, 64), (128, 96, 48), (32, 8, 1024)],
                         ids=lambda s: "x".join(map(str, s)))
def test_poisson_fused_matches_fp64_operator(ws, shape, path):
    """The fused solve (five half-spectrum passes with a real plan, six
    complex passes with a complex plan) and the composed one against the
    FP64 operator."""
    nz, ny, nx = shape
    if path == "complex" and not ws._poisson_fused_supported(shape):
        pytest.skip("no fused complex kernels for this grid")
    f = synth.normal_c(shape, seed=21).real
    ft = torch.from_numpy(f.astype(np.float32)).cuda()
    u = ws.poisson_solve(ft, path=path)
    u_ref = oracle.poisson_apply(f.astype(np.float32).astype(np.float64))
    e = rel_l2(to_host(u), u_ref)
    print(f"fused poisson ({path}) {shape}: rel_l2 {e:.3e}")
    assert e <= 1e-6
    u_c = ws.poisson_solve(ft, fused=False)        # composed from the plan and the pointwise kernels
    assert rel_l2(to_host(u_c), u_ref) <= 1e-6


def test_poisson_fused_gradient_and_in_place(ws):
    n = 64
    f, w = _poisson_inputs(n, 22)
    fg = torch.from_numpy(f.astype(np.float32)).cuda().requires_grad_(True)
    wt = torch.from_numpy(w.astype(np.float32)).cuda()
    (ws.poisson_solve(fg) * wt).sum().backward()
    g_ref = oracle.poisson_loss_grad(w.astype(np.float32).astype(np.float64))
    assert rel_l2(to_host(fg.grad), g_ref) <= 1e-6
    # f and u may be the same array, with a complex plan (work: the grid in
    # complex64) and with a real plan (work: the half spectrum)
    want = oracle.poisson_apply(f.astype(np.float32).astype(np.float64))
    x = torch.from_numpy(f.astype(np.float32)).cuda()
    plan = ws.Plan(n, n, n, "c64", -1, ws.FLAG_NO_PLANE)
    work = torch.empty(x.shape, dtype=torch.complex64, device="cuda")
    assert ws._poisson_solve(plan.handle, x.data_ptr(), x.data_ptr(), work.data_ptr(), ws._stream(None)) == 0
    # a complex plan with a fused plane pass has no six-pass solve
    assert ws._poisson_solve(ws.Plan(n, n, n, "c64", -1).handle, x.data_ptr(), x.data_ptr(), work.data_ptr(),
                             ws._stream(None)) == 2
    assert rel_l2(to_host(x), want) <= 1e-6
    x = torch.from_numpy(f.astype(np.float32)).cuda()
    rp = ws.RealPlan(n, n, n)
    work = torch.empty((n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
    assert ws._poisson_solve(rp.handle, x.data_ptr(), x.data_ptr(), work.data_ptr(), ws._stream(None)) == 0
    assert rel_l2(to_host(x), want) <= 1e-6


def test_poisson_unsupported_grid_composes(ws):
    shape = (48, 32, 96)                  # (nz, ny, nx): no fused z pass of 48 points, no fused 96-point x pass
    nz, ny, nx = shape
    f = synth.normal_c(shape, seed=23).real.astype(np.float32)
    ft = torch.from_numpy(f).cuda()
    plan = ws.get_plan(torch.empty(shape, dtype=torch.complex64, device="cuda"), -1)
    work = torch.empty(shape, dtype=torch.complex64, device="cuda")
    u = torch.empty_like(ft)
    assert ws._poisson_solve(plan.handle, ft.data_ptr(), u.data_ptr(), work.data_ptr(), ws._stream(None)) == 2
    rp = ws.RealPlan(nx, ny, nz)
    assert ws._poisson_solve(rp.handle, ft.data_ptr(), u.data_ptr(), work.data_ptr(), ws._stream(None)) == 2
    assert rel_l2(to_host(ws.poisson_solve(ft)), oracle.poisson_apply(f.astype(np.float64))) <= 1e-6
