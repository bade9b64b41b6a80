"""Canary checks: every entry point writes only inside its output (and, where
the interface says so, its work or in-place input) array.  Each array sits
between guard regions of known bytes inside one device allocation; after the
call every guard byte must be unchanged, and an input the interface leaves
alone must be bitwise unchanged.  Covers out-of-place and in-place complex
plans, split axes (four-step) with and without the plan's work buffer, 16-bit
storage, the batched calls, the real transforms and the Poisson solve."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import need_gpu

pytestmark = pytest.mark.gpu

GUARD = 1 << 20       # bytes before, between and after the arrays
PATTERN = 0xA5


@pytest.fixture(scope="module")
def ws():
    return need_gpu()


class Arena:
    """Arrays carved out of one allocation, each followed by a guard region."""

    def __init__(self, sizes):
        self.offs = []
        off = GUARD
        for n in sizes:
            self.offs.append((off, n))
            off += (n + 255) // 256 * 256 + GUARD
        self.buf = torch.full((off,), PATTERN, dtype=torch.uint8, device="cuda")

    def view(self, i, dtype, shape):
        off, n = self.offs[i]
        return self.buf[off:off + n].view(dtype).view(shape)

    def guards_intact(self) -> bool:
        torch.cuda.synchronize()
        mask = torch.ones_like(self.buf, dtype=torch.bool)
        for off, n in self.offs:
            mask[off:off + n] = False
        return bool((self.buf[mask] == PATTERN).all())


def c64(shape, seed):
    return torch.from_numpy(synth.normal_c(shape, seed=seed).astype(np.complex64)).cuda()


@pytest.mark.parametrize("shape", [(32, 48, 64), (1, 1, 65536), (1, 8192, 16), (2048, 2048, 4), (3, 27, 96)],
                         ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("in_place", [False, True], ids=["out-of-place", "in-place"])
def test_complex_plans(ws, shape, in_place):
    nz, ny, nx = shape
    nb = nx * ny * nz * 8
    ar = Arena([nb] if in_place else [nb, nb])
    x = ar.view(0, torch.complex64, shape)
    x.copy_(c64(shape, seed=nx + ny))
    before = x.clone()
    p = ws.Plan(nx, ny, nz, "c64", -1)
    y = x if in_place else ar.view(1, torch.complex64, shape)
    for call in (p.execute, p.execute_adjoint, p.execute_inverse):
        call(x, out=y)
        assert ar.guards_intact(), call.__name__
        if not in_place:
            assert torch.equal(x, before), f"{call.__name__} wrote its input"
    for i in range(p.num_passes):
        p.execute_pass(i, x, y)
        assert ar.guards_intact(), f"pass {i}"


@pytest.mark.parametrize("kind", ["fp16", "bf16"])
def test_16bit_in_place(ws, kind):
    shape = (16, 512, 64)
    nb = 16 * 512 * 64 * 4
    ar = Arena([nb])
    x = ar.view(0, torch.float16 if kind == "fp16" else torch.bfloat16, shape + (2,))
    x.copy_(torch.randn(shape + (2,), device="cuda"))
    p = ws.Plan(64, 512, 16, kind, -1)
    p.execute(x, out=x)
    p.execute_inverse(x, out=x)
    assert ar.guards_intact()


def test_batched_and_persistent(ws):
    shapes = [(32, 64, 96), (256, 32, 32), (128, 96, 64), (64, 1, 256)]
    sizes = [nx * ny * nz * 8 for nx, ny, nz in shapes]
    ar = Arena(sizes + sizes)
    plans = [ws.Plan(nx, ny, nz, "c64", -1) for nx, ny, nz in shapes]
    xs = [ar.view(i, torch.complex64, (nz, ny, nx)) for i, (nx, ny, nz) in enumerate(shapes)]
    ys = [ar.view(len(shapes) + i, torch.complex64, (nz, ny, nx)) for i, (nx, ny, nz) in enumerate(shapes)]
    for i, x in enumerate(xs):
        x.copy_(c64(x.shape, seed=70 + i))
    before = [x.clone() for x in xs]
    ws.execute_batched(plans, xs, ys)
    assert ar.guards_intact()
    assert all(torch.equal(x, b) for x, b in zip(xs, before))
    bp = ws.BatchPlan(plans, xs, ys)
    bp.execute()
    assert ar.guards_intact() and not bp.timed_out()
    assert all(torch.equal(x, b) for x, b in zip(xs, before))
    bp.close()
    ws.execute_batched(plans, xs, xs)              # in place
    assert ar.guards_intact()


@pytest.mark.parametrize("shape", [(64, 48, 96), (4, 2048, 16), (1, 1, 32768)], ids=lambda s: "x".join(map(str, s)))
def test_real_transforms(ws, shape):
    nz, ny, nx = shape
    hshape = (nz, ny, nx // 2 + 1)
    ar = Arena([nx * ny * nz * 4, (nx // 2 + 1) * ny * nz * 8, nx * ny * nz * 4])
    a = ar.view(0, torch.float32, shape)
    a.copy_(torch.randn(shape, device="cuda"))
    before = a.clone()
    H = ar.view(1, torch.complex64, hshape)
    r = ar.view(2, torch.float32, shape)
    p = ws.RealPlan(nx, ny, nz)
    p.r2c(a, H)
    assert ar.guards_intact() and torch.equal(a, before)
    p.c2r(H, r, inverse=True)                      # overwrites H, writes r
    assert ar.guards_intact()


@pytest.mark.parametrize("kind", ["real", "complex"])
def test_poisson_solve(ws, kind):
    n = 64
    wbytes = (n // 2 + 1) * n * n * 8 if kind == "real" else n ** 3 * 8
    ar = Arena([n ** 3 * 4, n ** 3 * 4, wbytes])
    f = ar.view(0, torch.float32, (n, n, n))
    f.copy_(torch.randn((n, n, n), device="cuda"))
    before = f.clone()
    u = ar.view(1, torch.float32, (n, n, n))
    work = ar.view(2, torch.complex64, (-1,))
    plan = ws.RealPlan(n, n, n) if kind == "real" else ws.Plan(n, n, n, "c64", -1, ws.FLAG_NO_PLANE)
    assert ws._poisson_solve(plan.handle, f.data_ptr(), u.data_ptr(), work.data_ptr(), ws._stream(None)) == 0
    assert ar.guards_intact() and torch.equal(f, before)
