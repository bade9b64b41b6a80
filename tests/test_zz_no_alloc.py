"""wsfft_poisson_solve_noalloc (work memory from the library's static
device buffer) against wsfft_poisson_solve with a caller-allocated work
array, through the C-ABI: two calls in a row, the second on a smaller grid,
with a real plan and with a complex plan; and the size limit."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import need_gpu, rel_l2, to_host

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 72 << 20


@pytest.fixture(scope="module")
def ws():
    return need_gpu()


def _solve_both(ws, plan, shape, work_shape, seed):
    f = torch.from_numpy(synth.normal_c(shape, seed=seed).real.astype(np.float32)).cuda()
    st = ws._stream(None)
    work = torch.empty(work_shape, dtype=torch.complex64, device="cuda")
    u_ref = torch.empty_like(f)
    assert ws._poisson_solve(plan.handle, f.data_ptr(), u_ref.data_ptr(), work.data_ptr(), st) == 0
    u = torch.full_like(f, float("nan"))
    assert ws._poisson_solve_noalloc(plan.handle, f.data_ptr(), u.data_ptr(), st) == 0
    a, b = to_host(u), to_host(u_ref)
    print(f"{shape}: rel_l2 {rel_l2(a, b):.3e}, bitwise equal {np.array_equal(a, b)}")
    assert np.isfinite(a).all()
    assert rel_l2(a, b) <= 1e-6


@pytest.mark.parametrize("kind", ["real", "complex"])
def test_noalloc_matches_solve_two_calls(ws, kind):
    # (nz, ny, nx); the first fills most of the buffer, the second is smaller
    shapes = [(256, 256, 256), (64, 32, 128)] if kind == "real" else [(128, 128, 256), (32, 64, 64)]
    for i, (nz, ny, nx) in enumerate(shapes):
        if kind == "real":
            plan = ws.RealPlan(nx, ny, nz)
            wshape = (nz, ny, nx // 2 + 1)
        else:
            plan = ws.Plan(nx, ny, nz, "c64", -1, ws.FLAG_NO_PLANE)   # the six-pass complex solve
            wshape = (nz, ny, nx)
        assert 8 * int(np.prod(wshape)) <= SCRATCH_BYTES
        _solve_both(ws, plan, (nz, ny, nx), wshape, seed=60 + i)


def test_noalloc_rejects_grids_beyond_the_buffer(ws):
    plan = ws.RealPlan(512, 256, 256)          # 257*256*256*8 bytes > 72 MiB
    f = torch.zeros((256, 256, 512), dtype=torch.float32, device="cuda")
    assert ws._poisson_solve_noalloc(plan.handle, f.data_ptr(), f.data_ptr(), ws._stream(None)) == 10
