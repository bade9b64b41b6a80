"""Parity of the HIP path (through the C-ABI) with the FP64 oracle, element
by element.  Bound: relative L2 <= 1e-6 for complex64 (round trip <= 2e-6)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import need_gpu, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-6
TOL_RT = 2e-6


@pytest.fixture(scope="module")
def ws():
    return need_gpu()


def run_plan(ws, a, sign=-1, mode="execute"):
    nz, ny, nx = a.shape
    p = ws.Plan(nx, ny, nz, "c64", sign)
    y = getattr(p, mode)(to_dev(a))
    return to_host(y), p


def test_32cubed_forward(ws):
    """Plain forward 32^3, re/im U[-1,1), seed 0."""
    a = synth.uniform_c((32, 32, 32), seed=0).astype(np.complex64)
    y, p = run_plan(ws, a)
    e = rel_l2(y, oracle.fftn(a.astype(np.complex128), -1))
    print(f"32^3 fwd rel_l2 {e:.3e}  {p.describe()}")
    assert e <= TOL


# (nx, ny, nz): tiles with ragged tails, radix 3, length-1 axes, the longest
# one-pass pencils of each layout, tiny axes
SHAPES = [
    (2, 1, 1), (3, 1, 1), (4, 2, 3), (6, 9, 12), (16, 16, 16), (24, 27, 16),
    (48, 36, 18), (96, 32, 12), (12, 96, 32), (64, 128, 256), (256, 64, 32),
    (27, 54, 81), (1, 1, 96), (1, 512, 1), (1, 2, 768), (1024, 1, 1), (16384, 1, 1),
    (8, 1024, 4), (2, 3, 1024), (243, 8, 9), (128, 128, 1), (2, 2, 2),
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("sign", [-1, 1])
def test_shapes_forward(ws, shape, sign):
    nx, ny, nz = shape
    a = synth.uniform_c((nz, ny, nx), seed=nx + 7 * ny + 31 * nz).astype(np.complex64)
    y, _ = run_plan(ws, a, sign)
    assert rel_l2(y, oracle.fftn(a.astype(np.complex128), sign)) <= TOL


@pytest.mark.parametrize("shape", [(16, 16, 16), (96, 32, 12), (27, 54, 81), (4096, 1, 1)], ids=str)
def test_adjoint_and_inverse(ws, shape):
    nx, ny, nz = shape
    a = synth.normal_c((nz, ny, nx), seed=3).astype(np.complex64)
    a128 = a.astype(np.complex128)
    y, p = run_plan(ws, a, -1, "execute_adjoint")
    assert rel_l2(y, oracle.fftn(a128, +1)) <= TOL
    y, p = run_plan(ws, a, -1, "execute_inverse")
    assert rel_l2(y, oracle.fftn(a128, +1) / a.size) <= TOL
    x = to_dev(a)
    r = p.execute_inverse(p.execute(x))
    assert rel_l2(to_host(r), a) <= TOL_RT


def test_dot_product_adjoint(ws):
    """<F x, y> = <x, F^H y> (FP32 bound 1e-6 relative)."""
    nx, ny, nz = 48, 32, 24
    x = to_dev(synth.normal_c((nz, ny, nx), seed=4))
    yv = to_dev(synth.normal_c((nz, ny, nx), seed=5))
    p = ws.Plan(nx, ny, nz, "c64", -1)
    Fx = p.execute(x).cpu().numpy().astype(np.complex128)
    FHy = p.execute_adjoint(yv).cpu().numpy().astype(np.complex128)
    xs, ys = x.cpu().numpy().astype(np.complex128), yv.cpu().numpy().astype(np.complex128)
    lhs, rhs = np.vdot(ys, Fx), np.vdot(FHy, xs)
    assert abs(lhs - rhs) / (np.linalg.norm(Fx) * np.linalg.norm(ys)) <= 1e-6


def test_in_place(ws):
    a = synth.uniform_c((32, 64, 96), seed=6).astype(np.complex64)
    p = ws.Plan(96, 64, 32, "c64", -1)
    x = to_dev(a)
    p.execute(x, out=x)
    assert rel_l2(to_host(x), oracle.fftn(a.astype(np.complex128))) <= TOL


def test_input_is_not_written(ws):
    a = synth.uniform_c((16, 32, 64), seed=7).astype(np.complex64)
    x = to_dev(a)
    ws.Plan(64, 32, 16, "c64", -1).execute(x)
    assert np.array_equal(to_host(x), a)


def test_identity_plan(ws):
    x = to_dev(np.array([[[1.5 - 2j]]]))
    y = ws.Plan(1, 1, 1, "c64", -1).execute(x)
    assert to_host(y)[0, 0, 0] == np.complex64(1.5 - 2j)


# --- axes split into two passes (four-step) ------------------------------------

@pytest.mark.parametrize("shape", [(65536, 1, 1), (32768, 2, 1), (8, 2048, 4), (4, 3, 2048),
                                   (2048, 2048, 1), (2, 1, 4096), (24576, 3, 1)],
                         ids=lambda s: "x".join(map(str, s)))
def test_four_step_axes(ws, shape):
    nx, ny, nz = shape
    a = synth.normal_c((nz, ny, nx), seed=8).astype(np.complex64)
    y, p = run_plan(ws, a, -1)
    print(p.describe())
    assert p.num_passes > sum(n > 1 for n in shape)
    assert rel_l2(y, oracle.fftn(a.astype(np.complex128), -1)) <= TOL
    y2, _ = run_plan(ws, a, -1, "execute_inverse")
    assert rel_l2(y2, oracle.fftn(a.astype(np.complex128), +1) / a.size) <= TOL


def test_two_split_axes_use_work_buffer(ws):
    nx, ny, nz = 4, 2048, 2048
    a = synth.normal_c((nz, ny, nx), seed=9).astype(np.complex64)
    p = ws.Plan(nx, ny, nz, "c64", -1)
    assert p.work_bytes == a.size * 8
    x = to_dev(a)
    ref = oracle.fftn(a.astype(np.complex128), -1)
    assert rel_l2(to_host(p.execute(x)), ref) <= TOL
    p.execute(x, out=x)    # in place through the work buffer
    assert rel_l2(to_host(x), ref) <= TOL


@pytest.mark.parametrize("shape", [(65536, 1, 1), (2048, 2048, 4), (8, 4096, 3)],
                         ids=lambda s: "x".join(map(str, s)))
def test_single_split_axis_in_place(ws, shape):
    """One split axis, in place: its first pass goes through the plan's work
    buffer, the rest run in place on the caller's array."""
    nx, ny, nz = shape
    a = synth.normal_c((nz, ny, nx), seed=10).astype(np.complex64)
    p = ws.Plan(nx, ny, nz, "c64", -1)
    assert p.work_bytes == a.size * 8
    x = to_dev(a)
    p.execute(x, out=x)
    ref = oracle.fftn(a.astype(np.complex128), -1)
    assert rel_l2(to_host(x), ref) <= TOL
    p.execute_inverse(x, out=x)
    assert rel_l2(to_host(x), a) <= TOL_RT


def test_2d_8192_squared_in_place(ws):
    """The 2D workload in place (its 8192-point strided axis is split)."""
    n = 8192
    a = synth.normal_c64((n, n), seed=1)
    p = ws.Plan(n, n, 1, "c64", -1)
    x = torch.from_numpy(a).cuda()
    p.execute(x, out=x)
    e = rel_l2(to_host(x), oracle.fftn(a.astype(np.complex128), -1))
    print(f"8192^2 in place rel_l2 {e:.3e}")
    assert e <= TOL


def test_batched_rejects_in_place_split_axis(ws):
    """Batched entries run pass-major, so an entry that would go through its
    plan's work buffer (one split axis, in place) is refused."""
    p = ws.Plan(65536, 1, 1, "c64", -1)
    x = to_dev(np.zeros((1, 1, 65536)))
    with pytest.raises(ws.WsfftError) as ei:
        ws.execute_batched([p], [x], [x])
    assert ei.value.status == 1


# --- full-size workloads -------------------------------------------------------------

def test_512cubed_forward_and_round_trip(ws):
    """512^3 complex64, re/im N(0,1) seed 1, every output element vs the oracle;
    launch configuration as benchmarked."""
    n = 512
    a = synth.normal_c64((n, n, n), seed=1)
    p = ws.Plan(n, n, n, "c64", -1)
    x = torch.from_numpy(a).cuda()
    y = p.execute(x)
    r = p.execute_inverse(y)
    yh, rh = to_host(y), to_host(r)
    del y, r, x
    torch.cuda.empty_cache()
    ref = oracle.fftn(a.astype(np.complex128), -1)
    e = rel_l2(yh, ref)
    del ref
    e_rt = rel_l2(rh, a)
    print(f"512^3 fwd rel_l2 {e:.3e} round trip {e_rt:.3e}  {p.describe()}")
    assert e <= TOL and e_rt <= TOL_RT


def test_2d_8192_squared(ws):
    n = 8192
    a = synth.normal_c64((n, n), seed=1)
    p = ws.Plan(n, n, 1, "c64", -1)
    yh = to_host(p.execute(torch.from_numpy(a).cuda()))
    e = rel_l2(yh, oracle.fftn(a.astype(np.complex128), -1))
    print(f"8192^2 fwd rel_l2 {e:.3e}  {p.describe()}")
    assert e <= TOL


def test_1d_batch_65536(ws):
    """Batch of 1024 pencils of length 65536 as one batched call of one plan;
    every 64th pencil checked against the oracle (CPU time)."""
    n, count = 65536, 1024
    a = synth.normal_c64((count, n), seed=1)
    p = ws.Plan(n, 1, 1, "c64", -1)
    x = torch.from_numpy(a).cuda()
    y = torch.empty_like(x)
    ws.execute_many(p, x, y, count)
    yh = to_host(y)
    sel = np.arange(0, count, 64)
    ref = oracle.fft1d_batch(a[sel].astype(np.complex128), -1)
    e = rel_l2(yh[sel], ref)
    print(f"1D 1024x65536 rel_l2 {e:.3e} (every 64th pencil)")
    assert e <= TOL


# --- limits of the axis lengths ---------------------------------------------------

@pytest.mark.parametrize("shape", [(1 << 20, 1, 1), (3 ** 12, 1, 1), (2, 6561, 3)],
                         ids=lambda s: "x".join(map(str, s)))
def test_longest_axes(ws, shape):
    """The longest axis a plan accepts (2^20, split 1024 x 1024), the longest
    pure radix-3 axis below it (3^12, split 729 x 729) and a long radix-3
    strided axis (6561 = 81 x 81)."""
    nx, ny, nz = shape
    a = synth.normal_c((nz, ny, nx), seed=12).astype(np.complex64)
    y, p = run_plan(ws, a, -1)
    e = rel_l2(y, oracle.fftn(a.astype(np.complex128), -1))
    print(f"{shape}: rel_l2 {e:.3e} [{p.describe()}]")
    assert e <= TOL
    y2, _ = run_plan(ws, a, -1, "execute_inverse")
    assert rel_l2(y2, oracle.fftn(a.astype(np.complex128), +1) / a.size) <= TOL


# --- fused x + y plane passes -------------------------------------------------------

PLANE_PAIRS = [(32, 32), (32, 64), (64, 32), (32, 96), (96, 32), (32, 128), (128, 32), (32, 256), (256, 32),
               (64, 64), (64, 96), (96, 64), (64, 128), (128, 64)]


@pytest.mark.parametrize("nx,ny", PLANE_PAIRS, ids=lambda v: str(v))
def test_plane_pass_shapes(ws, nx, ny):
    """Every (nx, ny) with a fused plane pass, with a few planes (nz = 3) and
    as a 2D array: forward, adjoint and inverse against the oracle, and the
    same bits as the separate x and y passes would give up to rounding."""
    for nz in (3, 1):
        a = synth.normal_c((nz, ny, nx), seed=nx * 7 + ny + nz).astype(np.complex64)
        p = ws.Plan(nx, ny, nz, "c64", -1)
        assert "plane" in p.describe(), p.describe()
        assert p.num_passes == (2 if nz > 1 else 1)
        x = to_dev(a)
        a64 = a.astype(np.complex128)
        assert rel_l2(to_host(p.execute(x)), oracle.fftn(a64, -1)) <= TOL
        assert rel_l2(to_host(p.execute_adjoint(x)), oracle.fftn(a64, +1)) <= TOL
        assert rel_l2(to_host(p.execute_inverse(x)), oracle.fftn(a64, +1) / a.size) <= TOL
        q = ws.Plan(nx, ny, nz, "c64", -1, ws.FLAG_NO_PLANE)
        assert "plane" not in q.describe()
        assert rel_l2(to_host(p.execute(x)), to_host(q.execute(x))) <= TOL


def test_plane_pass_in_place_and_32cubed(ws):
    """32^3 (the plain forward workload) runs as a plane pass and a z pass;
    in place as well."""
    a = synth.uniform_c((32, 32, 32), seed=0).astype(np.complex64)
    p = ws.Plan(32, 32, 32, "c64", -1)
    assert p.num_passes == 2, p.describe()
    x = to_dev(a)
    p.execute(x, out=x)
    assert rel_l2(to_host(x), oracle.fftn(a.astype(np.complex128), -1)) <= TOL
