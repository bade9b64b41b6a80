"""wsfft_execute_batched: many transforms in one call, each checked element by
element against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import need_gpu, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu
TOL = 1e-6


@pytest.fixture(scope="module")
def ws():
    return need_gpu()


def test_96_uneven_arrays(ws):
    """96 non-cubic arrays, each axis from {32, 64, 96, 128, 256}, U[-1,1), seed 3."""
    shapes = synth.batched_shapes(96, seed=3)
    arrays = synth.batched_arrays(shapes, seed=3)
    plans = [ws.Plan(nx, ny, nz, "c64", -1) for nx, ny, nz in shapes]
    xs = [to_dev(a) for a in arrays]
    ys = [torch.empty_like(x) for x in xs]
    ws.execute_batched(plans, xs, ys)
    torch.cuda.synchronize()
    worst = 0.0
    for a, y in zip(arrays, ys):
        e = rel_l2(y.cpu().numpy(), oracle.fftn(a.astype(np.complex64).astype(np.complex128), -1))
        worst = max(worst, e)
    print(f"96 arrays, {sum(a.size for a in arrays)} elements, worst rel_l2 {worst:.3e}")
    assert worst <= TOL


def test_tune_batched_then_execute(ws):
    """Batch-level tuning times each merged launch in every launch variant and
    records the fastest; the following batched calls run the recorded variants
    and still match the oracle, in both directions."""
    shapes = [(64, 128, 32), (64, 128, 32), (128, 64, 64), (128, 64, 64), (256, 32, 64), (256, 32, 64),
              (64, 256, 128), (64, 256, 128)]
    arrays = [synth.uniform_c((nz, ny, nx), seed=40 + i) for i, (nx, ny, nz) in enumerate(shapes)]
    plans = [ws.Plan(nx, ny, nz, "c64", -1, ws.FLAG_NO_PLANE) for nx, ny, nz in shapes]
    xs = [to_dev(a) for a in arrays]
    ys = [torch.empty_like(x) for x in xs]
    ws.tune_batched(plans, xs, ys)
    ws.tune_batched(plans, xs, ys, adjoint=True)
    for adjoint in (False, True):
        ws.execute_batched(plans, xs, ys, adjoint=adjoint)
        torch.cuda.synchronize()
        for a, y in zip(arrays, ys):
            want = oracle.fftn(a.astype(np.complex64).astype(np.complex128), +1 if adjoint else -1)
            assert rel_l2(y.cpu().numpy(), want) <= TOL
    # inputs are left alone (in != out)
    for a, x in zip(arrays, xs):
        assert np.array_equal(to_host(x), a.astype(np.complex64))


def test_batched_adjoint_matches_single_calls(ws):
    shapes = [(32, 64, 96), (96, 32, 32), (128, 32, 64), (64, 96, 32)]
    plans = [ws.Plan(*s, "c64", -1) for s in shapes]
    xs = [to_dev(synth.uniform_c((s[2], s[1], s[0]), seed=i)) for i, s in enumerate(shapes)]
    ys = [torch.empty_like(x) for x in xs]
    ws.execute_batched(plans, xs, ys, adjoint=True)
    for p, x, y in zip(plans, xs, ys):
        single = p.execute_adjoint(x)
        torch.cuda.synchronize()
        assert torch.equal(single, y)


PLANE_SHAPES = [(32, 32), (32, 64), (64, 32), (32, 96), (96, 32), (32, 128), (128, 32), (32, 256), (256, 32),
                (64, 64), (64, 96), (96, 64), (64, 128), (128, 64),
                (96, 96), (128, 96), (96, 128), (128, 128), (64, 256), (256, 64)]


@pytest.mark.parametrize("adjoint", [False, True], ids=["forward", "adjoint"])
@pytest.mark.parametrize("in_place", [False, True], ids=["out-of-place", "in-place"])
def test_mixed_plane_shapes_match_single_calls(ws, adjoint, in_place):
    """Every fused plane shape in one batch (the 9216- to 16384-value ones in
    1024-thread workgroups), 35 arrays of the 8192-value shapes among them
    (more than one mixed-shape launch holds), plus arrays without a plane
    pass: each result equals the array's own plan call bitwise, and the
    oracle for a few."""
    shapes = [(nx, ny, 1 + i % 3) for i, (nx, ny) in enumerate(PLANE_SHAPES)]
    big = [(32, 256), (256, 32), (64, 128), (128, 64)]
    shapes += [(*big[i % 4], 1 + i % 2) for i in range(35)]
    shapes += [(512, 8, 3), (16, 16, 4), (4096, 1, 1)]
    plans = [ws.Plan(nx, ny, nz, "c64", -1) for nx, ny, nz in shapes]
    arrays = [synth.uniform_c((nz, ny, nx), seed=300 + i).astype(np.complex64) for i, (nx, ny, nz) in enumerate(shapes)]
    xs = [to_dev(a) for a in arrays]
    ys = xs if in_place else [torch.empty_like(x) for x in xs]
    singles = []
    for p, a in zip(plans, arrays):
        x1 = to_dev(a)
        singles.append(p.execute_adjoint(x1) if adjoint else p.execute(x1))
    ws.execute_batched(plans, xs, ys, adjoint=adjoint)
    torch.cuda.synchronize()
    for i, (y, single) in enumerate(zip(ys, singles)):
        assert torch.equal(y, single), f"entry {i} shape {shapes[i]}"
    for i in (0, 8, 13, 14, 17, 19, 20, len(shapes) - 3):
        want = oracle.fftn(arrays[i].astype(np.complex128), +1 if adjoint else -1)
        assert rel_l2(to_host(ys[i]), want) <= TOL


def test_uniform_batch_is_one_array_per_entry(ws):
    """Same plan, buffers one array apart: the single-launch path."""
    n, count = 4096, 64
    a = synth.normal_c((count, n), seed=5).astype(np.complex64)
    x = to_dev(a)
    y = torch.empty_like(x)
    p = ws.Plan(n, 1, 1, "c64", -1)
    ws.execute_batched([p] * count, list(x), list(y))
    assert rel_l2(to_host(y), oracle.fft1d_batch(a.astype(np.complex128), -1)) <= TOL


def test_batch_of_3d_plans_uniform(ws):
    shape = (32, 48, 64)
    count = 5
    a = synth.uniform_c((count * 64, 48, 32), seed=6).astype(np.complex64)
    x = to_dev(a)
    y = torch.empty_like(x)
    p = ws.Plan(*shape, "c64", +1)
    xs, ys = list(x.view(count, -1)), list(y.view(count, -1))
    ws.execute_batched([p] * count, xs, ys)
    yh = to_host(y).reshape(count, 64, 48, 32)
    for i in range(count):
        ref = oracle.fftn(a.reshape(count, 64, 48, 32)[i].astype(np.complex128), +1)
        assert rel_l2(yh[i], ref) <= TOL


def test_batched_rejects_mixed_dtypes(ws):
    p1 = ws.Plan(32, 32, 1, "c64")
    p2 = ws.Plan(32, 32, 1, "fp16")
    x1 = torch.zeros((32, 32), dtype=torch.complex64, device="cuda")
    x2 = torch.zeros((32, 32, 2), dtype=torch.float16, device="cuda")
    with pytest.raises(ws.WsfftError) as ei:
        ws.execute_batched([p1, p2], [x1, x2], [x1.clone(), x2.clone()])
    assert ei.value.status == 1


def test_graph_capture_replays(ws):
    """The batched call captured into a HIP graph and replayed several times,
    with eager work between replays, matches the eager result every time."""
    shapes = [(64, 32, 96), (32, 96, 64), (96, 64, 32)]
    plans = [ws.Plan(*s, "c64", -1) for s in shapes]
    xs = [to_dev(synth.uniform_c((s[2], s[1], s[0]), seed=10 + i)) for i, s in enumerate(shapes)]
    ys = [torch.empty_like(x) for x in xs]
    ws.execute_batched(plans, xs, ys)
    torch.cuda.synchronize()
    eager = [y.clone() for y in ys]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for y in ys:
            y.zero_()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            ws.execute_batched(plans, xs, ys, stream=s)
    for rep in range(4):
        for y in ys:
            y.fill_(float(rep))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for y, e in zip(ys, eager):
            assert torch.equal(y, e), f"replay {rep}"


# --- one persistent launch per batch (batch plans) ----------------------------------

def test_batch_plan_96_uneven_one_launch(ws):
    shapes = synth.batched_shapes(96, seed=3)
    arrays = synth.batched_arrays(shapes, seed=3)
    plans = [ws.Plan(nx, ny, nz, "c64", -1) for nx, ny, nz in shapes]
    xs = [to_dev(a) for a in arrays]
    ys = [torch.empty_like(x) for x in xs]
    bp = ws.BatchPlan(plans, xs, ys)
    assert bp.tiles > 0
    for rep in range(3):          # counters reset themselves between launches
        for y in ys:
            y.fill_(float(rep + 1))
        bp.execute()
        torch.cuda.synchronize()
        assert not bp.timed_out()
        worst = 0.0
        for a, y in zip(arrays, ys):
            worst = max(worst, rel_l2(y.cpu().numpy(), oracle.fftn(a.astype(np.complex64).astype(np.complex128), -1)))
        print(f"batch plan, launch {rep}: {bp.tiles} tiles, worst rel_l2 {worst:.3e}")
        assert worst <= TOL


def test_batch_plan_adjoint_in_place_and_graph(ws):
    shapes = [(32, 64, 96), (256, 32, 32), (128, 96, 64), (64, 1, 256), (96, 32, 1)]
    plans = [ws.Plan(*s, "c64", -1) for s in shapes]
    arrays = [synth.uniform_c((s[2], s[1], s[0]), seed=40 + i).astype(np.complex64) for i, s in enumerate(shapes)]
    xs = [to_dev(a) for a in arrays]
    bp = ws.BatchPlan(plans, xs, xs, adjoint=True)       # in place
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            bp.execute(stream=s)
    # the input is restored before each replay, so every replay gives the adjoint of the input
    for rep in range(3):
        for x, a in zip(xs, arrays):
            x.copy_(torch.from_numpy(a))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert not bp.timed_out()
        for x, a in zip(xs, arrays):
            assert rel_l2(to_host(x), oracle.fftn(a.astype(np.complex128), +1)) <= TOL, f"replay {rep}"


def test_batch_plan_rejects_unsupported(ws):
    p = ws.Plan(512, 512, 1, "c64", -1)          # 512 has no persistent branch
    x = torch.zeros((512, 512), dtype=torch.complex64, device="cuda")
    with pytest.raises(ws.WsfftError) as ei:
        ws.BatchPlan([p], [x], [x.clone()])
    assert ei.value.status == 2
    p1, p2 = ws.Plan(32, 32, 1, "c64", -1), ws.Plan(32, 32, 1, "c64", +1)
    y = torch.zeros((32, 32), dtype=torch.complex64, device="cuda")
    with pytest.raises(ws.WsfftError) as ei:
        ws.BatchPlan([p1, p2], [y, y.clone()], [y.clone(), y.clone()])
    assert ei.value.status == 1


def test_batch_plan_timeout_is_per_launch(ws):
    """A launch whose dependency waits give up (forced from the host with a
    spin limit of 0 polls: the launch still runs every tile and exits) is
    reported by the check, and the next launch waits normally again and is
    correct: the timeout record does not carry over into later launches."""
    shapes = synth.batched_shapes(96, seed=3)
    arrays = synth.batched_arrays(shapes, seed=3)
    plans = [ws.Plan(nx, ny, nz, "c64", -1) for nx, ny, nz in shapes]
    xs = [to_dev(a) for a in arrays]
    ys = [torch.empty_like(x) for x in xs]
    bp = ws.BatchPlan(plans, xs, ys)
    bp.set_spin_limit(0)
    bp.execute()
    torch.cuda.synchronize()
    assert bp.timed_out()          # thousands of first-level tiles are still in flight at the first wait
    assert not bp.timed_out()      # the check clears the record
    bp.set_spin_limit(1 << 22)
    for y in ys:
        y.fill_(0.0)
    bp.execute()
    torch.cuda.synchronize()
    assert not bp.timed_out()
    worst = max(rel_l2(to_host(y), oracle.fftn(a.astype(np.complex64).astype(np.complex128), -1))
                for a, y in zip(arrays, ys))
    assert worst <= TOL
