"""The Infinity Cache policy of complex64 plans: cached passes for arrays of
64-128 MiB, cached x stores up to 256 MiB, and x/y passes in plane chunks
beyond.  The cached kernels run the same arithmetic as the streaming ones,
so every call is compared bitwise with the same call on a plan made with
FLAG_STREAMING (which the oracle parity tests of the other files pin); the
schedule each size takes is checked in the plan description."""
import pytest
import torch

import synth
from gpu_helpers import need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    return need_gpu()


# (nx, ny, nz), expected schedule: the labels of the x, y, z passes and the
# chunk size (planes) of the x and y passes
CASES = [
    ((256, 256, 64), ("contig", "strided", "strided"), 0),               # 32 MiB: streaming
    ((256, 256, 256), ("cached-contig", "cached-strided", "cached-strided"), 0),   # 128 MiB
    ((512, 512, 96), ("cached-store-contig", "strided", "strided"), 0),  # 192 MiB
    ((512, 512, 512), ("cached-store-contig", "strided", "strided"), 128),   # 2 GiB: 4 chunks
    ((256, 256, 768), ("cached-store-contig", "strided", "strided"), 384),   # 384 MiB: 2 chunks
    ((384, 384, 576), ("cached-store-contig", "strided", "strided"), 192),   # 648 MiB: 3 chunks
]


def labels(desc):
    """The layout label of each pass in a plan description, in order."""
    out = []
    for part in desc.split("[")[1:]:
        out.append(part.split(" ")[0])
    return tuple(out)


@pytest.mark.parametrize("shape,want,chunk", CASES, ids=["x".join(map(str, c[0])) for c in CASES])
def test_cache_policy_bitwise_equal_to_streaming(ws, shape, want, chunk):
    nx, ny, nz = shape
    x = torch.from_numpy(synth.normal_c64((nz, ny, nx), seed=11)).cuda()
    p = ws.Plan(nx, ny, nz, "c64", -1)
    q = ws.Plan(nx, ny, nz, "c64", -1, flags=ws.FLAG_STREAMING)
    d = p.describe()
    print(d)
    assert labels(d) == want, d
    if chunk:
        assert f"chunks of {chunk} planes" in d, d
    else:
        assert "chunks" not in d, d
    assert "cached" not in q.describe() and "chunks" not in q.describe()
    for call in ("execute", "execute_adjoint", "execute_inverse"):
        got = getattr(p, call)(x)
        ref = getattr(q, call)(x)
        torch.cuda.synchronize()
        assert torch.equal(torch.view_as_real(got), torch.view_as_real(ref)), call
        del got, ref
    # in place (the chunks of the x pass overwrite what they read)
    y1 = x.clone()
    y2 = x.clone()
    p.execute(y1, out=y1)
    q.execute(y2, out=y2)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(y1), torch.view_as_real(y2))
    # every pass alone, in order, equals the full call (the chunked passes
    # run over the whole array there)
    z = torch.empty_like(x)
    for i in range(p.num_passes):
        p.execute_pass(i, x, z)
    ref = q.execute(x)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(z), torch.view_as_real(ref))


def test_streaming_flag_only_for_what_it_names(ws):
    # accepted for every storage type; a 64^3 array takes no cache policy
    p = ws.Plan(64, 64, 64, "fp16", -1, flags=ws.FLAG_STREAMING)
    assert "cached" not in p.describe()


# 16-bit storage: cached-store x kernels only, so 512^3 (512 MiB) takes two
# chunks of 256 planes, and a 128 MiB array (which complex64 would run with
# cached loads and stores) stays streaming
@pytest.mark.parametrize("dtype,flags", [("fp16", 0), ("bf16", 0), ("fp16", 4)], ids=["fp16", "bf16", "fp16-math"])
@pytest.mark.parametrize("shape,want,chunk", [
    ((512, 512, 512), ("cached-store-contig", "strided", "strided"), 256),
    ((256, 256, 512), ("contig", "strided", "strided"), 0),
], ids=["512x512x512", "256x256x512"])
def test_cache_policy_16bit_bitwise_equal_to_streaming(ws, dtype, flags, shape, want, chunk):
    nx, ny, nz = shape
    tdt = torch.float16 if dtype == "fp16" else torch.bfloat16
    g = torch.Generator(device="cuda")
    g.manual_seed(12)
    x = (0.5 * torch.randn((nz, ny, nx, 2), generator=g, device="cuda")).to(tdt)
    p = ws.Plan(nx, ny, nz, dtype, -1, flags=flags)
    q = ws.Plan(nx, ny, nz, dtype, -1, flags=flags | ws.FLAG_STREAMING)
    d = p.describe()
    print(d)
    assert labels(d) == want, d
    assert (f"chunks of {chunk} planes" in d) if chunk else ("chunks" not in d), d
    for call in ("execute", "execute_inverse"):
        got = getattr(p, call)(x)
        ref = getattr(q, call)(x)
        torch.cuda.synchronize()
        assert torch.equal(got.view(torch.int16), ref.view(torch.int16)), call
        del got, ref
    y1 = x.clone()
    y2 = x.clone()
    p.execute(y1, out=y1)
    q.execute(y2, out=y2)
    torch.cuda.synchronize()
    assert torch.equal(y1.view(torch.int16), y2.view(torch.int16))



def test_batched_plans_with_cache_policy_match_single_calls(ws):
    """Plans of either policy mode inside wsfft_execute_batched (their cached
    kernels in merged launches; a chunked plan's passes over whole arrays)
    give the same bits as each plan's own call."""
    shapes = [(256, 256, 256), (512, 512, 96), (512, 512, 512), (64, 64, 64)]
    plans = [ws.Plan(nx, ny, nz, "c64", -1) for nx, ny, nz in shapes]
    xs = [torch.from_numpy(synth.normal_c64((nz, ny, nx), seed=20 + i)).cuda() for i, (nx, ny, nz) in enumerate(shapes)]
    ys = [torch.empty_like(x) for x in xs]
    for adjoint in (False, True):
        ws.execute_batched(plans, xs, ys, adjoint=adjoint)
        for p, x, y in zip(plans, xs, ys):
            ref = p.execute_adjoint(x) if adjoint else p.execute(x)
            torch.cuda.synchronize()
            assert torch.equal(torch.view_as_real(y), torch.view_as_real(ref)), (p.describe(), adjoint)
