"""Python binding of libwsfft: the MI355X multidimensional complex FFT.

Argument marshalling only -- every step of a transform runs in the HIP
kernels of ``libwsfft.so`` (built by ``python -m paper_2209_15040_amd.build``).
PyTorch supplies device memory and streams.  There is no CPU fallback: if the
library is missing, importing this package raises.

Tensor conventions (x fastest, as the C-ABI):

* complex64 tensors of shape (nz, ny, nx), (ny, nx) or (nx,);
* 16-bit storage as float16 / bfloat16 tensors with a trailing dimension of
  2 holding (re, im): shape (nz, ny, nx, 2) etc.

The names follow the C-ABI (``include/wsfft.h``): :class:`Plan` wraps
``wsfft_plan_create`` and its ``execute`` / ``execute_adjoint`` /
``execute_inverse``; :func:`execute_batched` wraps ``wsfft_execute_batched``.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwsfft.so")

C64, C16_FP16, C16_BF16 = 0, 1, 2
FLAG_FP32_TWIDDLES = 1
FLAG_TUNE = 2
FLAG_FP16_MATH = 4       # FP16 plans: packed FP16 butterfly arithmetic
FLAG_NO_PLANE = 8        # complex64 plans: keep the x and y passes separate (no fused plane pass)
FLAG_STREAMING = 16      # complex64 plans: every pass streaming, no Infinity Cache policy (no plane chunks)
DTYPES = {"c64": C64, "fp16": C16_FP16, "bf16": C16_BF16}
_TORCH_DTYPE = {C64: torch.complex64, C16_FP16: torch.float16, C16_BF16: torch.bfloat16}

STATUS = {
    0: "success", 1: "invalid value", 2: "unsupported size", 3: "null pointer",
    4: "misaligned pointer", 5: "out of device memory", 6: "no HIP device",
    7: "HIP runtime error", 8: "invalid plan", 9: "wrong device", 10: "exceeds the static scratch buffer",
}


class WsfftError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"wsfft {what}: {STATUS.get(status, status)} ({status})")


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2209_15040_amd.build` "
                      "(there is no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)
_vp, _i64, _int = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int


def _sig(name, restype, argtypes):
    fn = getattr(_lib, name)
    fn.restype = restype
    fn.argtypes = argtypes
    return fn


_plan_create_ex = _sig("wsfft_plan_create_ex", _vp, [_i64, _i64, _i64, _int, _int, ctypes.c_uint])
_get_last_error = _sig("wsfft_get_last_error", _int, [])
_execute = _sig("wsfft_execute", _int, [_vp, _vp, _vp, _vp])
_execute_adjoint = _sig("wsfft_execute_adjoint", _int, [_vp, _vp, _vp, _vp])
_execute_inverse = _sig("wsfft_execute_inverse", _int, [_vp, _vp, _vp, _vp])
_execute_batched = _sig("wsfft_execute_batched", _int,
                        [_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _int, _vp])
_tune_batched = _sig("wsfft_tune_batched", _int,
                     [_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _int, _vp])
_execute_pass = _sig("wsfft_execute_pass", _int, [_vp, _int, _int, _vp, _vp, _vp])
_scale_log2 = _sig("wsfft_plan_scale_log2", _int, [_vp])
_num_passes = _sig("wsfft_plan_num_passes", _int, [_vp])
_work_bytes = _sig("wsfft_plan_work_bytes", _i64, [_vp])
_describe = _sig("wsfft_plan_describe", _int, [_vp, ctypes.c_char_p, ctypes.c_size_t])
_destroy = _sig("wsfft_plan_destroy", None, [_vp])
_batch_create = _sig("wsfft_batch_plan_create", _vp,
                     [_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _int])
_batch_error = _sig("wsfft_batch_get_last_error", _int, [])
_batch_execute = _sig("wsfft_batch_execute", _int, [_vp, _vp])
_batch_tiles = _sig("wsfft_batch_plan_tiles", _i64, [_vp])
_batch_check = _sig("wsfft_batch_plan_check", _int, [_vp, ctypes.POINTER(_int)])
_batch_spin = _sig("wsfft_batch_plan_set_spin_limit", _int, [_vp, ctypes.c_uint])
_batch_destroy = _sig("wsfft_batch_plan_destroy", None, [_vp])
_real_to_complex = _sig("wsfft_real_to_complex", _int, [_vp, _vp, _i64, _vp])
_complex_real_part = _sig("wsfft_complex_real_part", _int, [_vp, _vp, _i64, _vp])
_poisson_symbol = _sig("wsfft_poisson_symbol", _int, [_vp, _i64, _i64, _i64, _vp])
_poisson_solve = _sig("wsfft_poisson_solve", _int, [_vp, _vp, _vp, _vp, _vp])
_poisson_solve_noalloc = _sig("wsfft_poisson_solve_noalloc", _int, [_vp, _vp, _vp, _vp])
_plan_create_real = _sig("wsfft_plan_create_real", _vp, [_i64, _i64, _i64, ctypes.c_uint])
_plan_create_real_ex = _sig("wsfft_plan_create_real_ex", _vp, [_i64, _i64, _i64, ctypes.c_uint, _i64])
_execute_r2c = _sig("wsfft_execute_r2c", _int, [_vp, _vp, _vp, _vp])
_execute_c2r = _sig("wsfft_execute_c2r", _int, [_vp, _vp, _vp, _vp])
_execute_c2r_inverse = _sig("wsfft_execute_c2r_inverse", _int, [_vp, _vp, _vp, _vp])
_plan_is_real = _sig("wsfft_plan_is_real", _int, [_vp])


def _check(st: int, what: str) -> None:
    if st != 0:
        raise WsfftError(st, what)


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def shape_xyz(shape, dtype: int):
    """(nx, ny, nz) of a tensor shape in the binding's conventions."""
    s = tuple(shape)
    if dtype != C64:
        if not s or s[-1] != 2:
            raise ValueError("16-bit storage needs a trailing (re, im) dimension of 2")
        s = s[:-1]
    if len(s) == 1:
        return s[0], 1, 1
    if len(s) == 2:
        return s[1], s[0], 1
    if len(s) == 3:
        return s[2], s[1], s[0]
    raise ValueError("rank 1..3 only")


class Plan:
    """A wsfft plan for an nx x ny x nz transform (``wsfft_plan_create_ex``).

    ``dtype``: "c64", "fp16" or "bf16" (16-bit tensors carry a trailing
    (re, im) axis).  ``flags``: FLAG_FP32_TWIDDLES, FLAG_TUNE, for "fp16"
    FLAG_FP16_MATH (packed FP16 butterflies instead of FP32 arithmetic), and
    for "c64" FLAG_NO_PLANE and FLAG_STREAMING."""

    def __init__(self, nx: int, ny: int = 1, nz: int = 1, dtype="c64", sign: int = -1, flags: int = 0):
        self.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        self.nx, self.ny, self.nz, self.sign, self.flags = int(nx), int(ny), int(nz), int(sign), int(flags)
        self.device = torch.cuda.current_device()
        h = _plan_create_ex(self.nx, self.ny, self.nz, self.dtype, self.sign, self.flags)
        if not h:
            raise WsfftError(_get_last_error(), f"plan_create({nx},{ny},{nz})")
        self._h = h

    @classmethod
    def for_tensor(cls, x: torch.Tensor, sign: int = -1, flags: int = 0) -> "Plan":
        dt = {torch.complex64: C64, torch.float16: C16_FP16, torch.bfloat16: C16_BF16}[x.dtype]
        return cls(*shape_xyz(x.shape, dt), dtype=dt, sign=sign, flags=flags)

    @property
    def handle(self) -> int:
        return self._h

    @property
    def size(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def scale_log2(self) -> int:
        return _scale_log2(self._h)

    @property
    def num_passes(self) -> int:
        return _num_passes(self._h)

    @property
    def work_bytes(self) -> int:
        return _work_bytes(self._h)

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(4096)
        _check(_describe(self._h, buf, len(buf)), "plan_describe")
        return buf.value.decode()

    def _check_tensor(self, t: torch.Tensor, name: str) -> None:
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
        if t.dtype != _TORCH_DTYPE[self.dtype]:
            raise TypeError(f"{name} has dtype {t.dtype}, plan wants {_TORCH_DTYPE[self.dtype]}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        per = 1 if self.dtype == C64 else 2
        if t.numel() != self.size * per:
            raise ValueError(f"{name} has {t.numel()} elements, plan wants {self.size * per}")

    def _run(self, fn, x, out, stream, what):
        self._check_tensor(x, "input")
        if out is None:
            out = torch.empty_like(x)
        self._check_tensor(out, "output")
        _check(fn(self._h, x.data_ptr(), out.data_ptr(), _stream(stream)), what)
        return out

    def execute(self, x, out=None, stream=None):
        """out = 2^-S * DFT with the plan's sign (unnormalised)."""
        return self._run(_execute, x, out, stream, "execute")

    def execute_adjoint(self, x, out=None, stream=None):
        """out = 2^-S * DFT with the opposite sign (unnormalised)."""
        return self._run(_execute_adjoint, x, out, stream, "execute_adjoint")

    def execute_inverse(self, x, out=None, stream=None):
        """out = 2^S / N * DFT with the opposite sign: the exact inverse of
        ``execute`` (S = 0 for complex64)."""
        return self._run(_execute_inverse, x, out, stream, "execute_inverse")

    def execute_pass(self, index: int, x, out, mode: int = 0, stream=None):
        """Only pass `index` of execute (mode 0) / adjoint (1) / inverse (2)."""
        self._check_tensor(x, "input")
        self._check_tensor(out, "output")
        _check(_execute_pass(self._h, int(index), int(mode), x.data_ptr(), out.data_ptr(), _stream(stream)),
               "execute_pass")
        return out

    def close(self) -> None:
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _batch_args(plans, ins, outs):
    n = len(plans)
    if len(ins) != n or len(outs) != n:
        raise ValueError("plans, ins and outs must have one entry each")
    for p, i, o in zip(plans, ins, outs):
        p._check_tensor(i, "input")
        p._check_tensor(o, "output")
    arr = ctypes.c_void_p * max(n, 1)
    return (n, arr(*[p.handle for p in plans]), arr(*[t.data_ptr() for t in ins]),
            arr(*[t.data_ptr() for t in outs]))


def execute_batched(plans, ins, outs, adjoint: bool = False, stream=None) -> None:
    """``wsfft_execute_batched`` over lists of plans and tensors."""
    n, ph, ip, op = _batch_args(plans, ins, outs)
    _check(_execute_batched(n, ph, ip, op, int(bool(adjoint)), _stream(stream)), "execute_batched")


def tune_batched(plans, ins, outs, adjoint: bool = False, stream=None) -> None:
    """``wsfft_tune_batched``: time each merged launch of this batch in every
    launch variant and record the fastest for later ``execute_batched`` calls
    (synchronises; `outs` hold unspecified values afterwards)."""
    n, ph, ip, op = _batch_args(plans, ins, outs)
    _check(_tune_batched(n, ph, ip, op, int(bool(adjoint)), _stream(stream)), "tune_batched")


def execute_many(plan: Plan, x: torch.Tensor, out: torch.Tensor, count: int, adjoint: bool = False,
                 stream=None) -> torch.Tensor:
    """``wsfft_execute_batched`` over `count` arrays stored back to back in
    `x` and `out` (one plan): the single-launch-per-pass batch."""
    import numpy as np
    per = 1 if plan.dtype == C64 else 2
    for t, nm in ((x, "input"), (out, "output")):
        if not t.is_cuda or t.dtype != _TORCH_DTYPE[plan.dtype] or not t.is_contiguous():
            raise ValueError(f"{nm} must be a contiguous device tensor of the plan's dtype")
        if t.numel() != plan.size * per * count:
            raise ValueError(f"{nm} holds {t.numel()} elements, want {plan.size * per * count}")
    span = plan.size * (8 if plan.dtype == C64 else 4)
    offs = np.arange(count, dtype=np.uint64) * np.uint64(span)
    ins = offs + np.uint64(x.data_ptr())
    outs = offs + np.uint64(out.data_ptr())
    hs = np.full(count, plan.handle, dtype=np.uint64)
    P = ctypes.POINTER(_vp)
    _check(_execute_batched(count, hs.ctypes.data_as(P), ins.ctypes.data_as(P), outs.ctypes.data_as(P),
                            int(bool(adjoint)), _stream(stream)), "execute_batched")
    return out


class BatchPlan:
    """``wsfft_batch_plan_create``: a batch bound to its buffers, executed as
    one persistent launch by :meth:`execute`.  Keeps the plans and tensors
    alive while it exists."""

    def __init__(self, plans, ins, outs, adjoint: bool = False):
        n = len(plans)
        if len(ins) != n or len(outs) != n:
            raise ValueError("plans, ins and outs must have one entry each")
        for p, i, o in zip(plans, ins, outs):
            p._check_tensor(i, "input")
            p._check_tensor(o, "output")
        arr = ctypes.c_void_p * max(n, 1)
        h = _batch_create(n, arr(*[p.handle for p in plans]), arr(*[t.data_ptr() for t in ins]),
                          arr(*[t.data_ptr() for t in outs]), int(bool(adjoint)))
        if not h:
            raise WsfftError(_batch_error(), "batch_plan_create")
        self._h = h
        self._keep = (list(plans), list(ins), list(outs))

    @property
    def tiles(self) -> int:
        return _batch_tiles(self._h)

    def execute(self, stream=None) -> None:
        _check(_batch_execute(self._h, _stream(stream)), "batch_execute")

    def timed_out(self) -> bool:
        """True if a dependency wait of any launch since creation or the
        previous call timed out; clears that record (synchronises)."""
        flag = _int(0)
        _check(_batch_check(self._h, ctypes.byref(flag)), "batch_plan_check")
        return bool(flag.value)

    def set_spin_limit(self, polls: int) -> None:
        """Polls after which a dependency wait gives up (diagnostic)."""
        _check(_batch_spin(self._h, int(polls)), "batch_plan_set_spin_limit")

    def close(self) -> None:
        if getattr(self, "_h", None):
            _batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RealPlan:
    """A real plan (``wsfft_plan_create_real``): the half spectrum of a real
    nx x ny x nz array (complex64, shape (nz, ny, nx/2 + 1)) and back.

    ``r2c(x)``: float32 (nz, ny, nx) -> complex64 half spectrum, forward sign,
    unnormalised.  ``c2r(X)``: half spectrum -> float32, sign +1, unnormalised
    (``inverse=True``: times 1/N, the inverse of ``r2c``); the C2R transform
    overwrites its input.  ``pitch`` (``wsfft_plan_create_real_ex``): half
    spectrum rows of ``pitch`` complex values, shape (nz, ny, pitch), of which
    [..., :nx/2 + 1] is the spectrum (a multiple of 16 aligns every row to
    cache lines); 0 is the compact layout."""

    def __init__(self, nx: int, ny: int = 1, nz: int = 1, flags: int = 0, pitch: int = 0):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.nxh = self.nx // 2 + 1
        self.pitch = int(pitch) if pitch else self.nxh
        self.device = torch.cuda.current_device()
        if pitch:
            h = _plan_create_real_ex(self.nx, self.ny, self.nz, int(flags), int(pitch))
        else:
            h = _plan_create_real(self.nx, self.ny, self.nz, int(flags))
        if not h:
            raise WsfftError(_get_last_error(), f"plan_create_real({nx},{ny},{nz}, pitch={pitch})")
        self._h = h

    @property
    def handle(self) -> int:
        return self._h

    @property
    def size(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def half_size(self) -> int:
        return self.pitch * self.ny * self.nz

    @property
    def num_passes(self) -> int:
        return _num_passes(self._h)

    @property
    def work_bytes(self) -> int:
        return _work_bytes(self._h)

    def half_shape(self, real_shape) -> tuple:
        return tuple(real_shape[:-1]) + (self.pitch,)

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(4096)
        _check(_describe(self._h, buf, len(buf)), "plan_describe")
        return buf.value.decode()

    @staticmethod
    def _check(t, dtype, n, name):
        if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dtype} device tensor")
        if t.numel() != n:
            raise ValueError(f"{name} has {t.numel()} elements, plan wants {n}")

    def r2c(self, x, out=None, stream=None):
        self._check(x, torch.float32, self.size, "input")
        if out is None:
            out = torch.empty(self.half_shape(x.shape), dtype=torch.complex64, device=x.device)
        self._check(out, torch.complex64, self.half_size, "output")
        _check(_execute_r2c(self._h, x.data_ptr(), out.data_ptr(), _stream(stream)), "execute_r2c")
        return out

    def c2r(self, X, out=None, stream=None, inverse: bool = False):
        """Overwrites X."""
        self._check(X, torch.complex64, self.half_size, "input")
        if out is None:
            out = torch.empty(tuple(X.shape[:-1]) + (self.nx,), dtype=torch.float32, device=X.device)
        self._check(out, torch.float32, self.size, "output")
        fn = _execute_c2r_inverse if inverse else _execute_c2r
        _check(fn(self._h, X.data_ptr(), out.data_ptr(), _stream(stream)), "execute_c2r")
        return out

    def execute_pass(self, index: int, x, out, mode: int = 0, stream=None):
        """Only pass `index` of r2c (mode 0) or c2r (1; 2 with 1/N)."""
        _check(_execute_pass(self._h, int(index), int(mode), x.data_ptr(), out.data_ptr(), _stream(stream)),
               "execute_pass")
        return out

    def close(self) -> None:
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- plan cache and functional forms ------------------------------------------------

_cache: dict = {}
_cache_mu = threading.Lock()


def _cached_plan(xyz, dt: int, sign: int, flags: int, device: torch.device) -> Plan:
    key = (tuple(xyz), dt, sign, flags, device.index)
    with _cache_mu:
        p = _cache.get(key)
        if p is None:
            with torch.cuda.device(device):
                p = Plan(*key[0], dtype=dt, sign=sign, flags=flags)
            _cache[key] = p
        return p


def _cached_real_plan(xyz, device: torch.device) -> RealPlan:
    key = ("real", tuple(xyz), device.index)
    with _cache_mu:
        p = _cache.get(key)
        if p is None:
            with torch.cuda.device(device):
                p = RealPlan(*xyz)
            _cache[key] = p
        return p


def _real_xyz(shape):
    s = tuple(shape)
    if not 1 <= len(s) <= 3:
        raise ValueError("rank 1..3 only")
    s = (1,) * (3 - len(s)) + s
    return s[2], s[1], s[0]


def rfftn(x: torch.Tensor) -> torch.Tensor:
    """Half spectrum (last axis nx//2 + 1) of the unnormalised forward DFT of
    a real float32 tensor of rank 1..3 (x = the last axis)."""
    return _cached_real_plan(_real_xyz(x.shape), x.device).r2c(x.contiguous())


def irfftn(X: torch.Tensor, nx: int) -> torch.Tensor:
    """The inverse of :func:`rfftn` (1/N included) for a real last axis of nx
    points; X is not modified."""
    xyz = (int(nx),) + _real_xyz(X.shape)[1:]
    return _cached_real_plan(xyz, X.device).c2r(X.contiguous().clone(), inverse=True)


def get_plan(x: torch.Tensor, sign: int = -1, flags: int = 0) -> Plan:
    dt = {torch.complex64: C64, torch.float16: C16_FP16, torch.bfloat16: C16_BF16}[x.dtype]
    return _cached_plan(shape_xyz(x.shape, dt), dt, sign, flags, x.device)


def fftn(x: torch.Tensor, sign: int = -1) -> torch.Tensor:
    """Unnormalised DFT over every axis of x (2^-S scaled for 16-bit storage)."""
    return get_plan(x, sign).execute(x)


def ifftn(x: torch.Tensor) -> torch.Tensor:
    """The inverse of :func:`fftn`: the opposite sign times 2^S/N (S = 0 for complex64)."""
    return get_plan(x, -1).execute_inverse(x)


# ---- autograd ------------------------------------------------------------------------
# PyTorch's convention for a C-linear map y = A x: grad_x = A^H grad_y.

class FFTn(torch.autograd.Function):
    """y = unnormalised DFT with kernel sign `sign`; backward = adjoint kernel."""

    @staticmethod
    def forward(ctx, x, sign: int = -1):
        ctx.sign = sign
        return get_plan(x, sign).execute(x.contiguous())

    @staticmethod
    def backward(ctx, g):
        return get_plan(g, ctx.sign).execute_adjoint(g.contiguous()), None


class IFFTn(torch.autograd.Function):
    """y = 2^S/N DFT with kernel sign -sign (S = 0 for complex64); backward = 2^S/N DFT
    with sign `sign`."""

    @staticmethod
    def forward(ctx, x, sign: int = -1):
        ctx.sign = sign
        return get_plan(x, sign).execute_inverse(x.contiguous())

    @staticmethod
    def backward(ctx, g):
        return get_plan(g, -ctx.sign).execute_inverse(g.contiguous()), None


def _real_to_complex_run(x: torch.Tensor) -> torch.Tensor:
    out = torch.empty(x.shape, dtype=torch.complex64, device=x.device)
    _check(_real_to_complex(x.data_ptr(), out.data_ptr(), x.numel(), _stream(None)), "real_to_complex")
    return out


def _complex_real_run(z: torch.Tensor) -> torch.Tensor:
    out = torch.empty(z.shape, dtype=torch.float32, device=z.device)
    _check(_complex_real_part(z.data_ptr(), out.data_ptr(), z.numel(), _stream(None)), "complex_real_part")
    return out


class RealToComplex(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        if x.dtype != torch.float32 or not x.is_cuda:
            raise TypeError("RealToComplex takes a float32 device tensor")
        return _real_to_complex_run(x.contiguous())

    @staticmethod
    def backward(ctx, g):
        return _complex_real_run(g.contiguous())


class ComplexRealPart(torch.autograd.Function):
    @staticmethod
    def forward(ctx, z):
        if z.dtype != torch.complex64 or not z.is_cuda:
            raise TypeError("ComplexRealPart takes a complex64 device tensor")
        return _complex_real_run(z.contiguous())

    @staticmethod
    def backward(ctx, g):
        return _real_to_complex_run(g.contiguous())


class PoissonSymbol(torch.autograd.Function):
    """X(k) -> -X(k)/|k|^2, k = 0 -> 0 (real multiplier: self-adjoint)."""

    @staticmethod
    def forward(ctx, z):
        if z.dtype != torch.complex64 or not z.is_cuda or z.dim() != 3:
            raise TypeError("PoissonSymbol takes a (nz, ny, nx) complex64 device tensor")
        out = z.contiguous().clone()
        nz, ny, nx = out.shape
        _check(_poisson_symbol(out.data_ptr(), nx, ny, nz, _stream(None)), "poisson_symbol")
        return out

    @staticmethod
    def backward(ctx, g):
        return PoissonSymbol.forward(ctx, g)


_work_cache: dict = {}


def _workspace(shape, device, stream: int) -> torch.Tensor:
    """A complex64 work array for the solve on this grid, device and stream,
    allocated on first use and reused by every later call (forward and
    backward alike): calls on one stream run in order, so they never overlap
    in it."""
    key = (tuple(shape), device.index, stream)
    with _cache_mu:
        w = _work_cache.get(key)
        if w is None:
            w = torch.empty(shape, dtype=torch.complex64, device=device)
            _work_cache[key] = w
        return w


def _poisson_fused(f: torch.Tensor, path: str):
    """wsfft_poisson_solve on a (nz, ny, nx) float32 tensor with a real plan
    (path "real": five half-spectrum passes) or a complex plan ("complex":
    six complex passes); None where the grid has no fused kernels."""
    xyz = shape_xyz(f.shape, C64)
    if path == "real":
        plan = _cached_real_plan(xyz, f.device)
        wshape = (xyz[2], xyz[1], xyz[0] // 2 + 1)
    else:
        # the six-pass complex solve needs separate x and y passes
        plan = _cached_plan(xyz, C64, -1, FLAG_NO_PLANE, f.device)
        wshape = tuple(f.shape)
    u = torch.empty_like(f)
    st_h = _stream(None)
    work = _workspace(wshape, f.device, st_h)
    st = _poisson_solve(plan.handle, f.data_ptr(), u.data_ptr(), work.data_ptr(), st_h)
    if st == 2:   # WSFFT_ERROR_UNSUPPORTED_SIZE
        return None
    _check(st, "poisson_solve")
    return u


class PoissonSolve(torch.autograd.Function):
    """The fused solve; the operator is linear and self-adjoint, so the
    backward pass is the same solve applied to the incoming gradient."""

    @staticmethod
    def forward(ctx, f, path: str = "real"):
        ctx.path = path
        return _poisson_fused(f.contiguous(), path)

    @staticmethod
    def backward(ctx, g):
        return _poisson_fused(g.contiguous(), ctx.path), None


def poisson_solve(f: torch.Tensor, fused: bool = True, path: str = "auto") -> torch.Tensor:
    """u = Re(IFFT(-FFT(f)/|k|^2)) on the periodic box [0, 2*pi)^3, differentiable.

    path "real": wsfft_poisson_solve with a real plan (five half-spectrum
    passes); "complex": with a complex plan (six complex passes); "composed":
    the complex plan's transforms and the elementwise kernels; "auto" (the
    default): the first of these the grid supports.  fused=False is
    "composed"."""
    if f.dtype != torch.float32 or not f.is_cuda or f.dim() != 3:
        raise TypeError("poisson_solve takes a (nz, ny, nx) float32 device tensor")
    if not fused:
        path = "composed"
    shape = tuple(f.shape)
    if path == "auto":
        path = ("real" if _poisson_real_supported(shape)
                else "complex" if _poisson_fused_supported(shape) else "composed")
    if path == "real" and not _poisson_real_supported(shape):
        raise ValueError(f"grid {shape} has no fused half-spectrum solve")
    if path == "complex" and not _poisson_fused_supported(shape):
        raise ValueError(f"grid {shape} has no fused complex solve")
    if path in ("real", "complex"):
        return PoissonSolve.apply(f, path)
    if path != "composed":
        raise ValueError(f"unknown path {path!r}")
    z = RealToComplex.apply(f)
    F = FFTn.apply(z, -1)
    U = PoissonSymbol.apply(F)
    u = IFFTn.apply(U, -1)
    return ComplexRealPart.apply(u)


_FUSED_LENGTHS = (32, 64, 128, 256, 512, 1024)


def _poisson_fused_supported(shape) -> bool:
    return len(shape) == 3 and all(n in _FUSED_LENGTHS for n in shape)


def _poisson_real_supported(shape) -> bool:
    """(nz, ny, nx): the fused z pass of the half-spectrum solve exists for nz
    in _FUSED_LENGTHS; nx is even (4 .. 32768) and ny at most 1024 (one pass)."""
    if len(shape) != 3:
        return False
    nz, ny, nx = shape
    return nz in _FUSED_LENGTHS and 1 < ny <= 1024 and _smooth23(ny) and nx % 2 == 0 and 4 <= nx <= 32768 \
        and _smooth23(nx)


def _smooth23(n: int) -> bool:
    if n < 1:
        return False
    for p in (2, 3):
        while n % p == 0:
            n //= p
    return n == 1
