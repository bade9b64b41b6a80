"""FP64 CPU oracle for the multidimensional complex-to-complex DFT.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``, never by the product package.
It shares no code with the HIP path.

The transform (paper, Section 1 and Section 2.2): a k-dimensional DFT is 1D
DFTs along each axis in turn, in any order.  Arrays are numpy complex128 with
shape ``(nz, ny, nx)`` (x fastest), i.e. element (x, y, z) at linear index
``x + nx*(y + ny*z)``.  ``sign=-1`` is the forward transform; no function
here normalises unless its name says so.

The arithmetic lives in ``wsfft_oracle.c`` (plain C, FP64, recursive
mixed-radix Cooley-Tukey, pthreads over pencils).  ``rfftn`` / ``irfftn``
define the half-spectrum forms of the same DFT for real input and output.
``poisson_*`` below follow the spectral Poisson operator
u = IFFT(-FFT(f)/|k|^2), k = 0 mode zeroed, which the differentiable-solve
workload defines.  Parity status: pinned (see ``tests/test_oracle.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wsfft_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile the C oracle with gcc (plain -O2, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
           "-pthread", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    for name in ("oracle_fftn", "oracle_fftn_zyx"):
        fn = getattr(lib, name)
        fn.argtypes = [dp, dp, i64, i64, i64, ctypes.c_int, ctypes.c_int]
        fn.restype = ctypes.c_int
    lib.oracle_fft1d_batch.argtypes = [dp, dp, i64, i64, ctypes.c_int, ctypes.c_int]
    lib.oracle_fft1d_batch.restype = ctypes.c_int
    _lib = lib
    return lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def _as_c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.complex128)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def fftn(a, sign: int = -1, threads: int | None = None, order: str = "xyz") -> np.ndarray:
    """Unnormalised 3D DFT of ``a`` (shape (nz, ny, nx), or lower rank which
    is read as trailing axes: (ny, nx) or (nx,)), axes taken x, y, z
    (``order='xyz'``) or z, y, x."""
    a = _as_c128(a)
    shape = a.shape
    if a.ndim == 1:
        nz, ny, nx = 1, 1, shape[0]
    elif a.ndim == 2:
        nz, (ny, nx) = 1, shape
    elif a.ndim == 3:
        nz, ny, nx = shape
    else:
        raise ValueError("oracle.fftn takes rank 1..3")
    out = np.empty_like(a)
    fn = _load().oracle_fftn if order == "xyz" else _load().oracle_fftn_zyx
    rc = fn(_ptr(a), _ptr(out), nx, ny, nz, int(sign), threads or default_threads())
    if rc != 0:
        raise RuntimeError(f"oracle_fftn failed with {rc}")
    return out


def ifftn(a, threads: int | None = None) -> np.ndarray:
    """Normalised inverse: (1/N) * the sign=+1 sum (paper, Section 4.2)."""
    a = _as_c128(a)
    return fftn(a, +1, threads) / a.size


def fft1d_batch(a, sign: int = -1, threads: int | None = None) -> np.ndarray:
    """Independent 1D transforms along the last axis of a 2D array."""
    a = _as_c128(a)
    if a.ndim != 2:
        raise ValueError("fft1d_batch takes (count, n)")
    out = np.empty_like(a)
    rc = _load().oracle_fft1d_batch(_ptr(a), _ptr(out), a.shape[1], a.shape[0],
                                    int(sign), threads or default_threads())
    if rc != 0:
        raise RuntimeError(f"oracle_fft1d_batch failed with {rc}")
    return out


# --- real input and real output ------------------------------------------------
# The transform of Section 1 applied to a real array: its DFT is Hermitian,
# X[-k] = conj(X[k]), so the bins kx = 0 .. nx//2 along x determine all the
# others.  The paper transforms complex data only (Section 5); these two
# functions define the half-spectrum forms by the full DFT above.

def rfftn(a, threads: int | None = None) -> np.ndarray:
    """Forward (sign -1) DFT of a real array of shape (nz, ny, nx) (or lower
    rank, trailing axes as in :func:`fftn`), kept for kx = 0 .. nx//2:
    shape (..., nx//2 + 1), unnormalised.  Definition: the full complex DFT
    of the real input, sliced."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        raise TypeError("rfftn takes a real array")
    X = fftn(a.astype(np.complex128), -1, threads)
    return np.ascontiguousarray(X[..., : a.shape[-1] // 2 + 1])


def _dft_along(a: np.ndarray, axis: int, sign: int, threads) -> np.ndarray:
    """Unnormalised 1D DFTs along one axis of a complex array."""
    m = np.ascontiguousarray(np.moveaxis(a, axis, -1))
    out = fft1d_batch(m.reshape(-1, m.shape[-1]), sign, threads).reshape(m.shape)
    return np.moveaxis(out, -1, axis)


def irfftn(H, nx: int, threads: int | None = None) -> np.ndarray:
    """Unnormalised complex-to-real transform (sign +1) of a half spectrum
    H of shape (..., nx//2 + 1) to a real array of shape (..., nx).

    Definition, one axis at a time: sign +1 DFTs along every axis but x (of
    the half spectrum as given); then along x the Hermitian extension
    Y[k] for 0 < k < nx/2, conj(Y[nx - k]) for k > nx/2, and the real parts
    of Y[0] and (nx even) Y[nx/2], whose imaginary parts a Hermitian
    spectrum does not have; its sign +1 DFT is real.  For the half spectrum
    of a real array a, irfftn(rfftn(a), nx) = N * a."""
    H = np.asarray(H, dtype=np.complex128)
    nh = nx // 2 + 1
    if H.shape[-1] != nh:
        raise ValueError(f"half spectrum of {nx} points has {nh} bins, got {H.shape[-1]}")
    Y = H
    for axis in range(H.ndim - 1):
        Y = _dft_along(Y, axis, +1, threads)
    ext = np.empty(H.shape[:-1] + (nx,), dtype=np.complex128)
    ext[..., :nh] = Y
    ext[..., 0] = Y[..., 0].real
    if nx % 2 == 0:
        ext[..., nx // 2] = Y[..., nx // 2].real
    k = np.arange(nh, nx)
    ext[..., k] = np.conj(Y[..., nx - k])
    return _dft_along(ext, H.ndim - 1, +1, threads).real


# --- spectral Poisson operator ------------------------------------------------

def integer_wavenumbers(n: int) -> np.ndarray:
    """k for a periodic grid on [0, 2*pi): 0, 1, ..., n/2-1, -n/2, ..., -1."""
    k = np.arange(n, dtype=np.float64)
    k[k >= (n + 1) // 2] -= n
    return k


def poisson_symbol(nx: int, ny: int, nz: int) -> np.ndarray:
    """-1/|k|^2 on the (nz, ny, nx) grid, with the k = 0 entry set to 0."""
    kx = integer_wavenumbers(nx)[None, None, :]
    ky = integer_wavenumbers(ny)[None, :, None]
    kz = integer_wavenumbers(nz)[:, None, None]
    k2 = kx * kx + ky * ky + kz * kz
    sym = np.zeros_like(k2)
    nz_mask = k2 != 0
    sym[nz_mask] = -1.0 / k2[nz_mask]
    return sym


def poisson_apply(f, threads: int | None = None) -> np.ndarray:
    """u = Re(IFFT(sym * FFT(f))) for real f of shape (nz, ny, nx), FP64."""
    f = np.asarray(f, dtype=np.float64)
    nz, ny, nx = f.shape
    F = fftn(f.astype(np.complex128), -1, threads)
    U = F * poisson_symbol(nx, ny, nz)
    return ifftn(U, threads).real


def poisson_loss(f, w, threads: int | None = None) -> float:
    """sum(u * w) in FP64."""
    return float(np.sum(poisson_apply(f, threads) * np.asarray(w, np.float64)))


def poisson_loss_grad(w, threads: int | None = None) -> np.ndarray:
    """d(sum(u*w))/df.  The operator f -> u is real, linear and self-adjoint
    (a real even Fourier multiplier), so the gradient is the operator applied
    to w."""
    return poisson_apply(w, threads)
