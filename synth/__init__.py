"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no transform arithmetic: it only draws random arrays and
rounds them to a storage type, so that the HIP path and the FP64 oracle are
fed the exact same stored values.  Arrays use shape (nz, ny, nx), x fastest.

Recipes (each workload's values, shapes and seeds):

* plain 3D forward, 32^3 complex64: re, im iid U[-1, 1), seed 0;
* 512^3 complex64 forward/inverse, 2D 8192^2 and 1D 1024 x 65536: re, im iid
  N(0, 1), seed 1;
* reduced-precision 512^3: re, im iid 0.5 * N(0, 1), drawn in FP64 and rounded
  to nearest-even FP16 or BF16, seed 2;
* 96 uneven arrays: each of nx, ny, nz drawn uniformly from
  {32, 64, 96, 128, 256}, redrawn while nx == ny == nz; values U[-1, 1), seed 3;
* Poisson on 256^3: f = sum of 64 Gaussian bumps of standard deviation
  0.05 * 2*pi on the periodic box [0, 2*pi)^3 (minimum-image distance),
  centres U[0, 2*pi)^3, amplitudes N(0, 1); w ~ N(0, 1); seed 4.

All draws use ``numpy.random.default_rng(seed)`` in FP64.
"""
from __future__ import annotations

import numpy as np

BATCH_AXIS_CHOICES = (32, 64, 96, 128, 256)


def uniform_c(shape, seed: int) -> np.ndarray:
    """complex128 with re, im iid U[-1, 1)."""
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, size=shape)
    im = rng.uniform(-1.0, 1.0, size=shape)
    return re + 1j * im


def normal_c(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """complex128 with re, im iid scale * N(0, 1)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(size=shape)
    im = rng.standard_normal(size=shape)
    if scale != 1.0:
        re *= scale
        im *= scale
    return re + 1j * im


def normal_c64(shape, seed: int, chunk: int = 1 << 24) -> np.ndarray:
    """complex64 draw of re, im iid N(0, 1) without a full FP64 temporary
    (the large workloads): values are the FP64 draws rounded to FP32.  The
    real and imaginary parts come from two generators seeded (seed, 0) and
    (seed, 1), drawn in order in blocks of ``chunk``."""
    n = int(np.prod(shape))
    out = np.empty(n, dtype=np.complex64)
    view = out.view(np.float32).reshape(n, 2)
    g_re = np.random.default_rng([seed, 0])
    g_im = np.random.default_rng([seed, 1])
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        view[s:e, 0] = g_re.standard_normal(e - s)
        view[s:e, 1] = g_im.standard_normal(e - s)
    return out.reshape(shape)


# --- storage rounding ----------------------------------------------------------

def to_fp16_pairs(z: np.ndarray) -> np.ndarray:
    """Round re and im to FP16 (nearest even); returns (..., 2) float16."""
    out = np.empty(z.shape + (2,), dtype=np.float16)
    out[..., 0] = z.real.astype(np.float16)
    out[..., 1] = z.imag.astype(np.float16)
    return out


def _f32_to_bf16_bits(x32: np.ndarray) -> np.ndarray:
    """Nearest-even rounding of FP32 values to the top 16 bits (BF16)."""
    b = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    rounded = (b + 0x7FFF + lsb) >> 16
    nan = np.isnan(x32)
    rounded = np.where(nan, (b >> 16) | 0x40, rounded)
    return rounded.astype(np.uint16)


def to_bf16_pairs(z: np.ndarray) -> np.ndarray:
    """Round re and im to BF16 (via FP32, nearest even); returns (..., 2)
    uint16 bit patterns."""
    out = np.empty(z.shape + (2,), dtype=np.uint16)
    out[..., 0] = _f32_to_bf16_bits(z.real.astype(np.float32))
    out[..., 1] = _f32_to_bf16_bits(z.imag.astype(np.float32))
    return out


def bf16_bits_to_f64(b: np.ndarray) -> np.ndarray:
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def pairs_to_c128(p: np.ndarray, kind: str) -> np.ndarray:
    """(..., 2) FP16 pairs or BF16 bit pairs back to complex128 (exact)."""
    if kind == "fp16":
        re, im = p[..., 0].astype(np.float64), p[..., 1].astype(np.float64)
    elif kind == "bf16":
        re, im = bf16_bits_to_f64(p[..., 0]), bf16_bits_to_f64(p[..., 1])
    else:
        raise ValueError(kind)
    return re + 1j * im


# --- workload generators ------------------------------------------------------

def batched_shapes(count: int = 96, seed: int = 3, choices=BATCH_AXIS_CHOICES):
    """Non-cubic (nx, ny, nz) triples drawn uniformly from ``choices``."""
    rng = np.random.default_rng(seed)
    shapes = []
    while len(shapes) < count:
        nx, ny, nz = (int(v) for v in rng.choice(choices, size=3))
        if nx == ny == nz:
            continue
        shapes.append((nx, ny, nz))
    return shapes


def batched_arrays(shapes, seed: int = 3):
    """One complex128 U[-1, 1) array per shape, (nz, ny, nx) each, drawn
    from a generator seeded (seed, i) for array i."""
    out = []
    for i, (nx, ny, nz) in enumerate(shapes):
        rng = np.random.default_rng([seed, i])
        re = rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
        im = rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
        out.append(re + 1j * im)
    return out


def gaussian_bumps(n: int, count: int = 64, width: float = 0.05, seed: int = 4) -> np.ndarray:
    """Real (n, n, n) field: sum of ``count`` periodic Gaussian bumps.
    sigma = width * 2*pi; distance is the minimum-image distance on
    [0, 2*pi)^3; grid point j sits at 2*pi*j/n."""
    rng = np.random.default_rng(seed)
    L = 2.0 * np.pi
    centres = rng.uniform(0.0, L, size=(count, 3))
    amps = rng.standard_normal(count)
    sigma = width * L
    g = np.arange(n) * (L / n)
    f = np.zeros((n, n, n), dtype=np.float64)
    for (cx, cy, cz), a in zip(centres, amps):
        def d1(c):
            d = np.abs(g - c)
            return np.minimum(d, L - d)
        ex = np.exp(-d1(cx) ** 2 / (2 * sigma * sigma))
        ey = np.exp(-d1(cy) ** 2 / (2 * sigma * sigma))
        ez = np.exp(-d1(cz) ** 2 / (2 * sigma * sigma))
        f += a * ez[:, None, None] * ey[None, :, None] * ex[None, None, :]
    return f


def poisson_weights(n: int, seed: int = 4) -> np.ndarray:
    """w ~ N(0, 1) on the (n, n, n) grid, from a generator seeded (seed, 1)."""
    return np.random.default_rng([seed, 1]).standard_normal((n, n, n))
