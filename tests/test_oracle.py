"""Pins for the FP64 oracle, independent of the oracle's own code.

Each test checks the oracle against something the mathematics or the paper
fixes: hand-derived textbook values, a brute-force evaluation of the DFT
definition, closed forms, invariants.  A dropped term, a wrong sign, a wrong
index or stride, or a transposed axis fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def rel_l2(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def to_xyz_array(flat, nx, ny, nz):
    return np.asarray(flat, np.complex128).reshape(nz, ny, nx)


# --- hand-derived values ---------------------------------------------------------

def _parse_golden(path):
    env = {"__builtins__": {}, "sqrt": math.sqrt}
    cases, cur = [], None
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        key, *rest = line.split()
        if key == "case":
            cur = {"name": rest[0]}
            cases.append(cur)
        elif key == "shape":
            cur["shape"] = tuple(int(v) for v in rest)
        elif key == "sign":
            cur["sign"] = int(rest[0])
        elif key in ("in", "out"):
            vals = []
            for tok in rest:
                re_s, im_s = tok.split(",")
                vals.append(complex(eval(re_s, env), eval(im_s, env)))
            cur[key] = np.array(vals)
    return cases


GOLDEN = _parse_golden(os.path.join(HERE, "golden", "textbook_dft.txt"))


@pytest.mark.parametrize("case", GOLDEN, ids=[c["name"] for c in GOLDEN])
def test_golden_textbook(case):
    nx, ny, nz = case["shape"]
    a = to_xyz_array(case["in"], nx, ny, nz)
    got = oracle.fftn(a, case["sign"])
    want = to_xyz_array(case["out"], nx, ny, nz)
    assert np.max(np.abs(got - want)) < 1e-13


# --- brute force ---------------------------------------------------------------

def brute_force_dft(a, sign):
    """The definition summed directly over every (input, output) pair, with
    the phase reduced exactly as an integer before scaling by 2*pi."""
    nz, ny, nx = a.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    # phase(k, j) = kx*x/nx + ky*y/ny + kz*z/nz, as a fraction of a turn
    ph = ((np.outer(x, x) % nx) / nx + (np.outer(y, y) % ny) / ny
          + (np.outer(z, z) % nz) / nz)
    M = np.exp(sign * 2j * np.pi * ph)     # rows: output k, cols: input j
    return (M @ a.ravel()).reshape(a.shape)


BF_DIMS = [1, 2, 3, 4, 5, 6, 8, 12, 16]
BF_SHAPES = [(nx, 1, 1) for nx in BF_DIMS] + [
    (2, 3, 1), (3, 2, 5), (4, 4, 4), (8, 6, 2), (5, 12, 3), (16, 12, 8),
    (1, 16, 6), (6, 1, 12), (12, 8, 16), (16, 16, 1), (1, 1, 16), (3, 5, 6),
]


@pytest.mark.parametrize("shape", BF_SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("sign", [-1, 1])
def test_brute_force(shape, sign):
    nx, ny, nz = shape
    a = synth.uniform_c((nz, ny, nx), seed=nx * 1000 + ny * 10 + nz)
    got = oracle.fftn(a, sign)
    assert rel_l2(got, brute_force_dft(a, sign)) < 1e-13


def test_brute_force_odd_primes():
    # factors other than 2 and 3 take the generic combine step
    for n in (7, 11, 13, 35, 49):
        a = synth.normal_c((1, 1, n), seed=n)
        assert rel_l2(oracle.fftn(a), brute_force_dft(a, -1)) < 1e-13


# --- closed forms ----------------------------------------------------------------

SHAPES = [(32, 32, 32), (8, 16, 4), (96, 32, 12), (6, 9, 27), (64, 1, 1), (1, 48, 1)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_delta_origin_gives_ones(shape):
    nx, ny, nz = shape
    a = np.zeros((nz, ny, nx), np.complex128)
    a[0, 0, 0] = 1.0
    assert np.max(np.abs(oracle.fftn(a) - 1.0)) < 1e-14


@pytest.mark.parametrize("shape", [(8, 4, 2), (32, 32, 32), (12, 6, 9)], ids=str)
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_delta_one_step_along_each_axis(shape, axis):
    """delta at unit distance along axis a: X = exp(-2*pi*i*k_a/n_a), constant
    over the other axes.  Fixes the sign and which axis is which."""
    nx, ny, nz = shape
    a = np.zeros((nz, ny, nx), np.complex128)
    idx = [0, 0, 0]
    n = [nx, ny, nz][axis]
    idx[2 - axis] = 1 % n
    a[tuple(idx)] = 1.0
    k = np.arange(n)
    w = np.exp(-2j * np.pi * k * (1 % n) / n)
    shape_b = [1, 1, 1]
    shape_b[2 - axis] = n
    want = np.broadcast_to(w.reshape(shape_b), a.shape)
    assert np.max(np.abs(oracle.fftn(a) - want)) < 1e-13


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_constant(shape):
    nx, ny, nz = shape
    c = 0.75 - 0.25j
    X = oracle.fftn(np.full((nz, ny, nx), c))
    N = nx * ny * nz
    assert abs(X[0, 0, 0] - c * N) < 1e-12 * N
    X[0, 0, 0] = 0
    assert np.max(np.abs(X)) < 1e-12 * N


@pytest.mark.parametrize("shape,m", [((16, 8, 4), (3, 5, 1)), ((96, 12, 6), (17, 7, 4)),
                                     ((27, 18, 8), (26, 0, 3))], ids=str)
def test_plane_wave(shape, m):
    nx, ny, nz = shape
    mx, my, mz = m
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a = np.exp(2j * np.pi * ((mx * x % nx) / nx + (my * y % ny) / ny + (mz * z % nz) / nz))
    X = oracle.fftn(a)
    N = nx * ny * nz
    want = np.zeros_like(X)
    want[mz, my, mx] = N
    assert np.max(np.abs(X - want)) < 1e-11 * N


@pytest.mark.parametrize("shape", [(16, 8, 4), (24, 9, 32), (5, 7, 6)], ids=str)
def test_shift_theorem(shape):
    nx, ny, nz = shape
    a = synth.normal_c((nz, ny, nx), seed=11)
    s = (3 % nx, 2 % ny, 5 % nz)
    shifted = np.roll(a, shift=(s[2], s[1], s[0]), axis=(0, 1, 2))   # a(x - s)
    kz, ky, kx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phase = np.exp(-2j * np.pi * ((kx * s[0] % nx) / nx + (ky * s[1] % ny) / ny
                                  + (kz * s[2] % nz) / nz))
    assert rel_l2(oracle.fftn(shifted), phase * oracle.fftn(a)) < 1e-13


@pytest.mark.parametrize("shape", [(32, 16, 8), (96, 6, 12), (7, 9, 10)], ids=str)
def test_geometric_sequence_product(shape):
    """a[x,y,z] = rx^x ry^y rz^z has the product of per-axis geometric sums:
    X_k = (1 - r^n) / (1 - r exp(-2*pi*i*k/n)) on each axis."""
    nx, ny, nz = shape
    r = [0.9 * np.exp(0.3j), 1.05 * np.exp(-0.7j), 0.8 + 0.1j]
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a = r[0] ** x * r[1] ** y * r[2] ** z

    def geo(rr, n):
        k = np.arange(n)
        return (1 - rr ** n) / (1 - rr * np.exp(-2j * np.pi * k / n))

    want = (geo(r[2], nz)[:, None, None] * geo(r[1], ny)[None, :, None]
            * geo(r[0], nx)[None, None, :])
    assert rel_l2(oracle.fftn(a), want) < 1e-12


# --- invariants --------------------------------------------------------------------

@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_parseval_and_round_trip(shape):
    nx, ny, nz = shape
    a = synth.uniform_c((nz, ny, nx), seed=5)
    X = oracle.fftn(a)
    N = a.size
    assert abs(np.vdot(X, X).real - N * np.vdot(a, a).real) < 1e-12 * N * np.vdot(a, a).real
    assert rel_l2(oracle.ifftn(X), a) < 1e-14


@pytest.mark.parametrize("shape", [(16, 12, 8), (9, 4, 6)], ids=str)
def test_hermitian_symmetry_for_real_input(shape):
    nx, ny, nz = shape
    a = synth.normal_c((nz, ny, nx), seed=6).real.astype(np.complex128)
    X = oracle.fftn(a)
    Xneg = np.roll(np.flip(X, axis=(0, 1, 2)), shift=1, axis=(0, 1, 2))   # X[-k]
    assert rel_l2(Xneg, np.conj(X)) < 1e-14


def test_linearity():
    a = synth.uniform_c((8, 12, 16), seed=7)
    b = synth.normal_c((8, 12, 16), seed=8)
    al, be = 0.3 - 1.2j, -2.0 + 0.5j
    assert rel_l2(oracle.fftn(al * a + be * b), al * oracle.fftn(a) + be * oracle.fftn(b)) < 1e-14


@pytest.mark.parametrize("shape", [(16, 12, 8), (32, 3, 64)], ids=str)
def test_axis_order_and_transpose(shape):
    nx, ny, nz = shape
    a = synth.uniform_c((nz, ny, nx), seed=9)
    X = oracle.fftn(a)
    assert rel_l2(oracle.fftn(a, order="zyx"), X) < 1e-14
    # transposing the input transposes the output
    at = np.ascontiguousarray(a.transpose(2, 1, 0))
    assert rel_l2(oracle.fftn(at), X.transpose(2, 1, 0)) < 1e-14


def test_thread_count_does_not_change_bits():
    a = synth.normal_c((16, 24, 32), seed=10)
    assert np.array_equal(oracle.fftn(a, threads=1), oracle.fftn(a, threads=7))


def test_fft1d_batch_matches_rows():
    a = synth.normal_c((6, 96), seed=12)
    got = oracle.fft1d_batch(a)
    for i in range(6):
        assert rel_l2(got[i], oracle.fftn(a[i])) < 1e-15


def test_numpy_cross_check():
    """Secondary check only (the paper validated against NumPy)."""
    a = synth.normal_c((64, 96, 128), seed=13)
    assert rel_l2(oracle.fftn(a), np.fft.fftn(a)) < 1e-12


# --- spectral Poisson operator -----------------------------------------------------

def test_wavenumbers():
    assert list(oracle.integer_wavenumbers(8)) == [0, 1, 2, 3, -4, -3, -2, -1]
    assert list(oracle.integer_wavenumbers(5)) == [0, 1, 2, -2, -1]


def test_poisson_single_mode():
    """f = cos(kx x + ky y + kz z) solves to u = -f / |k|^2 (Laplacian symbol -|k|^2)."""
    n = 16
    g = np.arange(n) * 2 * np.pi / n
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    k = (3, -2, 5)
    f = np.cos(k[0] * x + k[1] * y + k[2] * z)
    u = oracle.poisson_apply(f)
    assert np.max(np.abs(u + f / (9 + 4 + 25))) < 1e-14


def test_poisson_constant_is_removed():
    u = oracle.poisson_apply(np.full((8, 8, 8), 3.0))
    assert np.max(np.abs(u)) < 1e-14


def test_poisson_gradient_by_finite_differences():
    """The loss is linear in f, so central differences are exact up to
    rounding; every coordinate is checked on a small grid."""
    n = 6
    f = synth.gaussian_bumps(n, count=4, seed=21)
    w = synth.poisson_weights(n, seed=21)
    g = oracle.poisson_loss_grad(w)
    h = 1e-3
    fd = np.empty_like(f)
    for idx in np.ndindex(f.shape):
        fp = f.copy(); fp[idx] += h
        fm = f.copy(); fm[idx] -= h
        fd[idx] = (oracle.poisson_loss(fp, w) - oracle.poisson_loss(fm, w)) / (2 * h)
    assert np.max(np.abs(fd - g)) < 1e-10


def test_poisson_self_adjoint():
    a = synth.normal_c((8, 10, 12), seed=22).real
    b = synth.normal_c((8, 10, 12), seed=23).real
    lhs = np.sum(oracle.poisson_apply(a) * b)
    rhs = np.sum(a * oracle.poisson_apply(b))
    assert abs(lhs - rhs) < 1e-13 * np.sqrt(np.sum(a * a) * np.sum(b * b))


# --- real input, half spectrum (rfftn) and its complex-to-real inverse (irfftn) ---

RSHAPES = [(1, 1, 2), (1, 1, 7), (1, 1, 8), (3, 4, 6), (2, 5, 9), (4, 3, 12), (6, 2, 16)]   # (nz, ny, nx)


@pytest.mark.parametrize("shape", RSHAPES, ids=lambda s: "x".join(map(str, s)))
def test_rfftn_brute_force(shape):
    """The half spectrum is bins kx = 0 .. nx//2 of the directly summed DFT."""
    a = synth.normal_c(shape, seed=sum(shape)).real
    want = brute_force_dft(a.astype(np.complex128), -1)[..., : shape[-1] // 2 + 1]
    got = oracle.rfftn(a)
    assert got.shape == want.shape
    assert rel_l2(got, want) < 1e-13


@pytest.mark.parametrize("shape", [(4, 6, 8), (3, 5, 9), (1, 1, 16)], ids=lambda s: "x".join(map(str, s)))
def test_rfftn_hermitian_reconstruction(shape):
    """The full DFT of a real array is recovered from the half spectrum by
    X[kx, ky, kz] = conj(X[-kx, -ky, -kz])."""
    nz, ny, nx = shape
    a = synth.uniform_c(shape, seed=7 * nx).real
    H = oracle.rfftn(a)
    full = np.empty(shape, np.complex128)
    nh = nx // 2 + 1
    full[..., :nh] = H
    for kx in range(nh, nx):
        # -k taken modulo each axis length
        full[..., kx] = np.conj(H[(-np.arange(nz)) % nz][:, (-np.arange(ny)) % ny][..., nx - kx])
    assert rel_l2(full, brute_force_dft(a.astype(np.complex128), -1)) < 1e-13


@pytest.mark.parametrize("nx,m", [(16, 0), (16, 3), (16, 8), (12, 5), (9, 4)])
def test_rfftn_cosine(nx, m):
    """cos(2*pi*m*x/nx) has N/2 in bin m (N at m = 0 and m = nx/2) and 0 elsewhere."""
    ny, nz = 3, 2
    x = np.arange(nx)
    a = np.broadcast_to(np.cos(2 * np.pi * m * x / nx), (nz, ny, nx))
    H = oracle.rfftn(np.ascontiguousarray(a))
    want = np.zeros((nz, ny, nx // 2 + 1), np.complex128)
    N = nx * ny * nz
    want[0, 0, m] = N if (m == 0 or 2 * m == nx) else N / 2
    assert np.max(np.abs(H - want)) < 1e-12 * N


@pytest.mark.parametrize("shape", [(4, 6, 8), (3, 5, 9), (2, 2, 2), (1, 1, 16), (8, 4, 12)],
                         ids=lambda s: "x".join(map(str, s)))
def test_irfftn_round_trip(shape):
    """irfftn(rfftn(a)) = N * a for real a."""
    a = synth.normal_c(shape, seed=3 * sum(shape)).real
    back = oracle.irfftn(oracle.rfftn(a), shape[-1])
    assert back.dtype == np.float64 and back.shape == a.shape
    assert rel_l2(back, a.size * a) < 1e-13


@pytest.mark.parametrize("nx", [8, 9, 12])
def test_irfftn_single_bin_closed_forms(nx):
    """One nonzero bin c at (kx, ky, kz) = (m, q, 0): the output is
    2 Re(c exp(2*pi*i*(m x/nx + q y/ny))) for 0 < m < nx/2; at m = 0 and
    m = nx/2 only Re(c) counts: Re(c) exp-free in x (or (-1)^x) times
    Re(exp(2*pi*i*q y/ny)).  Fixes the sign along y and x and the
    discarded imaginary parts."""
    ny, nz = 5, 3
    nh = nx // 2 + 1
    x = np.arange(nx)[None, None, :]
    y = np.arange(ny)[None, :, None]
    c = 0.75 - 1.25j
    for m in range(nh):
        for q in (0, 2):
            H = np.zeros((nz, ny, nh), np.complex128)
            H[0, q, m] = c
            got = oracle.irfftn(H, nx)
            ph = np.exp(2j * np.pi * q * y / ny)
            if m == 0 or 2 * m == nx:
                # the x step keeps the real part of the y-transformed bin
                want = np.broadcast_to((c * ph).real * np.cos(np.pi * 2 * m * x / nx), (nz, ny, nx))
            else:
                want = np.broadcast_to(2 * (c * ph * np.exp(2j * np.pi * m * x / nx)).real, (nz, ny, nx))
            assert np.max(np.abs(got - want)) < 1e-12, (m, q)


def test_real_forms_numpy_cross_check():
    """NumPy's real transforms as a secondary check (never the oracle)."""
    a = synth.normal_c((12, 16, 18), seed=91).real
    H = oracle.rfftn(a)
    assert rel_l2(H, np.fft.rfftn(a)) < 1e-12
    Hr = synth.normal_c(H.shape, seed=92)
    assert rel_l2(oracle.irfftn(Hr, 18), np.fft.irfftn(Hr, s=a.shape, axes=(0, 1, 2)) * a.size) < 1e-12
