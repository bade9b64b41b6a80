/*
 * Elementwise companions of the FFT for the differentiable spectral Poisson
 * solve u = Re(IFFT(-FFT(f) / |k|^2)) with the k = 0 mode set to zero, on a
 * periodic box [0, 2*pi)^3 with integer wavenumbers.  (The paper's method
 * is the FFT itself; these are the pointwise steps of that workload, so the
 * whole solve and its adjoint run on the GPU.)
 *
 * All pointers are device pointers owned by the caller; every call only
 * enqueues one kernel on `stream`, validates its arguments first and
 * returns a wsfft_status_t.  n = 0 is a no-op.
 */
#ifndef WSFFT_POINTWISE_H
#define WSFFT_POINTWISE_H

#include <stdint.h>
#include "wsfft.h"

#ifdef __cplusplus
extern "C" {
#endif

/* out[i] = in[i] + 0i for i in [0, n).  in: n FP32 (4-byte aligned);
 * out: n complex64 (8-byte aligned).  Its adjoint is wsfft_complex_real_part. */
wsfft_status_t wsfft_real_to_complex(const float* in, void* out, int64_t n, hipStream_t stream);

/* out[i] = Re(in[i]) for i in [0, n).  in: n complex64; out: n FP32.
 * Its adjoint is wsfft_real_to_complex. */
wsfft_status_t wsfft_complex_real_part(const void* in, float* out, int64_t n, hipStream_t stream);

/* In place on an nx x ny x nz complex64 array (x fastest): multiplies entry
 * (kx, ky, kz) by -1/(kx^2 + ky^2 + kz^2) and sets the k = 0 entry to zero.
 * Wavenumbers are j for j < ceil(n/2) and j - n otherwise.  The multiplier
 * is real, so the operation is its own adjoint. */
wsfft_status_t wsfft_poisson_symbol(void* data, int64_t nx, int64_t ny, int64_t nz, hipStream_t stream);

/* The whole solve u = Re(F^{-1}[-F[f](k) / |k|^2]) (k = 0 mode zero,
 * wavenumbers as above, F^{-1} including 1/N) without separate elementwise
 * passes.
 *
 * With a real plan of the grid (wsfft_plan_create_real(nx, ny, nz, 0)): five
 * passes over the half spectrum, each moving about half the bytes of a
 * complex pass: the R2C x pass reads f, the forward y pass, one z pass that
 * transforms each z pencil forward, applies the multiplier (kx = 0 .. nx/2)
 * and transforms it back, the inverse y pass, and the C2R x pass that stores
 * u with 1/N.  work: (nx/2+1)*ny*nz complex64.  The fused z pass exists for
 * nz of 32, 64, 128, 256, 512 or 1024 points.
 *
 * With a WSFFT_C64 complex plan of the grid (any sign): six complex passes;
 * the first forward pass reads the real input, the last forward pass
 * applies the multiplier as it stores, and the last inverse pass stores only
 * the real part.  work: nx*ny*nz complex64.  Every axis needs a fused kernel
 * (32, 64, 128, 256, 512 or 1024 points) and a pass of its own: a plan with
 * a fused xy-plane pass (see WSFFT_FLAG_NO_PLANE) is unsupported.
 *
 * f, u: nx*ny*nz FP32 device arrays (x fastest, 4-byte aligned; f and u may
 * be the same array).  work: caller-owned, 8-byte aligned, disjoint from f
 * and u.  Enqueues the launches on `stream`; no allocation or
 * synchronisation.  Returns WSFFT_ERROR_UNSUPPORTED_SIZE for grids without
 * the fused kernels (every axis must be longer than 1 and, for real plans,
 * no axis split); callers then compose the solve from a plan and the three
 * calls above.  The operator is linear and self-adjoint, so its adjoint is
 * the same call. */
wsfft_status_t wsfft_poisson_solve(wsfft_plan_t plan, const float* f, float* u, void* work, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same solve as
 * wsfft_poisson_solve, with its work array taken from a static device buffer
 * of the library instead of an argument.  The buffer holds 72 MiB
 * (75497472 bytes) per GPU, from the library's load until the process ends:
 * enough for a real plan with (nx/2+1)*ny*nz*8 bytes up to that (256^3:
 * 64.5 MiB) or a complex plan with nx*ny*nz*8.  A larger grid returns
 * WSFFT_ERROR_EXCEEDS_SCRATCH before any device work.  The call allocates
 * nothing (the buffer's address on the current device is looked up once, at
 * the first call on that device).  Every call on one GPU shares that GPU's
 * buffer, which keeps the last call's contents (the solve needs no cleared
 * memory): calls that overlap on one GPU -- on different streams, threads or
 * processes' graphs replayed concurrently -- race and give wrong results.
 * Other arguments, errors and results as wsfft_poisson_solve. */
wsfft_status_t wsfft_poisson_solve_noalloc(wsfft_plan_t plan, const float* f, float* u, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* WSFFT_POINTWISE_H */
