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

#ifdef __cplusplus
}
#endif

#endif /* WSFFT_POINTWISE_H */
