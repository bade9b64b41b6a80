// Elementwise kernels around the FFT for the spectral Poisson solve
// u = IFFT(-FFT(f) / |k|^2), k = 0 mode zeroed: widening a real field to
// complex, taking the real part, and the spectral multiply.  Each is one
// streaming pass; grid-stride loops with 16-byte accesses where possible.
#include <hip/hip_runtime.h>

#include "../../include/wsfft.h"
#include "../../include/wsfft_pointwise.h"

namespace {

constexpr int kThreads = 256;

unsigned blocks_for(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b > 65536) b = 65536;   // grid-stride beyond this
    return (unsigned)(b < 1 ? 1 : b);
}

__global__ __launch_bounds__(kThreads) void real_to_complex_kernel(const float* __restrict__ in,
                                                                   float2* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        out[i] = make_float2(in[i], 0.0f);
}

__global__ __launch_bounds__(kThreads) void complex_real_part_kernel(const float2* __restrict__ in,
                                                                     float* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        out[i] = in[i].x;
}

// Integer wavenumber of index j on an axis of length n: j for j < ceil(n/2),
// j - n otherwise (the Nyquist index n/2 of an even axis maps to -n/2).
__device__ __forceinline__ float wavenumber(int64_t j, int64_t n) {
    return (float)(j < (n + 1) / 2 ? j : j - n);
}

__global__ __launch_bounds__(kThreads) void poisson_symbol_kernel(float2* __restrict__ x, int64_t nx,
                                                                  int64_t ny, int64_t nz) {
    const int64_t n = nx * ny * nz;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const int64_t ix = i % nx, r = i / nx;
        const int64_t iy = r % ny, iz = r / ny;
        const float kx = wavenumber(ix, nx), ky = wavenumber(iy, ny), kz = wavenumber(iz, nz);
        const float k2 = kx * kx + ky * ky + kz * kz;
        const float s = k2 > 0.0f ? -1.0f / k2 : 0.0f;
        const float2 v = x[i];
        x[i] = make_float2(v.x * s, v.y * s);
    }
}

bool aligned(const void* p, uintptr_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace

extern "C" {

wsfft_status_t wsfft_real_to_complex(const float* in, void* out, int64_t n, hipStream_t stream) {
    if (n < 0) return WSFFT_ERROR_INVALID_VALUE;
    if (n == 0) return WSFFT_SUCCESS;
    if (!in || !out) return WSFFT_ERROR_NULL_POINTER;
    if (!aligned(in, 4) || !aligned(out, 8)) return WSFFT_ERROR_MISALIGNED;
    hipLaunchKernelGGL(real_to_complex_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, stream, in,
                       (float2*)out, n);
    return hipGetLastError() == hipSuccess ? WSFFT_SUCCESS : WSFFT_ERROR_HIP;
}

wsfft_status_t wsfft_complex_real_part(const void* in, float* out, int64_t n, hipStream_t stream) {
    if (n < 0) return WSFFT_ERROR_INVALID_VALUE;
    if (n == 0) return WSFFT_SUCCESS;
    if (!in || !out) return WSFFT_ERROR_NULL_POINTER;
    if (!aligned(in, 8) || !aligned(out, 4)) return WSFFT_ERROR_MISALIGNED;
    hipLaunchKernelGGL(complex_real_part_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, stream,
                       (const float2*)in, out, n);
    return hipGetLastError() == hipSuccess ? WSFFT_SUCCESS : WSFFT_ERROR_HIP;
}

wsfft_status_t wsfft_poisson_symbol(void* data, int64_t nx, int64_t ny, int64_t nz, hipStream_t stream) {
    if (nx < 1 || ny < 1 || nz < 1) return WSFFT_ERROR_INVALID_VALUE;
    if (!data) return WSFFT_ERROR_NULL_POINTER;
    if (!aligned(data, 8)) return WSFFT_ERROR_MISALIGNED;
    hipLaunchKernelGGL(poisson_symbol_kernel, dim3(blocks_for(nx * ny * nz)), dim3(kThreads), 0, stream,
                       (float2*)data, nx, ny, nz);
    return hipGetLastError() == hipSuccess ? WSFFT_SUCCESS : WSFFT_ERROR_HIP;
}

}  // extern "C"
