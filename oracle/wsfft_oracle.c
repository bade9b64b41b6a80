/*
 * FP64 CPU oracle for the multidimensional complex-to-complex DFT.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, table or helper with the
 * HIP implementation.
 *
 * What it computes (paper, Section 1 and Section 2.2): the DFT of a k-dimensional
 * array equals 1D DFTs applied along each axis in turn ("supersteps"), in any
 * order.  Here an array is stored x fastest, element (x, y, z) at linear index
 * x + nx*(y + ny*z), re/im interleaved (paper, Section 4.1 keeps re and im of
 * each element side by side).  The result is
 *
 *   X[kx,ky,kz] = sum_{x,y,z} a[x,y,z] * exp(sign * 2*pi*i * (kx*x/nx + ky*y/ny + kz*z/nz))
 *
 * unnormalised; sign = -1 is the forward transform (the pencil pseudocode of
 * Section 4.1 multiplies odd terms by the conjugate root, and the paper checks
 * its output against NumPy, whose forward kernel is exp(-2*pi*i*jk/n)).  The
 * inverse of Section 4.2 is the sign = +1 sum scaled by 1/N; scaling is left to
 * the caller.
 *
 * Each 1D transform is a recursive mixed-radix Cooley-Tukey decimation in time
 * (Section 4.1 describes the radix-2 case: split into even and odd
 * subsequences, transform each, recombine with roots of unity).  Here the
 * split is by the smallest prime factor p of n, so every n is handled: radix 2
 * and 3 for the sizes the GPU supports, and an O(p) combine for any other
 * prime.  Roots of unity are evaluated in FP64 from the exactly reduced integer
 * argument (q*k mod n), never by repeated multiplication.
 *
 * Pencils are independent within an axis, so they are split across POSIX
 * threads with no reduction: the output does not depend on the thread count.
 *
 * Parity status: pinned.  The tests check this file against a brute-force
 * evaluation of the definition above, closed forms (delta, constant, plane
 * wave, geometric sequence, shift theorem), hand-derived textbook values,
 * Parseval, Hermitian symmetry, linearity and the round trip.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double re, im; } oc_t;

/* exp(sign * 2*pi*i * t / n) for integer 0 <= t < n. */
static oc_t root_of_unity(int64_t t, int64_t n, int sign)
{
    /* Reduce to an angle in [0, 2*pi) from the exact integer ratio. */
    const double ang = 2.0 * M_PI * (double)t / (double)n;
    oc_t w;
    w.re = cos(ang);
    w.im = (double)sign * sin(ang);
    return w;
}

static int64_t smallest_prime_factor(int64_t n)
{
    if (n % 2 == 0) return 2;
    for (int64_t p = 3; p * p <= n; p += 2)
        if (n % p == 0) return p;
    return n;
}

/* Table of the n-th roots of unity W_n^j, j in [0, n). */
static oc_t* make_roots(int64_t n, int sign)
{
    oc_t* w = (oc_t*)malloc((size_t)n * sizeof(oc_t));
    if (!w) return NULL;
    for (int64_t j = 0; j < n; ++j) w[j] = root_of_unity(j, n, sign);
    return w;
}

/*
 * out[0..n) = DFT_n of in[0], in[s], in[2s], ...
 * roots: W_ntop^j for j in [0, ntop); W_n^j = roots[j * (ntop / n)].
 * tmp: at least n elements of scratch, never aliasing out.
 */
static void dft_rec(const oc_t* in, int64_t s, oc_t* out, int64_t n,
                    const oc_t* roots, int64_t ntop, oc_t* tmp)
{
    if (n == 1) { out[0] = in[0]; return; }
    const int64_t p = smallest_prime_factor(n);
    const int64_t m = n / p;
    /* Sub-transform q takes the elements whose index is q mod p; its output
     * goes to out[q*m .. q*m + m). */
    for (int64_t q = 0; q < p; ++q)
        dft_rec(in + q * s, s * p, out + q * m, m, roots, ntop, tmp);
    /* Recombine: X[k1 + m*k2] = sum_q W_n^(q*(k1 + m*k2)) F_q[k1]. */
    const int64_t rstride = ntop / n;
    for (int64_t k1 = 0; k1 < m; ++k1) {
        for (int64_t q = 0; q < p; ++q) tmp[q] = out[q * m + k1];
        for (int64_t k2 = 0; k2 < p; ++k2) {
            const int64_t k = k1 + m * k2;
            double re = 0.0, im = 0.0;
            for (int64_t q = 0; q < p; ++q) {
                const oc_t w = roots[((q * k) % n) * rstride];
                re += tmp[q].re * w.re - tmp[q].im * w.im;
                im += tmp[q].re * w.im + tmp[q].im * w.re;
            }
            out[k].re = re;
            out[k].im = im;
        }
    }
}

/* One 1D transform over a strided pencil: in and out are pencil bases. */
static void dft_pencil(const oc_t* in, oc_t* out, int64_t n, int64_t stride,
                       const oc_t* roots, oc_t* buf, oc_t* res, oc_t* tmp)
{
    for (int64_t j = 0; j < n; ++j) buf[j] = in[j * stride];
    dft_rec(buf, 1, res, n, roots, n, tmp);
    for (int64_t j = 0; j < n; ++j) out[j * stride] = res[j];
}

typedef struct {
    const oc_t* src;
    oc_t* dst;
    int64_t n, stride;      /* pencil length and element stride          */
    int64_t inner, outer;   /* pencil (i, o) base = i + o * inner * n    */
    int64_t p0, p1;         /* pencil range [p0, p1) of inner * outer    */
    const oc_t* roots;
    int status;
} axis_job_t;

static void* axis_worker(void* arg)
{
    axis_job_t* J = (axis_job_t*)arg;
    oc_t* buf = (oc_t*)malloc((size_t)J->n * 3 * sizeof(oc_t));
    if (!buf) { J->status = -1; return NULL; }
    for (int64_t p = J->p0; p < J->p1; ++p) {
        const int64_t i = p % J->inner, o = p / J->inner;
        const int64_t base = i + o * J->inner * J->n;
        dft_pencil(J->src + base, J->dst + base, J->n, J->stride, J->roots,
                   buf, buf + J->n, buf + 2 * J->n);
    }
    free(buf);
    J->status = 0;
    return NULL;
}

/* Transform every pencil along one axis.  The pencils of axis a with
 * length n have element stride `inner` (product of the faster axes) and
 * there are inner*outer of them. */
static int transform_axis(const oc_t* src, oc_t* dst, int64_t n, int64_t inner,
                          int64_t outer, int sign, int nthreads)
{
    if (n == 1) {
        if (src != dst) memcpy(dst, src, (size_t)(inner * outer) * sizeof(oc_t));
        return 0;
    }
    oc_t* roots = make_roots(n, sign);
    if (!roots) return -1;
    const int64_t npencils = inner * outer;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > npencils) nthreads = (int)npencils;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    axis_job_t* jobs = (axis_job_t*)malloc(sizeof(axis_job_t) * (size_t)nthreads);
    if (!th || !jobs) { free(roots); free(th); free(jobs); return -1; }
    int rc = 0;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].src = src; jobs[t].dst = dst;
        jobs[t].n = n; jobs[t].stride = inner;
        jobs[t].inner = inner; jobs[t].outer = outer;
        jobs[t].p0 = npencils * t / nthreads;
        jobs[t].p1 = npencils * (t + 1) / nthreads;
        jobs[t].roots = roots;
        jobs[t].status = -1;
    }
    int started = 0;
    for (int t = 1; t < nthreads; ++t, ++started)
        if (pthread_create(&th[t], NULL, axis_worker, &jobs[t]) != 0) break;
    axis_worker(&jobs[0]);
    for (int t = 1; t <= started; ++t) pthread_join(th[t], NULL);
    for (int t = 0; t < nthreads; ++t)
        if (t <= started && jobs[t].status != 0) rc = -1;
    if (started != nthreads - 1) rc = -1;
    free(th); free(jobs); free(roots);
    return rc;
}

/*
 * 3D transform, x then y then z (any order gives the same result in exact
 * arithmetic; Section 1).  in and out may alias.  Returns 0 on success.
 */
int oracle_fftn(const double* in, double* out, int64_t nx, int64_t ny,
                int64_t nz, int sign, int nthreads)
{
    if (nx < 1 || ny < 1 || nz < 1 || (sign != 1 && sign != -1)) return -2;
    const oc_t* a = (const oc_t*)in;
    oc_t* b = (oc_t*)out;
    if (transform_axis(a, b, nx, 1, ny * nz, sign, nthreads)) return -1;
    if (transform_axis(b, b, ny, nx, nz, sign, nthreads)) return -1;
    if (transform_axis(b, b, nz, nx * ny, 1, sign, nthreads)) return -1;
    return 0;
}

/* Same transform with the axes taken z, then y, then x. */
int oracle_fftn_zyx(const double* in, double* out, int64_t nx, int64_t ny,
                    int64_t nz, int sign, int nthreads)
{
    if (nx < 1 || ny < 1 || nz < 1 || (sign != 1 && sign != -1)) return -2;
    const oc_t* a = (const oc_t*)in;
    oc_t* b = (oc_t*)out;
    if (transform_axis(a, b, nz, nx * ny, 1, sign, nthreads)) return -1;
    if (transform_axis(b, b, ny, nx, nz, sign, nthreads)) return -1;
    if (transform_axis(b, b, nx, 1, ny * nz, sign, nthreads)) return -1;
    return 0;
}

/*
 * `count` independent 1D transforms of length n, pencil i at in + i*n
 * (contiguous batch).  in and out may alias.
 */
int oracle_fft1d_batch(const double* in, double* out, int64_t n, int64_t count,
                       int sign, int nthreads)
{
    if (n < 1 || count < 0 || (sign != 1 && sign != -1)) return -2;
    if (count == 0) return 0;
    return transform_axis((const oc_t*)in, (oc_t*)out, n, 1, count, sign, nthreads);
}
