/*
 * wsfft: multidimensional complex-to-complex FFT for AMD Instinct MI355X
 * (gfx950), computed as one batched pencil pass ("superstep") per axis with
 * the data redistribution between supersteps done by the passes' own
 * addressing.
 *
 * The problem (paper, Section 1 and Section 2.2): for an nx x ny x nz array a,
 *
 *   X[kx,ky,kz] = sum_{x,y,z} a[x,y,z] exp(sign * 2*pi*i * (kx*x/nx + ky*y/ny + kz*z/nz))
 *
 * computed as 1D DFTs along x, then y, then z (the order does not change the
 * exact result).  sign = -1 is the forward transform.  The inverse of
 * Section 4.2 conjugates the roots of unity and scales by 1/N; here that is
 * wsfft_execute_inverse (or wsfft_execute_adjoint plus a 1/N scale).
 *
 * Layout: dense, interleaved complex, x fastest: element (x, y, z) sits at
 * linear index x + nx*(y + ny*z) -- a contiguous torch tensor of shape
 * (nz, ny, nx).  2D arrays use nz = 1, 1D arrays ny = nz = 1.  Storage types:
 *   WSFFT_C64       FP32 re, FP32 im (8 bytes, 8-byte aligned)
 *   WSFFT_C16_FP16  FP16 re, FP16 im (4 bytes, 4-byte aligned)
 *   WSFFT_C16_BF16  BF16 re, BF16 im (4 bytes, 4-byte aligned)
 * Arithmetic is FP32 (the paper measures FP32 and FP16; Section 4.1 and
 * Section 5), or packed FP16 for WSFFT_C16_FP16 plans created with
 * WSFFT_FLAG_FP16_MATH.  Twiddle factors are evaluated in FP64 on the host and rounded
 * once to nearest even: to the storage type for the 16-bit types, to FP32 for
 * WSFFT_C64 or when WSFFT_FLAG_FP32_TWIDDLES is given.  (The inter-pass
 * twiddles of a WSFFT_C64 unit-stride axis split in two passes are FP64
 * products of two such host tables, formed on the device and rounded once to
 * FP32.)
 *
 * Reduced precision: each pass p of a 16-bit plan multiplies its output by
 * 2^-s_p with s_p = ceil(log2(n_p) / 2), so the stored result is
 * 2^-S * DFT(a) with S = sum of s_p (wsfft_plan_scale_log2), and the inverse
 * (wsfft_execute_inverse) undoes it.  WSFFT_C64 plans have S = 0.
 *
 * Errors: every call validates its arguments before touching the device and
 * returns a status; wsfft_plan_create* return NULL and record the status for
 * wsfft_get_last_error() (thread-local).  Execution calls only enqueue work on
 * the given stream (0 = the null stream): they never allocate, copy from the
 * host or synchronise, so they can be captured in a HIP graph.  Device-side
 * faults surface at the caller's next synchronisation, as in HIP.
 *
 * Ownership: the caller owns `in` and `out` (device pointers on the device
 * that was current when the plan was created) and keeps them alive until the
 * stream work completes.  A plan owns its twiddle tables and, for axes longer
 * than one pass can hold, its work buffer.  Plans are immutable after
 * creation, so one plan may run concurrently on several streams -- except
 * calls that use the plan's work buffer (below), which must not run
 * concurrently with each other.  `in == out` (in place) is allowed for every
 * plan.  Otherwise `in` and `out` must not overlap, and `in` is never written.
 *
 * Work buffer: an axis longer than one pass holds is split into two passes
 * (four-step, paper Section 8), and the first of them cannot write the
 * positions it reads.  A plan with such an axis therefore owns a work buffer
 * of one array (wsfft_plan_work_bytes), allocated at creation; calls go
 * through it when the plan has two split axes, or when it has one and the
 * call is in place.
 *
 * Logging: with the environment variable WSFFT_LOG=1 every plan creation
 * prints the plan's pass schedule (axis, layout, length, kernel variant,
 * workgroup size, tile width, LDS bytes, grid) to stderr.
 */
#ifndef WSFFT_H
#define WSFFT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wsfft_plan_s* wsfft_plan_t;

typedef enum {
    WSFFT_C64 = 0,
    WSFFT_C16_FP16 = 1,
    WSFFT_C16_BF16 = 2
} wsfft_dtype_t;

typedef enum {
    WSFFT_SUCCESS = 0,
    WSFFT_ERROR_INVALID_VALUE = 1,    /* a size < 1, sign not +-1, unknown dtype or flag, count < 0 */
    WSFFT_ERROR_UNSUPPORTED_SIZE = 2, /* an axis with a prime factor other than 2 or 3, or too large */
    WSFFT_ERROR_NULL_POINTER = 3,
    WSFFT_ERROR_MISALIGNED = 4,       /* a pointer not aligned to its element size */
    WSFFT_ERROR_OUT_OF_MEMORY = 5,
    WSFFT_ERROR_NO_DEVICE = 6,        /* no visible HIP device */
    WSFFT_ERROR_HIP = 7,              /* a HIP runtime call failed (e.g. a launch) */
    WSFFT_ERROR_INVALID_PLAN = 8,     /* NULL, destroyed, or created on another device */
    WSFFT_ERROR_WRONG_DEVICE = 9,     /* current device differs from the plan's */
    WSFFT_ERROR_EXCEEDS_SCRATCH = 10  /* more work memory than the static scratch buffer holds */
} wsfft_status_t;

/* Plan flags for wsfft_plan_create_ex. */
#define WSFFT_FLAG_FP32_TWIDDLES 1u   /* 16-bit plans: keep twiddles in FP32 */
#define WSFFT_FLAG_TUNE 2u            /* time each pass's kernel variants at creation */
/* WSFFT_C16_FP16 plans only (else WSFFT_ERROR_INVALID_VALUE): butterflies in
 * packed FP16 arithmetic instead of FP32, as in the paper's FP16 runs (§4.1,
 * §5.1).  Values stay FP16 pairs in registers and LDS; each pass scales its
 * loaded values by its 2^-s_p (so the output is the same 2^-S * DFT as
 * without the flag) and every arithmetic step rounds to FP16.  Twiddles are
 * FP16 whatever WSFFT_FLAG_FP32_TWIDDLES says. */
#define WSFFT_FLAG_FP16_MATH 4u
/* WSFFT_C64 plans whose x and y axes each take one pass and whose xy-plane
 * holds at most 16384 values (axes of 32 .. 256 points) fuse the x and y
 * supersteps into one pass over whole planes in LDS (two HBM round trips
 * for a 3D array instead of three).  This flag keeps them separate. */
#define WSFFT_FLAG_NO_PLANE 8u
/* Infinity Cache policy.  3D plans of three single passes (x, y, z) by
 * default route data through the 256 MB Infinity Cache by array size A:
 * 64 MiB < A <= 128 MiB (WSFFT_C64 only): every pass with cached loads and
 * stores (the next pass reads its input from the cache); 128 MiB < A <=
 * 256 MiB: the x pass with cached stores; A > 256 MiB: the x and y passes run
 * chunk by chunk over groups of xy-planes of at most 256 MiB, the x pass of a
 * chunk with cached stores, so that its y pass reads the chunk from the cache
 * (the z pass then runs once over the whole array).  Results are bitwise
 * equal to the streaming schedule; only the memory traffic differs.  This
 * flag keeps every pass streaming (non-temporal loads and stores, no
 * chunks). */
#define WSFFT_FLAG_STREAMING 16u

/*
 * Autotuning.  Passes of the hot lengths (powers of two up to 1024 strided,
 * 16384 contiguous) have several compiled launch variants (radix schedule,
 * tile width).  With WSFFT_FLAG_TUNE or the environment WSFFT_TUNE=1, plan
 * creation picks, per pass geometry, the variant recorded in the tuning cache
 * ($WSFFT_TUNE_CACHE, else $HOME/.cache/wsfft_tune.txt), or times every
 * variant of uncached geometries with HIP events on two temporary device
 * buffers of one array each (allocated and freed inside plan creation) and
 * appends the winner to the cache.  Without a request, the cache is read only
 * when $WSFFT_TUNE_CACHE is set, so by default a plan's kernels depend on its
 * arguments alone.  WSFFT_TUNE=0 disables both, and the diagnostic
 * WSFFT_TUNE_FORCE=<v> selects variant v wherever it exists.  Execution is
 * unaffected: the chosen kernels are fixed in the plan.
 */

/*
 * Create a plan for an nx x ny x nz transform of the given storage type with
 * kernel sign `sign` (-1 forward, +1 backward).  Every axis length must be
 * of the form 2^a 3^b and at most WSFFT_MAX_AXIS (2^20); an axis longer than
 * one pass holds (16384 unit-stride, 1024 strided) must split into two
 * factors of at most 1024.  The whole array holds at most 2^40 elements and
 * each pass at most 2^32 - 1 work-items.  Builds the twiddle tables (one per
 * distinct pass length) in FP64 on the host, rounds them and copies them to
 * the current device.
 * Returns NULL on error (see wsfft_get_last_error).
 */
#define WSFFT_MAX_AXIS 1048576
wsfft_plan_t wsfft_plan_create(int64_t nx, int64_t ny, int64_t nz, wsfft_dtype_t dtype, int sign);
wsfft_plan_t wsfft_plan_create_ex(int64_t nx, int64_t ny, int64_t nz, wsfft_dtype_t dtype, int sign,
                                  unsigned flags);

/* Status of the last wsfft_plan_create* call on this thread. */
wsfft_status_t wsfft_get_last_error(void);

/* out = 2^-S * sum with the plan's sign (unnormalised).  The superstep
 * sequence of Section 1: one pass per axis of length > 1. */
wsfft_status_t wsfft_execute(wsfft_plan_t plan, const void* in, void* out, hipStream_t stream);

/* out = 2^-S * sum with the opposite sign, unnormalised: the adjoint (conjugate
 * transpose) of wsfft_execute for C64 plans.  Section 4.2's inverse reverses
 * the steps with conjugated roots. */
wsfft_status_t wsfft_execute_adjoint(wsfft_plan_t plan, const void* in, void* out, hipStream_t stream);

/* out = 2^S / N * sum with the opposite sign: the inverse of wsfft_execute
 * (Section 4.2), wsfft_execute_inverse(wsfft_execute(a)) = a.  C64 plans
 * (S = 0) fold the 1/N into the last pass; 16-bit plans scale pass p by
 * 2^s_p / n_p (about 1/sqrt(n_p), like the forward 2^-s_p), which keeps every
 * stored value in range. */
wsfft_status_t wsfft_execute_inverse(wsfft_plan_t plan, const void* in, void* out, hipStream_t stream);

/*
 * `count` independent transforms in one call: transform i runs plans[i] from
 * in[i] to out[i] (adjoint != 0 selects wsfft_execute_adjoint semantics).
 * Plans may differ in shape; they must share dtype and device.  The work is
 * issued pass by pass: all arrays' first passes in one launch, then all
 * second passes, then all third (fewer launches when shapes allow), so the
 * whole batch is a handful of launches that a HIP graph can capture.  The
 * same plan may appear several times (e.g. one plan over many pencils);
 * entries whose call would use their plan's work buffer (see above) may not
 * (WSFFT_ERROR_INVALID_VALUE).  When every entry uses the same plan and
 * both in[i] and out[i] advance by exactly one array per entry, each pass is
 * a single launch over the whole batch.  Validation covers every entry
 * before any work is enqueued.
 */
wsfft_status_t wsfft_execute_batched(int count, const wsfft_plan_t* plans, const void* const* in,
                                     void* const* out, int adjoint, hipStream_t stream);

/*
 * Batch-level autotuning (paper Section 5.3 runs many small transforms side
 * by side; here their merged launches are tuned as launched).  Runs the batch
 * of wsfft_execute_batched with the same arguments, timing every merged
 * launch (several arrays' pass in one launch) in each compiled launch variant
 * with HIP events on `stream`, and records the fastest for that launch, keyed
 * by its kernel shape, storage type, sign and every member's geometry, for
 * the rest of the process.  Later wsfft_execute_batched calls that produce
 * the same launch run the recorded variant (otherwise the one most of its
 * entries' plans chose).  Argument checks as for wsfft_execute_batched.
 * Synchronises `stream`.  Each launch runs several times, so afterwards
 * `out` holds unspecified values (and so does `in` where in == out); the
 * caller's next wsfft_execute_batched computes the transform as usual.
 * Thread-safe; the records are process-wide.
 */
wsfft_status_t wsfft_tune_batched(int count, const wsfft_plan_t* plans, const void* const* in, void* const* out,
                                  int adjoint, hipStream_t stream);

/* Enqueue only pass `index` (0-based, < wsfft_plan_num_passes) of the
 * transform wsfft_execute (mode 0), wsfft_execute_adjoint (1) or
 * wsfft_execute_inverse (2) would run, with the same buffers.  Running every
 * index in order equals the full call (a plan whose x and y passes run in
 * plane chunks runs each over the whole array here); one index alone is for
 * per-pass timing and profiling.  On a real plan, mode 0 indexes the passes of
 * wsfft_execute_r2c, modes 1 and 2 those of wsfft_execute_c2r and
 * wsfft_execute_c2r_inverse (4-byte alignment is checked for both buffers). */
wsfft_status_t wsfft_execute_pass(wsfft_plan_t plan, int index, int mode, const void* in, void* out,
                                  hipStream_t stream);

/*
 * Batch plans: a whole batch as ONE persistent kernel launch.
 *
 * wsfft_batch_plan_create binds `count` plans and their buffers (same
 * meaning as wsfft_execute_batched; buffers must stay valid while the batch
 * plan is used), checks every entry, uploads a table of the supersteps of all
 * arrays and allocates the batch plan's own completion counters.
 * wsfft_batch_execute then enqueues one launch of a resident grid that walks
 * every tile of every pass of every array in superstep order; tiles of
 * superstep L start once all tiles of superstep L-1 (of every array) are
 * done, a grid-wide barrier per superstep inside the one launch.  No host
 * copies or allocations happen in execute, so it can be captured in a HIP
 * graph.  A batch plan must not run concurrently with itself (its counters
 * are shared by its launches).  Supported: WSFFT_C64 plans whose axes are 32,
 * 64, 96, 128 or 256 long (or 1), one effective sign across the batch; other
 * batches return WSFFT_ERROR_UNSUPPORTED_SIZE and should use
 * wsfft_execute_batched.  Dependency waits are bounded: a launch in which one
 * timed out has invalid results and is counted on the device;
 * wsfft_batch_plan_check synchronises the device, reports whether any launch
 * since the plan's creation or the previous check timed out, and clears the
 * count.  Each launch starts with fresh counters, so a timed-out launch does
 * not affect later ones.  wsfft_batch_plan_set_spin_limit (a diagnostic)
 * sets the polls after which a wait gives up (default 2^22); a tiny limit
 * forces timeouts from the host, and the launch still runs every tile and
 * exits.  NULL on error (wsfft_batch_get_last_error).
 */
typedef struct wsfft_batch_plan_s* wsfft_batch_plan_t;
wsfft_batch_plan_t wsfft_batch_plan_create(int count, const wsfft_plan_t* plans, const void* const* in,
                                           void* const* out, int adjoint);
wsfft_status_t wsfft_batch_get_last_error(void);
wsfft_status_t wsfft_batch_execute(wsfft_batch_plan_t batch, hipStream_t stream);
int64_t wsfft_batch_plan_tiles(wsfft_batch_plan_t batch);      /* work items per execution; -1 invalid */
wsfft_status_t wsfft_batch_plan_check(wsfft_batch_plan_t batch, int* timed_out);
wsfft_status_t wsfft_batch_plan_set_spin_limit(wsfft_batch_plan_t batch, unsigned polls);
void wsfft_batch_plan_destroy(wsfft_batch_plan_t batch);

/*
 * Real input and output (complex64 storage, FP32 arithmetic).  The paper's
 * transform (Section 1) of a real array is Hermitian, X[-k] = conj(X[k]), so
 * the bins kx = 0 .. nx/2 determine it: the half spectrum, an
 * (nx/2 + 1) x ny x nz complex64 array, x fastest (the shape (nz, ny,
 * nx/2 + 1) of a contiguous tensor).  The paper evaluates complex data only
 * (Section 5); these calls halve the bytes every pass moves for real data.
 *
 * wsfft_plan_create_real: nx even, 4 <= nx <= 32768, every axis 2^a 3^b and
 * at most WSFFT_MAX_AXIS (ny, nz longer than 1024 split into two passes
 * through a plan-owned work buffer of one half spectrum); flags must be 0.
 * NULL on error (wsfft_get_last_error).  The x pass transforms the nx reals
 * of a pencil as nx/2 complex pairs and recombines the even and odd halves;
 * the y and z passes are the complex passes over the half spectrum.
 *
 * wsfft_execute_r2c: out = the half spectrum of the forward (sign -1),
 * unnormalised transform of the real array `in` (nx*ny*nz FP32, 4-byte
 * aligned); out: (nx/2+1)*ny*nz complex64, 8-byte aligned.  `in` is not
 * written.
 * wsfft_execute_c2r: out = the sign +1, unnormalised transform of the
 * Hermitian extension of the half spectrum `in`: sign +1 DFTs along z and y
 * as given, then along x the extension Y[k], conj(Y[nx-k]) with the real
 * parts of Y[0] and Y[nx/2] (their imaginary parts are ignored).  `in` is
 * overwritten (its y and z passes run in place there); out: nx*ny*nz FP32.
 * wsfft_execute_c2r_inverse: the same times 1/(nx*ny*nz), so that
 * c2r_inverse(r2c(a)) = a.
 * `in` and `out` must not overlap (in == out returns
 * WSFFT_ERROR_INVALID_VALUE); wsfft_execute and the complex calls return
 * WSFFT_ERROR_INVALID_VALUE for a real plan, and the real calls for a complex
 * plan.  Enqueue only, like every execute call.
 * wsfft_plan_is_real: 1 for a real plan, 0 for a complex one, -1 invalid.
 *
 * wsfft_plan_create_real_ex: the same with half-spectrum rows `half_pitch`
 * complex values apart (0: nx/2 + 1, the compact layout above; otherwise at
 * least nx/2 + 1, else WSFFT_ERROR_INVALID_VALUE): element (kx, y, z) of the
 * half spectrum sits at kx + half_pitch*(y + ny*z), a tensor of shape (nz,
 * ny, half_pitch) of which [..., :nx/2+1] is the spectrum.  Compact rows of
 * nx/2 + 1 complex64 are not whole 128-byte cache lines apart, so passes
 * that stream across rows share lines between tiles; a pitch that is a
 * multiple of 16 makes every row line-aligned, and the plan's y and z
 * passes then stream whole rows.  Those passes transform the padding columns
 * along with the spectrum, so the padding positions hold unspecified values
 * after a call (they never reach the result).  The Poisson solve
 * (wsfft_pointwise.h) takes compact real plans only.
 */
wsfft_plan_t wsfft_plan_create_real(int64_t nx, int64_t ny, int64_t nz, unsigned flags);
wsfft_plan_t wsfft_plan_create_real_ex(int64_t nx, int64_t ny, int64_t nz, unsigned flags, int64_t half_pitch);
wsfft_status_t wsfft_execute_r2c(wsfft_plan_t plan, const float* in, void* out, hipStream_t stream);
wsfft_status_t wsfft_execute_c2r(wsfft_plan_t plan, void* in, float* out, hipStream_t stream);
wsfft_status_t wsfft_execute_c2r_inverse(wsfft_plan_t plan, void* in, float* out, hipStream_t stream);
int wsfft_plan_is_real(wsfft_plan_t plan);

/* S of the stored 2^-S scaling (0 for WSFFT_C64); -1 for an invalid plan. */
int wsfft_plan_scale_log2(wsfft_plan_t plan);

/* Number of HBM passes one execute makes (real plans: wsfft_execute_r2c);
 * -1 for an invalid plan. */
int wsfft_plan_num_passes(wsfft_plan_t plan);

/* Bytes of plan-owned device work buffer (one array, for real plans one
 * half spectrum, if an axis is split into two passes, else 0); -1 for an
 * invalid plan. */
int64_t wsfft_plan_work_bytes(wsfft_plan_t plan);

/* Writes a one-line, NUL-terminated description of the pass schedule into
 * buf (at most len bytes).  Returns the status. */
wsfft_status_t wsfft_plan_describe(wsfft_plan_t plan, char* buf, size_t len);

/* Synchronises the plan's device, then frees the plan.  NULL is ignored. */
void wsfft_plan_destroy(wsfft_plan_t plan);

/* Static string for a status code. */
const char* wsfft_status_string(wsfft_status_t status);

#ifdef __cplusplus
}
#endif

#endif /* WSFFT_H */
