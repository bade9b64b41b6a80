// Device side of the pencil FFT passes for gfx950 (CDNA4, wave64).
//
// One pass = one superstep of the multidimensional FFT (paper, Section 1 and
// Section 2.2): a batch of independent 1D DFTs ("pencils") of length N along
// one axis.  The redistribution between supersteps (paper, Section 4.3) is
// done by addressing: a workgroup loads a tile of pencils straight from HBM
// with coalesced row segments, transforms them through registers and LDS and
// writes the results back to the same positions.
//
// Each 1D transform is a Stockham autosort Cooley-Tukey FFT (paper, Section
// 4.1 describes the radix-2 form, which keeps the even and odd halves
// contiguous so no bit reversal is needed).  Here the stages use radix 2, 3,
// 4, 8 and 16.  Stage s with radix R and current sub-transform length Ns
// takes butterfly b in [0, N/R):
//   inputs  x[b + r*N/R], r in [0, R)
//   twiddle x[b + r*N/R] *= W_(Ns*R)^((b mod Ns) * r)
//   R-point DFT
//   outputs y[(b div Ns)*Ns*R + (b mod Ns) + r*Ns]
// The first stage's inputs and the last stage's outputs both sit at
// b + r*N/R, so global loads and stores share one coalesced pattern.
//
// Complex products use fused multiply-adds (paper, Section 4.1 fuses the
// four multiplies and two adds of a complex product into FMAC operations).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace wsfft {

// ---------------------------------------------------------------- complex ---
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 w) {
    return make_float2(fmaf(a.x, w.x, -a.y * w.y), fmaf(a.x, w.y, a.y * w.x));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a * (SIGN * i)
template <int SIGN> __device__ __forceinline__ float2 crot90(float2 a) {
    return SIGN < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}
__device__ __forceinline__ float2 cneg(float2 a) { return make_float2(-a.x, -a.y); }
// v + s*t
__device__ __forceinline__ float2 cfma_s(float2 t, float s, float2 v) {
    return make_float2(fmaf(s, t.x, v.x), fmaf(s, t.y, v.y));
}
// a * h*(sr + i*si) with sr, si = +-1 (an eighth turn when h = 1/sqrt(2))
template <bool RP, bool IP> __device__ __forceinline__ float2 crot45(float2 a, float h) {
    const float ax = a.x, ay = a.y;
    const float re = (RP ? ax : -ax) - (IP ? ay : -ay);
    const float im = (IP ? ax : -ax) + (RP ? ay : -ay);
    return make_float2(h * re, h * im);
}
template <class C> __device__ __forceinline__ C cconst(double re, double im);
template <> __device__ __forceinline__ float2 cconst<float2>(double re, double im) {
    return make_float2((float)re, (float)im);
}

// The same operations on packed FP16 pairs (re in the low half): one packed
// instruction per complex add, two per complex multiply.
typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ h16x2 hswap(h16x2 a) { return __builtin_shufflevector(a, a, 1, 0); }
__device__ __forceinline__ h16x2 hsplat(_Float16 x) { return (h16x2){x, x}; }
__device__ __forceinline__ h16x2 cadd(h16x2 a, h16x2 b) { return a + b; }
__device__ __forceinline__ h16x2 csub(h16x2 a, h16x2 b) { return a - b; }
__device__ __forceinline__ h16x2 cneg(h16x2 a) { return -a; }
__device__ __forceinline__ h16x2 cmul(h16x2 a, h16x2 w) {
    // (a.x w.x - a.y w.y, a.y w.x + a.x w.y)
    const h16x2 wi = (h16x2){-w.y, w.y};
    return __builtin_elementwise_fma(hswap(a), wi, a * hsplat(w.x));
}
__device__ __forceinline__ h16x2 cscale(h16x2 a, float s) { return a * hsplat((_Float16)s); }
template <int SIGN> __device__ __forceinline__ h16x2 crot90(h16x2 a) {
    const h16x2 b = hswap(a);
    return SIGN < 0 ? b * (h16x2){1, -1} : b * (h16x2){-1, 1};
}
__device__ __forceinline__ h16x2 cfma_s(h16x2 t, float s, h16x2 v) {
    return __builtin_elementwise_fma(t, hsplat((_Float16)s), v);
}
template <bool RP, bool IP> __device__ __forceinline__ h16x2 crot45(h16x2 a, float h) {
    const _Float16 r = (_Float16)(RP ? h : -h), i = (_Float16)(IP ? h : -h);
    return __builtin_elementwise_fma(hswap(a), (h16x2){-i, i}, a * hsplat(r));
}
template <> __device__ __forceinline__ h16x2 cconst<h16x2>(double re, double im) {
    return (h16x2){(_Float16)re, (_Float16)im};
}
typedef float f32x2 __attribute__((ext_vector_type(2)));
// A table entry (FP32 pair) as a register value.
template <class C> __device__ __forceinline__ C cvt_value(f32x2 w);
template <> __device__ __forceinline__ float2 cvt_value<float2>(f32x2 w) { return make_float2(w.x, w.y); }
template <> __device__ __forceinline__ h16x2 cvt_value<h16x2>(f32x2 w) { return __builtin_convertvector(w, h16x2); }

// ------------------------------------------------------- small-radix DFTs ---
// In-place R-point DFT of v[0..R) with kernel exp(SIGN * 2*pi*i*j*k/R).
template <int R, int SIGN> struct Dft;

template <int SIGN> struct Dft<2, SIGN> {
    template <class C> static __device__ __forceinline__ void run(C* v) {
        const C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <int SIGN> struct Dft<3, SIGN> {
    template <class C> static __device__ __forceinline__ void run(C* v) {
        const float h = 0.86602540378443864676f;   // sin(2*pi/3)
        const C t = cadd(v[1], v[2]);
        const C d = csub(v[1], v[2]);
        const C m = cfma_s(t, -0.5f, v[0]);
        const C r = crot90<SIGN>(cscale(d, h));   // SIGN*i*sin(2pi/3)*d
        v[0] = cadd(v[0], t);
        v[1] = cadd(m, r);
        v[2] = csub(m, r);
    }
};

template <int SIGN> struct Dft<4, SIGN> {
    template <class C> static __device__ __forceinline__ void run(C* v) {
        const C t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        const C t2 = cadd(v[1], v[3]), t3 = crot90<SIGN>(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
};

// 8 = 2 x 4: even/odd 4-point DFTs, odd part twiddled by W_8^k.
template <int SIGN> struct Dft<8, SIGN> {
    template <class C> static __device__ __forceinline__ void run(C* v) {
        const float c = 0.70710678118654752440f;
        C e[4] = {v[0], v[2], v[4], v[6]};
        C o[4] = {v[1], v[3], v[5], v[7]};
        Dft<4, SIGN>::run(e);
        Dft<4, SIGN>::run(o);
        // W_8^1 = c*(1 + SIGN*i), W_8^2 = SIGN*i, W_8^3 = c*(-1 + SIGN*i)
        o[1] = crot45<true, (SIGN > 0)>(o[1], c);
        o[2] = crot90<SIGN>(o[2]);
        o[3] = crot45<false, (SIGN > 0)>(o[3], c);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = cadd(e[k], o[k]);
            v[k + 4] = csub(e[k], o[k]);
        }
    }
};

// ------------------------------------------- compile-time roots of unity ---
constexpr double kTwoPi = 6.28318530717958647692528676655900577;

constexpr double taylor_sin(double x) {   // |x| <= pi/4
    double term = x, sum = x;
    for (int k = 1; k < 12; ++k) {
        term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double taylor_cos(double x) {   // |x| <= pi/4
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 12; ++k) {
        term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}
struct CosSin {
    double c, s;
};
// cos and sin of 2*pi*m/R, reduced to the first octant by exact symmetry.
constexpr CosSin root_cs(int m, int R) {
    m = ((m % R) + R) % R;
    const int u = 4 * m, q = u / R, r = u % R;   // angle = (pi/2) * (q + r/R)
    double c = 1.0, s = 0.0;
    if (2 * r <= R) {
        const double phi = (kTwoPi / 4.0) * r / R;
        c = taylor_cos(phi);
        s = taylor_sin(phi);
    } else {
        const double phi = (kTwoPi / 4.0) * (R - r) / R;
        c = taylor_sin(phi);
        s = taylor_cos(phi);
    }
    switch (q & 3) {
        case 0: return {c, s};
        case 1: return {-s, c};
        case 2: return {-c, -s};
        default: return {s, -c};
    }
}

// a * W_R^M with W_R = exp(SIGN*2*pi*i/R); quarter turns are exact swaps,
// eighth turns cost one multiply per component.
template <int R, int M, int SIGN, class C>
__device__ __forceinline__ C twc(C a) {
    constexpr int m = M % R;
    if constexpr (m == 0) {
        return a;
    } else if constexpr ((4 * m) % R == 0) {
        constexpr int q = 4 * m / R;
        if constexpr (q == 1) return crot90<SIGN>(a);
        else if constexpr (q == 2) return cneg(a);
        else return crot90<-SIGN>(a);
    } else if constexpr ((8 * m) % R == 0) {
        constexpr CosSin w = root_cs(m, R);
        constexpr float h = 0.70710678118654752440f;
        constexpr bool cp = w.c > 0, sp = (SIGN * w.s) > 0;   // signs of re, im of W
        return crot45<cp, sp>(a, h);
    } else {
        constexpr CosSin w = root_cs(m, R);
        return cmul(a, cconst<C>(w.c, SIGN * w.s));
    }
}

// Composite R = R1*R2 DFT (Cooley-Tukey within registers):
//   X[k1 + R1*k2] = sum_n2 W_R2^(n2 k2) W_R^(n2 k1) sum_n1 x[R2 n1 + n2] W_R1^(n1 k1)
template <int R1, int R2, int SIGN> struct DftComp {
    static constexpr int R = R1 * R2;
    template <int I, class C>
    static __device__ __forceinline__ void twiddle(C* y) {
        if constexpr (I < R) {
            constexpr int n2 = I / R1, k1 = I % R1;
            y[I] = twc<R, n2 * k1, SIGN>(y[I]);
            twiddle<I + 1>(y);
        }
    }
    template <class C> static __device__ __forceinline__ void run(C* v) {
        C y[R];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) {
            C u[R1];
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) u[n1] = v[R2 * n1 + n2];
            Dft<R1, SIGN>::run(u);
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) y[n2 * R1 + k1] = u[k1];
        }
        twiddle<0>(y);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            C w[R2];
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) w[n2] = y[n2 * R1 + k1];
            Dft<R2, SIGN>::run(w);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = w[k2];
        }
    }
};

template <int SIGN> struct Dft<6, SIGN> : DftComp<2, 3, SIGN> {};
template <int SIGN> struct Dft<9, SIGN> : DftComp<3, 3, SIGN> {};
template <int SIGN> struct Dft<12, SIGN> : DftComp<4, 3, SIGN> {};
template <int SIGN> struct Dft<16, SIGN> : DftComp<4, 4, SIGN> {};
template <int SIGN> struct Dft<18, SIGN> : DftComp<2, 9, SIGN> {};
template <int SIGN> struct Dft<24, SIGN> : DftComp<8, 3, SIGN> {};
template <int SIGN> struct Dft<27, SIGN> : DftComp<3, 9, SIGN> {};
template <int SIGN> struct Dft<32, SIGN> : DftComp<8, 4, SIGN> {};

// ------------------------------------------------------ stage schedule ---
struct Radices {
    int n;
    int r[24];
};

constexpr bool has_dft(int r, int rmax) {
    return r <= rmax && (r == 2 || r == 3 || r == 4 || r == 6 || r == 8 || r == 9 || r == 12 || r == 16 ||
                         r == 18 || r == 24 || r == 27 || r == 32);
}

// Smallest possible largest factor when N splits into exactly `s` radices,
// each at most rmax with a DFT above (0: impossible).
constexpr int best_max(int N, int s, int rmax) {
    if (s == 1) return has_dft(N, rmax) ? N : 0;
    int best = 0;
    for (int r = 2; r <= rmax; ++r) {
        if (N % r || !has_dft(r, rmax)) continue;
        const int m = best_max(N / r, s - 1, rmax);
        if (!m) continue;
        const int worst = m > r ? m : r;
        if (!best || worst < best) best = worst;
    }
    return best;
}

// Radix schedules: plan 0 allows radices up to 32 (fewest stages, most
// registers), plan 1 up to 16, plan 2 up to 8.
constexpr int plan_rmax(int plan) { return plan == 0 ? 32 : (plan == 1 ? 16 : 8); }
constexpr int kTwPlans = 3;   // radix plans 0, 1, 2

// Stage radices of a length N = 2^a 3^b: the fewest stages allowed by the
// plan's largest radix, then the most even split; ascending order.
constexpr Radices make_radices(int N, int plan = 0) {
    Radices R{0, {}};
    if (N <= 1) return R;
    const int rmax = plan_rmax(plan);   // every 2^a 3^b splits into radices 2 and 3
    int s = 1;
    while (!best_max(N, s, rmax)) ++s;
    int m = N;
    for (int left = s; left > 1; --left) {
        const int cap = best_max(m, left, rmax);
        int pick = 0;   // smallest radix that keeps the remaining split within cap
        for (int r = 2; r <= cap && !pick; ++r)
            if (m % r == 0 && has_dft(r, rmax) && best_max(m / r, left - 1, rmax) &&
                best_max(m / r, left - 1, rmax) <= cap)
                pick = r;
        R.r[R.n++] = pick;
        m /= pick;
    }
    R.r[R.n++] = m;
    return R;
}

constexpr int max_radix(const Radices& R) {
    int m = 1;
    for (int i = 0; i < R.n; ++i) m = R.r[i] > m ? R.r[i] : m;
    return m;
}

constexpr int stage_ns(const Radices& R, int s) {
    int p = 1;
    for (int i = 0; i < s; ++i) p *= R.r[i];
    return p;
}

// Stage twiddle table of a radix plan: for every stage s >= 1 (radix R,
// sub-length Ns) a block of (R - 1) * Ns entries, entry (r - 1) * Ns + k
// holding W_{Ns*R}^{k*r}, blocks in stage order.  Lanes that take
// consecutive butterflies (consecutive k) read consecutive entries.  The
// blocks fill N - R_0 < N entries; tables are allotted N.
constexpr int stage_tw_offset(const Radices& R, int s) {
    int off = 0;
    for (int i = 1; i < s; ++i) off += (R.r[i] - 1) * stage_ns(R, i);
    return off;
}

// --------------------------------------------------------- storage types ---
// All pass data lives in device (global) memory; the explicit address space
// keeps accesses as global loads/stores even in code that is not inlined into
// a kernel, where pointers would otherwise be generic (flat).
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <class T> using gptr = __attribute__((address_space(1))) T*;
template <class T> using gcptr = const __attribute__((address_space(1))) T*;
template <class T> __device__ __forceinline__ gcptr<T> gload_ptr(const void* p) { return (gcptr<T>)p; }
template <class T> __device__ __forceinline__ gptr<T> gstore_ptr(void* p) { return (gptr<T>)p; }
// base + 32-bit byte offset: a wave-uniform base stays in scalar registers and
// the access takes the (scalar base, vector offset) form
template <class T> __device__ __forceinline__ gcptr<T> gload_at(const char* base, uint32_t off) {
    return (gcptr<T>)(base + off);
}
template <class T> __device__ __forceinline__ gptr<T> gstore_at(char* base, uint32_t off) {
    return (gptr<T>)(base + off);
}


struct IoC64 {   // complex64: FP32 re, FP32 im
    using value_type = float2;
    static constexpr bool scale_at_load = false;
    static constexpr int bytes = 8;
    static __device__ __forceinline__ float2 load(const void* p, int64_t i) {
        const f32x2 v = gload_ptr<f32x2>(p)[i];
        return make_float2(v.x, v.y);
    }
    static __device__ __forceinline__ void store(void* p, int64_t i, float2 v) {
        f32x2 w;
        w.x = v.x;
        w.y = v.y;
        gstore_ptr<f32x2>(p)[i] = w;
    }
    // streaming variants: data touched once per pass, no reuse in cache
    static __device__ __forceinline__ float2 load_nt(const void* p, int64_t i) {
        const f32x2 v = __builtin_nontemporal_load(gload_ptr<f32x2>(p) + i);
        return make_float2(v.x, v.y);
    }
    // elements i and i+1 in one access (i even, 16-byte aligned)
    static __device__ __forceinline__ void load2_nt(const void* p, int64_t i, float2& a, float2& b) {
        const f32x4 v = __builtin_nontemporal_load(gload_ptr<f32x4>(p) + i / 2);
        a = make_float2(v.x, v.y);
        b = make_float2(v.z, v.w);
    }
    static __device__ __forceinline__ void store2_nt(void* p, int64_t i, float2 a, float2 b) {
        f32x4 w;
        w.x = a.x; w.y = a.y; w.z = b.x; w.w = b.y;
        __builtin_nontemporal_store(w, gstore_ptr<f32x4>(p) + i / 2);
    }
    static __device__ __forceinline__ void store_nt(void* p, int64_t i, float2 v) {
        f32x2 w;
        w.x = v.x;
        w.y = v.y;
        __builtin_nontemporal_store(w, gstore_ptr<f32x2>(p) + i);
    }
    // byte-addressed forms (base + off), one and two elements
    template <bool NT> static __device__ __forceinline__ float2 ld(const char* b, uint32_t off) {
        const f32x2 v = NT ? __builtin_nontemporal_load(gload_at<f32x2>(b, off)) : *gload_at<f32x2>(b, off);
        return make_float2(v.x, v.y);
    }
    template <bool NT> static __device__ __forceinline__ void st(char* b, uint32_t off, float2 v) {
        f32x2 w;
        w.x = v.x;
        w.y = v.y;
        if (NT) __builtin_nontemporal_store(w, gstore_at<f32x2>(b, off));
        else *gstore_at<f32x2>(b, off) = w;
    }
    static __device__ __forceinline__ void ld2_nt(const char* b, uint32_t off, float2& x, float2& y) {
        const f32x4 v = __builtin_nontemporal_load(gload_at<f32x4>(b, off));
        x = make_float2(v.x, v.y);
        y = make_float2(v.z, v.w);
    }
    static __device__ __forceinline__ void st2_nt(char* b, uint32_t off, float2 x, float2 y) {
        f32x4 w;
        w.x = x.x; w.y = x.y; w.z = y.x; w.w = y.y;
        __builtin_nontemporal_store(w, gstore_at<f32x4>(b, off));
    }
};

struct IoF16 {   // FP16 re, FP16 im
    using value_type = float2;
    static constexpr bool scale_at_load = false;
    static constexpr int bytes = 4;
    static __device__ __forceinline__ float2 load(const void* p, int64_t i) {
        const uint32_t w = gload_ptr<uint32_t>(p)[i];
        return __half22float2(__builtin_bit_cast(__half2, w));
    }
    static __device__ __forceinline__ void store(void* p, int64_t i, float2 v) {
        gstore_ptr<uint32_t>(p)[i] = __builtin_bit_cast(uint32_t, __float22half2_rn(v));
    }
    static __device__ __forceinline__ float2 load_nt(const void* p, int64_t i) {
        const uint32_t w = __builtin_nontemporal_load(gload_ptr<uint32_t>(p) + i);
        return __half22float2(__builtin_bit_cast(__half2, w));
    }
    static __device__ __forceinline__ void store_nt(void* p, int64_t i, float2 v) {
        __builtin_nontemporal_store(__builtin_bit_cast(uint32_t, __float22half2_rn(v)),
                                    gstore_ptr<uint32_t>(p) + i);
    }
    // pairs move as one 64-bit scalar access
    static __device__ __forceinline__ void load2_nt(const void* p, int64_t i, float2& a, float2& b) {
        const uint64_t w = __builtin_nontemporal_load(gload_ptr<uint64_t>(p) + i / 2);
        a = __half22float2(__builtin_bit_cast(__half2, (uint32_t)w));
        b = __half22float2(__builtin_bit_cast(__half2, (uint32_t)(w >> 32)));
    }
    static __device__ __forceinline__ void store2_nt(void* p, int64_t i, float2 a, float2 b) {
        const uint64_t w = (uint64_t)__builtin_bit_cast(uint32_t, __float22half2_rn(a)) |
                           ((uint64_t)__builtin_bit_cast(uint32_t, __float22half2_rn(b)) << 32);
        __builtin_nontemporal_store(w, gstore_ptr<uint64_t>(p) + i / 2);
    }
    static __device__ __forceinline__ float2 unpack(uint32_t w) { return __half22float2(__builtin_bit_cast(__half2, w)); }
    static __device__ __forceinline__ uint32_t pack(float2 v) { return __builtin_bit_cast(uint32_t, __float22half2_rn(v)); }
    template <bool NT> static __device__ __forceinline__ float2 ld(const char* b, uint32_t off) {
        return unpack(NT ? __builtin_nontemporal_load(gload_at<uint32_t>(b, off)) : *gload_at<uint32_t>(b, off));
    }
    template <bool NT> static __device__ __forceinline__ void st(char* b, uint32_t off, float2 v) {
        if (NT) __builtin_nontemporal_store(pack(v), gstore_at<uint32_t>(b, off));
        else *gstore_at<uint32_t>(b, off) = pack(v);
    }
    static __device__ __forceinline__ void ld2_nt(const char* b, uint32_t off, float2& x, float2& y) {
        const uint64_t w = __builtin_nontemporal_load(gload_at<uint64_t>(b, off));
        x = unpack((uint32_t)w);
        y = unpack((uint32_t)(w >> 32));
    }
    static __device__ __forceinline__ void st2_nt(char* b, uint32_t off, float2 x, float2 y) {
        __builtin_nontemporal_store((uint64_t)pack(x) | ((uint64_t)pack(y) << 32), gstore_at<uint64_t>(b, off));
    }
};

// FP16 storage with FP16 arithmetic: values stay packed FP16 pairs in
// registers and LDS (4 bytes per element), so a tile holds half the state of
// the FP32-arithmetic types; loads and stores need no conversion.
struct IoF16M {
    using value_type = h16x2;
    static constexpr bool scale_at_load = true;
    static constexpr int bytes = 4;
    static __device__ __forceinline__ h16x2 load(const void* p, int64_t i) {
        return __builtin_bit_cast(h16x2, gload_ptr<uint32_t>(p)[i]);
    }
    static __device__ __forceinline__ void store(void* p, int64_t i, h16x2 v) {
        gstore_ptr<uint32_t>(p)[i] = __builtin_bit_cast(uint32_t, v);
    }
    static __device__ __forceinline__ h16x2 load_nt(const void* p, int64_t i) {
        return __builtin_bit_cast(h16x2, __builtin_nontemporal_load(gload_ptr<uint32_t>(p) + i));
    }
    static __device__ __forceinline__ void store_nt(void* p, int64_t i, h16x2 v) {
        __builtin_nontemporal_store(__builtin_bit_cast(uint32_t, v), gstore_ptr<uint32_t>(p) + i);
    }
    static __device__ __forceinline__ void load2_nt(const void* p, int64_t i, h16x2& a, h16x2& b) {
        const uint64_t w = __builtin_nontemporal_load(gload_ptr<uint64_t>(p) + i / 2);
        a = __builtin_bit_cast(h16x2, (uint32_t)w);
        b = __builtin_bit_cast(h16x2, (uint32_t)(w >> 32));
    }
    static __device__ __forceinline__ void store2_nt(void* p, int64_t i, h16x2 a, h16x2 b) {
        const uint64_t w = (uint64_t)__builtin_bit_cast(uint32_t, a) | ((uint64_t)__builtin_bit_cast(uint32_t, b) << 32);
        __builtin_nontemporal_store(w, gstore_ptr<uint64_t>(p) + i / 2);
    }
    template <bool NT> static __device__ __forceinline__ h16x2 ld(const char* b, uint32_t off) {
        return __builtin_bit_cast(h16x2, NT ? __builtin_nontemporal_load(gload_at<uint32_t>(b, off))
                                            : *gload_at<uint32_t>(b, off));
    }
    template <bool NT> static __device__ __forceinline__ void st(char* b, uint32_t off, h16x2 v) {
        const uint32_t w = __builtin_bit_cast(uint32_t, v);
        if (NT) __builtin_nontemporal_store(w, gstore_at<uint32_t>(b, off));
        else *gstore_at<uint32_t>(b, off) = w;
    }
    static __device__ __forceinline__ void ld2_nt(const char* b, uint32_t off, h16x2& x, h16x2& y) {
        const uint64_t w = __builtin_nontemporal_load(gload_at<uint64_t>(b, off));
        x = __builtin_bit_cast(h16x2, (uint32_t)w);
        y = __builtin_bit_cast(h16x2, (uint32_t)(w >> 32));
    }
    static __device__ __forceinline__ void st2_nt(char* b, uint32_t off, h16x2 x, h16x2 y) {
        __builtin_nontemporal_store((uint64_t)__builtin_bit_cast(uint32_t, x) | ((uint64_t)__builtin_bit_cast(uint32_t, y) << 32),
                                    gstore_at<uint64_t>(b, off));
    }
};

// BF16 = top 16 bits of an FP32; storage rounds to nearest even, both
// components in one conversion (v_cvt_pk_bf16_f32 on gfx950).
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t f32x2_to_bf16x2_rne(float re, float im) {
    f32x2 v;
    v.x = re;
    v.y = im;
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

struct IoBF16 {  // BF16 re (low half), BF16 im (high half)
    using value_type = float2;
    static constexpr bool scale_at_load = false;
    static constexpr int bytes = 4;
    static __device__ __forceinline__ float2 load(const void* p, int64_t i) {
        const uint32_t w = gload_ptr<uint32_t>(p)[i];
        return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
    }
    static __device__ __forceinline__ void store(void* p, int64_t i, float2 v) {
        gstore_ptr<uint32_t>(p)[i] = f32x2_to_bf16x2_rne(v.x, v.y);
    }
    static __device__ __forceinline__ float2 load_nt(const void* p, int64_t i) {
        const uint32_t w = __builtin_nontemporal_load(gload_ptr<uint32_t>(p) + i);
        return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
    }
    static __device__ __forceinline__ void store_nt(void* p, int64_t i, float2 v) {
        __builtin_nontemporal_store(f32x2_to_bf16x2_rne(v.x, v.y), gstore_ptr<uint32_t>(p) + i);
    }
    static __device__ __forceinline__ void load2_nt(const void* p, int64_t i, float2& a, float2& b) {
        const uint64_t w = __builtin_nontemporal_load(gload_ptr<uint64_t>(p) + i / 2);
        const uint32_t lo = (uint32_t)w, hi = (uint32_t)(w >> 32);
        a = make_float2(__uint_as_float(lo << 16), __uint_as_float(lo & 0xffff0000u));
        b = make_float2(__uint_as_float(hi << 16), __uint_as_float(hi & 0xffff0000u));
    }
    static __device__ __forceinline__ void store2_nt(void* p, int64_t i, float2 a, float2 b) {
        const uint64_t w = (uint64_t)f32x2_to_bf16x2_rne(a.x, a.y) | ((uint64_t)f32x2_to_bf16x2_rne(b.x, b.y) << 32);
        __builtin_nontemporal_store(w, gstore_ptr<uint64_t>(p) + i / 2);
    }
    static __device__ __forceinline__ float2 unpack(uint32_t w) {
        return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
    }
    static __device__ __forceinline__ uint32_t pack(float2 v) { return f32x2_to_bf16x2_rne(v.x, v.y); }
    template <bool NT> static __device__ __forceinline__ float2 ld(const char* b, uint32_t off) {
        return unpack(NT ? __builtin_nontemporal_load(gload_at<uint32_t>(b, off)) : *gload_at<uint32_t>(b, off));
    }
    template <bool NT> static __device__ __forceinline__ void st(char* b, uint32_t off, float2 v) {
        if (NT) __builtin_nontemporal_store(pack(v), gstore_at<uint32_t>(b, off));
        else *gstore_at<uint32_t>(b, off) = pack(v);
    }
    static __device__ __forceinline__ void ld2_nt(const char* b, uint32_t off, float2& x, float2& y) {
        const uint64_t w = __builtin_nontemporal_load(gload_at<uint64_t>(b, off));
        x = unpack((uint32_t)w);
        y = unpack((uint32_t)(w >> 32));
    }
    static __device__ __forceinline__ void st2_nt(char* b, uint32_t off, float2 x, float2 y) {
        __builtin_nontemporal_store((uint64_t)pack(x) | ((uint64_t)pack(y) << 32), gstore_at<uint64_t>(b, off));
    }
};

// Kernel feature flags (template parameter FLAGS).
enum : int {
    kFlagNontemporal = 1,   // streaming (non-temporal) global loads and stores
    kFlagFourStep = 8,      // first pass of a split axis: inter-pass twiddles
                            // and the transposed store (PassArgs tw4_mode,
                            // tstore) are compiled in only with this flag
    kFlagPairs = 16,        // contiguous layout: thread j owns butterflies
                            // j*NB .. j*NB+NB-1 of every stage, so its first
                            // loads and last stores come in adjacent pairs that
                            // move as one wider access
    // Fused Poisson solve (complex64 storage only):
    kFlagRealIn = 32,       // contiguous layout: the input is real FP32 (imaginary part 0)
    kFlagPoisson = 64,      // strided layout, z pass of an (nx, ny, N) grid: every stored
                            // element is multiplied by -1/|k|^2 of its frequency (0 at k = 0)
    kFlagRealOut = 128,     // strided layout: only the real part is stored, as FP32
    // Real input and output (complex64 storage; the half spectrum of a real
    // array of 2N points along x is the N + 1 bins kx = 0 .. N):
    kFlagR2C = 256,         // contiguous layout: pencil q holds 2N reals read as N complex
                            // z[m] = a[2m] + i a[2m+1]; after the N-point FFT an epilogue
                            // through LDS stores the N + 1 half-spectrum bins at q*os1_out
    kFlagC2R = 512,         // contiguous layout: a prologue through LDS turns the N + 1 bins at
                            // q*os1_in into the N-point spectrum whose inverse FFT is the 2N
                            // reals as N complex pairs, stored at q*os1_out
    kFlagSolveZ = 1024,     // strided layout, z pass of a Poisson solve: forward FFT, times
                            // -1/|k|^2, inverse FFT (opposite sign) of each pencil in one tile
    kFlagTemporalStore = 2048,  // with kFlagNontemporal: streaming loads but ordinary (cached)
                                // stores, so partial lines written by neighbouring accesses merge
                                // in the cache before they reach memory
};

// -------------------------------------------------------------- pass args ---
// A pass transforms pencils of length N.  Two layouts:
//   contiguous: pencil q in [0, C) has element e at q*os1_in + e (stride 1)
//   strided:    pencil (c, o1, o2), c in [0, C) a unit-stride column index,
//               element e at c + e*es_in + o1*os1_in + o2*os2_in
// Outputs go to c*cs_out + e*es_out + o1*os1_out + o2*os2_out (strided) or
// q*os1_out + e (contiguous).  The second set of strides lets the first pass
// of a two-pass (four-step) axis write its results transposed.
struct PassArgs {
    const void* src;
    void* dst;
    const float2* tw;     // stage twiddles of the kernel's radix plan (stage_tw_offset), N entries
    const float2* tw4;    // four-step twiddles (M entries, see tw4_mode), or null
    int64_t M;            // full axis length for tw4
    int64_t C, O1, O2;
    int64_t es_in, os1_in, os2_in;
    int64_t es_out, cs_out, os1_out, os2_out;
    int32_t tw4_mode;     // 0: none; 1: output e of column c times W_M^(c*e), table entry c*N + e;
                          // 2: times W_M^(o1*e), table entry o1*e
    int32_t tstore;       // strided layout only: store columns as contiguous runs via LDS
    int32_t tw4_shift;    // complex64 mode 1 with tstore: tw4 holds two FP64 tables instead,
                          // W_M^j for j < 2^tw4_shift, then W_M^(j * 2^tw4_shift)
    float scale;          // multiplies every stored value
    int32_t sym_nx;       // kFlagPoisson / kFlagSolveZ: column c of the z pass is
    int32_t sym_ny;       //   (x, y) = (c mod sym_nx, c div sym_nx)
    int32_t sym_half;     //   nonzero: the columns are a half spectrum, kx = x (else the wavenumber of x)
    int32_t xcd_order;    // nonzero: each XCD takes a contiguous range of tiles (see xcd_tile)
    // strided layout: nonzero flattens the columns over (column, o1) pairs:
    // C counts flat_c * (the original O1) columns, column i is original column
    // i mod flat_c of outer index i div flat_c (O1 = 1), so tiles run on across
    // the outer index instead of leaving a ragged tile at each one (cs_out = 1)
    int64_t flat_c;
};

// One array of a merged batch launch: the fields of a direct pass that differ
// between arrays sharing one kernel.  Tiles [previous tile_end, tile_end) of
// the launch belong to this array.
struct ArrayDesc {
    const void* src;
    void* dst;
    int64_t C, O1, es, os1;
    int64_t tile_end;
    float scale;
    int32_t pad;
};
constexpr int kMaxBatchDescs = 40;
struct BatchTable {
    int32_t count;      // 0: a single-array launch described by PassArgs alone
    int32_t pad;
    ArrayDesc d[kMaxBatchDescs];
};

// Workgroups are dispatched to the 8 XCDs of the chip in turn (workgroup b
// to XCD b mod 8), and each XCD has its own L2.  This maps workgroup b to a
// tile so that XCD x works through the contiguous range of tiles
// [x*q + min(x, r), ...) (q = blocks / 8, r = blocks mod 8), in order: tiles
// that share cache lines (neighbouring columns of rows that are not
// line-aligned) then meet in one L2.  A bijection on [0, blocks).
constexpr unsigned kXcds = 8;
__device__ __forceinline__ int64_t xcd_tile(unsigned b, unsigned blocks) {
    const unsigned x = b % kXcds, i = b / kXcds, q = blocks / kXcds, r = blocks % kXcds;
    return (int64_t)x * q + (x < r ? x : r) + i;
}

// Per-thread context of one tile.  Besides the element indices, the split
// form of the addresses: element e of this thread's pencil or column is at
// ib + (e - le_in) * ies + il (bytes), where ib and ies are the same for the
// whole wave and il is a 32-bit per-lane offset; le_in is the part of e that
// varies across the wave's lanes (j, or j * NB for paired slots).  Likewise
// ob, oes, ol for the stored elements.  Lanes of a ragged tile past the last
// pencil or column load the tile's first one instead (it always exists;
// pencils are independent and such lanes never store), so split loads need
// no per-element predicate.  split is false when a lane offset could exceed
// 32 bits (strides of several GiB); the 64-bit element-index form is used
// then.
struct PassCtx {
    int p, j;
    bool valid;
    bool split;
    int64_t col;          // global column (strided) or pencil (contiguous)
    int64_t o1;
    int64_t base_in, base_out;
    const char* ib;
    char* ob;
    int64_t ies, oes;
    uint32_t il, ol;
};

// ------------------------------------------------------------ the kernel ---
// N: pencil length.  T: threads per pencil.  P: pencils (contiguous layout)
// or columns (strided layout) per workgroup.  K: the LDS
// exchanges run in K rounds over N/K elements of each pencil (rows of a
// strided tile), so a wide tile or a long pencil needs only
// 1/K of its size in LDS and more workgroups stay resident per CU.
template <int N, int T, int P, bool STRIDED, class IO, int SIGN, int FLAGS = 0, int K = 1, int PLAN = 0>
struct PencilPass {
    // register and LDS value of one complex element: FP32 pairs, or packed
    // FP16 pairs for the FP16-arithmetic storage type
    using V = typename IO::value_type;
    // FP16 arithmetic applies the pass scale to the loaded values, so
    // intermediate sums stay within the FP16 range
    static constexpr bool SCALE_IN = IO::scale_at_load;
    static_assert(N % K == 0, "K must divide N");
    static constexpr bool NT = (FLAGS & kFlagNontemporal) != 0;
    static constexpr bool NTS = NT && (FLAGS & kFlagTemporalStore) == 0;   // streaming stores
    static constexpr bool FOURSTEP = (FLAGS & kFlagFourStep) != 0;
    static constexpr bool REALIN = (FLAGS & kFlagRealIn) != 0;
    static constexpr bool REALOUT = (FLAGS & kFlagRealOut) != 0;
    static constexpr bool POISSON = (FLAGS & kFlagPoisson) != 0;
    static constexpr bool R2C = (FLAGS & kFlagR2C) != 0;
    static constexpr bool C2R = (FLAGS & kFlagC2R) != 0;
    static constexpr bool SOLVEZ = (FLAGS & kFlagSolveZ) != 0;
    static_assert(!REALIN || !STRIDED, "real input is read by contiguous passes");
    static_assert(!(REALOUT || POISSON) || (STRIDED && !FOURSTEP), "fused outputs are strided direct passes");
    static_assert(!(R2C || C2R) || (!STRIDED && !FOURSTEP && !REALIN && sizeof(V) == 8),
                  "real-data passes: contiguous pencils with FP32 values");
    static_assert(!SOLVEZ || (STRIDED && !FOURSTEP && !POISSON && !REALOUT && sizeof(V) == 8),
                  "the fused solve is a strided complex64 direct pass");
    static constexpr int64_t BI = REALIN ? 4 : IO::bytes;    // bytes per input element
    static constexpr int64_t BO = REALOUT ? 4 : IO::bytes;   // bytes per output element
    __device__ __forceinline__ static V gload(const void* p, int64_t i) {
        if constexpr (NT) return IO::load_nt(p, i);
        else return IO::load(p, i);
    }
    __device__ __forceinline__ static void gstore(void* p, int64_t i, V v) {
        if constexpr (NTS) IO::store_nt(p, i, v);
        else IO::store(p, i, v);
    }
    // first-pass input and last-pass output, real where the fused flags say so
    __device__ __forceinline__ static V gload_in(const void* p, int64_t i) {
        if constexpr (REALIN) return make_float2(__builtin_nontemporal_load(gload_ptr<float>(p) + i), 0.f);
        else return gload(p, i);
    }
    __device__ __forceinline__ static void gstore_out(void* p, int64_t i, V v) {
        if constexpr (REALOUT) __builtin_nontemporal_store(v.x, gstore_ptr<float>(p) + i);
        else gstore(p, i, v);
    }
    __device__ __forceinline__ static V ld_in(const char* b, uint32_t off) {
        if constexpr (REALIN) return make_float2(__builtin_nontemporal_load(gload_at<float>(b, off)), 0.f);
        else return IO::template ld<NT>(b, off);
    }
    __device__ __forceinline__ static void st_out(char* b, uint32_t off, V v) {
        if constexpr (REALOUT) __builtin_nontemporal_store(v.x, gstore_at<float>(b, off));
        else IO::template st<NTS>(b, off, v);
    }
    static constexpr Radices RD = make_radices(N, PLAN);
    static constexpr int NS = RD.n;
    static constexpr int ROWS = N / K;   // LDS rows per exchange round
    // LDS layout: strided tiles store [element][column] with one V of
    // padding per row; contiguous tiles store [pencil][element] with one
    // V of padding after every 2^PADSH elements, which spreads the
    // radix-stride writes of the first stages over all banks.
    static constexpr bool PAIRS = !STRIDED && (FLAGS & kFlagPairs) != 0;
    // first-stage writes land R0 (times the slots per thread, when paired)
    // elements apart: pad once per that many elements
    static constexpr int pad_shift() {
        int r = RD.r[0] * (PAIRS ? ((N / RD.r[0] + T - 1) / T) : 1), sh = 0;
        while (r % 2 == 0) { r /= 2; ++sh; }
        return sh < 3 ? 3 : (sh > 6 ? 6 : sh);
    }
    static constexpr int PADSH = pad_shift();
    static constexpr int LDS_ROW = STRIDED ? (P + 1) : (ROWS + (ROWS >> PADSH) + 1);
    static constexpr int LDS_ELEMS = STRIDED ? ROWS * (P + 1) : P * LDS_ROW;
    static constexpr int lds_bytes() { return LDS_ELEMS * (int)sizeof(V); }
    static constexpr int threads() { return T * P; }

    template <int S> struct St {
        static constexpr int R = RD.r[S];
        static constexpr int Ns = stage_ns(RD, S);
        static constexpr int NBF = N / R;               // butterflies
        static constexpr int NB = (NBF + T - 1) / T;    // per thread
        static constexpr int TWS = N / (Ns * R);        // twiddle table stride
        static constexpr bool FULL = NB * T == NBF;     // every thread busy
        // butterfly of thread j's slot t
        static constexpr __host__ __device__ int bf(int j, int t) { return PAIRS ? j * NB + t : j + t * T; }
    };

    static constexpr int maxv() {
        int m = 1;
        for (int s = 0; s < NS; ++s) {
            const int R = RD.r[s];
            const int nb = (N / R + T - 1) / T;
            m = nb * R > m ? nb * R : m;
        }
        return m;
    }

    __device__ __forceinline__ static int lidx(int p, int e) {
        return STRIDED ? e * LDS_ROW + p : p * LDS_ROW + e + (e >> PADSH);
    }

    // Exchange round of the value in slot (t, r) when written after stage SO
    // (W) or read before stage SI (R; SI = SO + 1, or 0 when a second
    // transform of the same pencils follows): the round if it is the same
    // for every thread j, else -1 (decided at run time).  Tables are built at
    // compile time, so after unrolling each access is either kept in exactly
    // one round or decided by one compare.
    template <int SO, int SI = SO + 1> struct Rounds {
        int w[St<SO>::NB][St<SO>::R];
        int r[St<SI>::NB][St<SI>::R];
        constexpr Rounds() : w(), r() {
            using Q = St<SO>;
            using Q2 = St<SI>;
            for (int t = 0; t < Q::NB; ++t)
                for (int rr = 0; rr < Q::R; ++rr) {
                    int h = -2;
                    for (int j = 0; j < T; ++j) {
                        const int b = Q::bf(j, t);
                        if (!Q::FULL && b >= Q::NBF) continue;
                        const int e = (b / Q::Ns) * Q::Ns * Q::R + b % Q::Ns + rr * Q::Ns;
                        const int hh = e / ROWS;
                        h = (h == -2 || h == hh) ? hh : -1;
                    }
                    w[t][rr] = h;
                }
            for (int t = 0; t < Q2::NB; ++t)
                for (int rr = 0; rr < Q2::R; ++rr) {
                    int h = -2;
                    for (int j = 0; j < T; ++j) {
                        const int b = Q2::bf(j, t);
                        if (!Q2::FULL && b >= Q2::NBF) continue;
                        const int hh = (b + rr * Q2::NBF) / ROWS;
                        h = (h == -2 || h == hh) ? hh : -1;
                    }
                    r[t][rr] = h;
                }
        }
    };

    using Ctx = PassCtx;

    // Twiddle table entry (global memory, 32-bit offset).
    __device__ __forceinline__ static V tw_at(const float2* tw, int i) {
        return cvt_value<V>(*gload_at<f32x2>(reinterpret_cast<const char*>(tw), (uint32_t)i * 8u));
    }
    // The stored value: the pass scale, unless it was applied at the load.
    __device__ __forceinline__ static V oscale(V v, const PassArgs& a) {
        if constexpr (SCALE_IN) return v;
        else return cscale(v, a.scale);
    }

    template <int S>
    __device__ __forceinline__ static void butterflies(V* v, int j, const float2* tw) {
        using Q = St<S>;
#pragma unroll
        for (int t = 0; t < Q::NB; ++t) {
            const int b = Q::bf(j, t);
            if (!Q::FULL && b >= Q::NBF) continue;
            V* u = v + t * Q::R;
            if (S > 0) {
                const int k = b % Q::Ns;
                constexpr int off = stage_tw_offset(RD, S);
#pragma unroll
                for (int r = 1; r < Q::R; ++r) {
                    V w = tw_at(tw, off + (r - 1) * Q::Ns + k);
                    if (SIGN > 0) w.y = -w.y;
                    u[r] = cmul(u[r], w);
                }
            }
            Dft<Q::R, SIGN>::run(u);
        }
    }

    // Stage S outputs (vo) -> stage SI inputs (vi, by default stage S+1)
    // through LDS, in K rounds of ROWS rows.  lead: the LDS may still be read
    // by the previous exchange.
    template <int S, int SI = S + 1>
    __device__ __forceinline__ static void exchange(V* lds, const V* vo, V* vi, int p, int j,
                                                    bool lead) {
        using Q = St<S>;
        using Q2 = St<SI>;
        constexpr Rounds<S, SI> RT{};
#pragma unroll
        for (int h = 0; h < K; ++h) {
            if (lead || h > 0) __syncthreads();
#pragma unroll
            for (int t = 0; t < Q::NB; ++t) {
                const int b = Q::bf(j, t);
                if (!Q::FULL && b >= Q::NBF) continue;
                const int o = (b / Q::Ns) * Q::Ns * Q::R + b % Q::Ns;
#pragma unroll
                for (int r = 0; r < Q::R; ++r) {
                    const int e = o + r * Q::Ns;
                    const int hs = RT.w[t][r];
                    if (K == 1 || hs == h || (hs < 0 && e / ROWS == h))
                        lds[lidx(p, e - h * ROWS)] = vo[t * Q::R + r];
                }
            }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < Q2::NB; ++t) {
                const int b = Q2::bf(j, t);
                if (!Q2::FULL && b >= Q2::NBF) continue;
#pragma unroll
                for (int r = 0; r < Q2::R; ++r) {
                    const int e = b + r * Q2::NBF;
                    const int hs = RT.r[t][r];
                    if (K == 1 || hs == h || (hs < 0 && e / ROWS == h))
                        vi[t * Q2::R + r] = lds[lidx(p, e - h * ROWS)];
                }
            }
        }
    }

    // Four-step twiddle W_M^{g*e} of output element e (tw4_mode != 0); g < M/N
    // and e < N, so g*e < M.  Mode 1 (g = column) reads the table laid out by
    // output position, entry g*N + e, so lanes with consecutive e read
    // consecutive entries; mode 2 (g = o1, the same for the whole tile) reads
    // the plain table W_M^m at m = g*e.
    // Complex64 pass A of a unit-stride split axis (tw4_mode 1) takes its
    // twiddles from two small FP64 tables instead of one entry per output:
    // W_M^m = W_M^(m mod 2^s) * W_M^(2^s * (m div 2^s)), rounded once to FP32.
    // With the transposed store each thread keeps one element over columns D
    // apart (TW_RECUR), so the products run as an FP64 recurrence.
    static constexpr bool TW64 = FOURSTEP && STRIDED && std::is_same<IO, IoC64>::value;
    static constexpr bool TW_RECUR = TW64 && (T * P) % ROWS == 0;
    // W_M^m (m < M) from the two FP64 tables at a.tw4 (tw4_shift)
    __device__ __forceinline__ static double2 root64(const PassArgs& a, uint32_t m) {
        const double2* lo = reinterpret_cast<const double2*>(a.tw4);
        const double2 p = lo[m & ((1u << a.tw4_shift) - 1u)];
        const double2 q = lo[(1u << a.tw4_shift) + (m >> a.tw4_shift)];
        return make_double2(p.x * q.x - p.y * q.y, p.x * q.y + p.y * q.x);
    }
    // W_M^m with the pass's sign, rounded once to FP32 (complex64 only)
    __device__ __forceinline__ static V tw64_of(const PassArgs& a, uint32_t m) {
        if constexpr (TW64) {
            const double2 w = root64(a, m);
            return make_float2((float)w.x, SIGN > 0 ? -(float)w.y : (float)w.y);
        } else {
            return cconst<V>(1.0, 0.0);   // never called: only complex64 passes hold FP64 tables
        }
    }
    __device__ __forceinline__ static V tw4_of(int e, int64_t col, int64_t o1, const PassArgs& a) {
        if constexpr (TW64) {
            if (a.tw4_mode == 1) return tw64_of(a, (uint32_t)col * (uint32_t)e);
        }
        const uint32_t m = a.tw4_mode == 1 ? (uint32_t)col * N + e : (uint32_t)o1 * e;   // < M <= 2^20
        const f32x2 wv = *gload_at<f32x2>(reinterpret_cast<const char*>(a.tw4), m * 8u);
        V w = cvt_value<V>(wv);
        if (SIGN > 0) w.y = -w.y;
        return w;
    }

    // Integer wavenumber of index i on an axis of length n: i below ceil(n/2),
    // i - n from there on (the Nyquist index of an even axis maps to -n/2).
    __device__ __forceinline__ static float wavenumber(int64_t i, int64_t n) {
        return (float)(i < (n + 1) / 2 ? i : i - n);
    }
    // kx^2 + ky^2 of this thread's column of the z pass (kFlagPoisson,
    // kFlagSolveZ); the columns of a half spectrum are kx = 0 .. nx/2.
    __device__ __forceinline__ static float kxy2_of(const Ctx& c, const PassArgs& a) {
        const int64_t x = c.col % a.sym_nx, y = c.col / a.sym_nx;
        const float kx = a.sym_half ? (float)x : wavenumber(x, a.sym_nx), ky = wavenumber(y, a.sym_ny);
        return kx * kx + ky * ky;
    }
    // A stored value: the pass scale and, for the Poisson z pass, -1/|k|^2 of
    // output element e (its kz index), 0 at k = 0.
    __device__ __forceinline__ static V finish(V v, int e, float kxy2, const PassArgs& a) {
        v = oscale(v, a);
        if constexpr (POISSON) {
            const float kz = wavenumber(e, N);
            const float k2 = kxy2 + kz * kz;
            const float m = k2 > 0.f ? -__builtin_amdgcn_rcpf(k2) : 0.f;
            v = make_float2(v.x * m, v.y * m);
        }
        return v;
    }

    // kFlagR2C epilogue.  The N-point transform Z of z[m] = a[2m] + i a[2m+1]
    // carries the transforms of the even and odd samples,
    // E = (Z[k] + conj Z[N-k]) / 2 and O = (Z[k] - conj Z[N-k]) / (2i), and
    // the 2N-point transform of a is X[k] = E + W^k O, X[N-k] = conj(E - W^k O)
    // with W = exp(SIGN 2 pi i / 2N); each thread takes pairs (k, N-k),
    // k = 0 .. N/2 (k = 0 gives bins 0 and N).  a.tw4 entry k (k <= N/2)
    // holds exp(-2 pi i k / 2N).
    template <int S>
    __device__ __forceinline__ static void store_r2c(V* lds, const V* v, const Ctx& c, const PassArgs& a) {
        using Q = St<S>;
        __syncthreads();   // the last exchange's reads are done
#pragma unroll
        for (int t = 0; t < Q::NB; ++t) {
            const int b = Q::bf(c.j, t);
            if (!Q::FULL && b >= Q::NBF) continue;
#pragma unroll
            for (int r = 0; r < Q::R; ++r) lds[lidx(c.p, b + r * Q::NBF)] = v[t * Q::R + r];
        }
        __syncthreads();
        if (!c.valid) return;
        constexpr int H = N / 2;
        constexpr int PER = (H + 1 + T - 1) / T;
        const char* twb = reinterpret_cast<const char*>(a.tw4);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int k = c.j + i * T;
            if (k > H) continue;
            const float2 zk = lds[lidx(c.p, k)];
            const float2 zm = lds[lidx(c.p, k == 0 ? 0 : N - k)];
            const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
            const float2 d = make_float2(0.5f * (zk.x - zm.x), 0.5f * (zk.y + zm.y));   // (Z[k] - conj Z[N-k]) / 2
            const float2 o = make_float2(d.y, -d.x);                                      // -i times that
            const f32x2 wv = *gload_at<f32x2>(twb, (uint32_t)k * 8u);
            float2 w = make_float2(wv.x, wv.y);
            if (SIGN > 0) w.y = -w.y;
            const float2 wo = cmul(o, w);
            gstore(a.dst, c.base_out + k, oscale(cadd(e, wo), a));
            if (k != N - k) {
                const float2 m = csub(e, wo);
                gstore(a.dst, c.base_out + (N - k), oscale(make_float2(m.x, -m.y), a));
            }
        }
    }

    // kFlagC2R prologue: the inverse of the epilogue above.  From the N + 1
    // half-spectrum bins X of a pencil, with A = X[k] and B = conj X[N-k],
    // Z[k] = (A + B) + i V^k (A - B) and Z[N-k] = conj((A + B) - i V^k (A - B)),
    // V = exp(SIGN 2 pi i / 2N), is the N-point spectrum whose transform (sign
    // SIGN, unnormalised) is z[m] = a[2m] + i a[2m+1], a the 2N-point transform
    // of the Hermitian extension of X.  Bins 0 and N contribute their real
    // parts only (a Hermitian spectrum has no imaginary part there).  Z goes
    // to LDS in natural order and the first stage reads it from there.
    __device__ __forceinline__ static void load_c2r(V* v, const Ctx& c, const PassArgs& a, V* lds) {
        constexpr int H = N / 2;
        constexpr int PER = (H + 1 + T - 1) / T;
        const char* twb = reinterpret_cast<const char*>(a.tw4);
        // lanes past the last pencil read the tile's first pencil (never stored)
        const int64_t base = c.valid ? c.base_in : (c.col - c.p) * a.os1_in;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int k = c.j + i * T;
            if (k > H) continue;
            float2 A = gload(a.src, base + k);
            float2 Bc = gload(a.src, base + (N - k));
            if (k == 0) {
                A.y = 0.f;
                Bc.y = 0.f;
            }
            const float2 B = make_float2(Bc.x, -Bc.y);
            const f32x2 wv = *gload_at<f32x2>(twb, (uint32_t)k * 8u);
            float2 w = make_float2(wv.x, wv.y);
            if (SIGN > 0) w.y = -w.y;
            const float2 t1 = cadd(A, B);
            const float2 t2 = crot90<1>(cmul(csub(A, B), w));   // i V^k (A - B)
            lds[lidx(c.p, k)] = cadd(t1, t2);
            if (k != 0 && k != N - k) {
                const float2 m = csub(t1, t2);
                lds[lidx(c.p, N - k)] = make_float2(m.x, -m.y);
            }
        }
        __syncthreads();
        using Q = St<0>;
#pragma unroll
        for (int t = 0; t < Q::NB; ++t) {
            const int b = Q::bf(c.j, t);
            if (!Q::FULL && b >= Q::NBF) continue;
#pragma unroll
            for (int r = 0; r < Q::R; ++r) v[t * Q::R + r] = lds[lidx(c.p, b + r * Q::NBF)];
        }
    }

    // kFlagSolveZ: after the forward stages, multiply every value by
    // -1/|k|^2 of its frequency (0 at k = 0), then run the stages of the
    // opposite sign on the same registers (through LDS when the last and
    // the first stage hold different elements), which end in the store.
    template <int S>
    __device__ __forceinline__ static void solve_z(V* lds, V* v, const Ctx& c, const PassArgs& a) {
        using Q = St<S>;
        const float kxy2 = kxy2_of(c, a);
#pragma unroll
        for (int t = 0; t < Q::NB; ++t) {
            const int b = Q::bf(c.j, t);
            if (!Q::FULL && b >= Q::NBF) continue;
#pragma unroll
            for (int r = 0; r < Q::R; ++r) {
                const float kz = wavenumber(b + r * Q::NBF, N);
                const float k2 = kxy2 + kz * kz;
                const float m = k2 > 0.f ? -1.0f / k2 : 0.f;
                v[t * Q::R + r] = cscale(v[t * Q::R + r], m);
            }
        }
        using Inv = PencilPass<N, T, P, STRIDED, IO, -SIGN, (FLAGS & ~kFlagSolveZ), K, PLAN>;
        if constexpr (RD.r[0] == RD.r[NS - 1]) {
            Inv::template stages<0>(lds, v, c, a, a.tw, true);
        } else {
            V w[maxv()];
            exchange<S, 0>(lds, v, w, c.p, c.j, true);
            Inv::template stages<0>(lds, w, c, a, a.tw, true);
        }
    }

    template <int S>
    __device__ __forceinline__ static void store_last(V* lds, const V* v, const Ctx& c,
                                                      const PassArgs& a) {
        using Q = St<S>;
        if constexpr (R2C) {
            store_r2c<S>(lds, v, c, a);
            return;
        }
        if (FOURSTEP && STRIDED && a.tstore) {
            // Results go to LDS in natural element order, ROWS rows per round,
            // and each column leaves as contiguous runs of ROWS elements.
            const int64_t c0 = c.col - c.p;
            const int64_t b0 = c.base_out - c.p * a.cs_out;
            // tile-uniform bases with 32-bit per-lane byte offsets: the store
            // offset pl*cs_out + e*es_out (when it fits) and the twiddle entry,
            // (c0 + pl)*N + e (mode 1) or o1*e (mode 2), both below M
            constexpr int64_t B = IO::bytes;
            char* const obase = static_cast<char*>(a.dst) + b0 * B;
            const bool fit = (P * a.cs_out + N * a.es_out) * B < (int64_t(1) << 32);
            const uint32_t cs32 = (uint32_t)(a.cs_out * B), es32 = (uint32_t)(a.es_out * B);
            const char* const twbase = reinterpret_cast<const char*>(a.tw4) + (a.tw4_mode == 1 ? c0 * N * 8 : 0);
            const uint32_t o1w = (uint32_t)c.o1;
#pragma unroll
            for (int h = 0; h < K; ++h) {
                __syncthreads();
#pragma unroll
                for (int t = 0; t < Q::NB; ++t) {
                    const int b = Q::bf(c.j, t);
                    if (!Q::FULL && b >= Q::NBF) continue;
#pragma unroll
                    for (int r = 0; r < Q::R; ++r) {
                        const int e = b + r * Q::NBF;
                        if (K == 1 || e / ROWS == h) lds[lidx(c.p, e - h * ROWS)] = v[t * Q::R + r];
                    }
                }
                // each thread stores PER elements of this round; their
                // twiddles are all requested before the first use
                constexpr int PER = (ROWS * P + T * P - 1) / (T * P);
                V w4[PER];
                bool tw_done = false;
                if constexpr (TW_RECUR) {
                    if (a.tw4_mode == 1) {
                        tw_done = true;
                        // complex64: the thread's element e is the same in all its
                        // columns, which are D apart, so W_M^((c0 + pl) * e) runs
                        // as an FP64 recurrence from W_M^((c0 + pl0) * e) with step
                        // W_M^(D * e), rounded once to FP32 per use (reading one
                        // table entry per output made such a pass 14% slower)
                        constexpr int D = T * P / ROWS;
                        const uint32_t pl0 = threadIdx.x / ROWS;
                        const uint64_t e = threadIdx.x % ROWS + (uint64_t)h * ROWS, M = (uint64_t)a.M;
                        uint64_t x0 = (uint64_t)(c0 + pl0) * e, xs = (uint64_t)D * e;
                        if (x0 >= M) x0 %= M;
                        if (xs >= M) xs %= M;
                        double2 w = root64(a, (uint32_t)x0);
                        const double2 st = root64(a, (uint32_t)xs);
#pragma unroll
                        for (int i = 0; i < PER; ++i) {
                            const int pl = (int)pl0 + i * D;
                            if (pl < P && c0 + pl < a.C) {
                                w4[i] = make_float2((float)w.x, SIGN > 0 ? -(float)w.y : (float)w.y);
                            } else {
                                w4[i] = cconst<V>(1.0, 0.0);
                            }
                            w = make_double2(w.x * st.x - w.y * st.y, w.x * st.y + w.y * st.x);
                        }
                    }
                }
                if (!tw_done && FOURSTEP && a.tw4_mode != 0) {
#pragma unroll
                    for (int i = 0; i < PER; ++i) {
                        const int idx = threadIdx.x + i * T * P;
                        const int pl = idx / ROWS, el = idx % ROWS;
                        const uint32_t e = (uint32_t)(el + h * ROWS);
                        const uint32_t m = a.tw4_mode == 1 ? (uint32_t)pl * N + e : o1w * e;
                        if (TW64 && a.tw4_mode == 1 && idx < ROWS * P && c0 + pl < a.C) {
                            w4[i] = tw64_of(a, (uint32_t)(c0 + pl) * e);
                        } else if (idx < ROWS * P && c0 + pl < a.C) {
                            const f32x2 wv = *gload_at<f32x2>(twbase, m * 8u);
                            w4[i] = cvt_value<V>(wv);
                            if (SIGN > 0) w4[i].y = -w4[i].y;
                        } else {
                            w4[i] = cconst<V>(1.0, 0.0);
                        }
                    }
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < PER; ++i) {
                    const int idx = threadIdx.x + i * T * P;
                    if (idx >= ROWS * P) continue;
                    const int pl = idx / ROWS, el = idx % ROWS, e = el + h * ROWS;
                    const int64_t col = c0 + pl;
                    if (col >= a.C) continue;
                    V x = lds[lidx(pl, el)];
                    if (FOURSTEP && a.tw4_mode != 0) x = cmul(x, w4[i]);
                    if (fit) IO::template st<NTS>(obase, (uint32_t)pl * cs32 + (uint32_t)e * es32, oscale(x, a));
                    else gstore(a.dst, b0 + pl * a.cs_out + (int64_t)e * a.es_out, oscale(x, a));
                }
            }
            return;
        }
        if (!c.valid) return;
        const int64_t es = STRIDED ? a.es_out : 1;
        if (FOURSTEP && a.tw4_mode != 0) {
            // all twiddle requests first, then the stores
            V w4[Q::NB * Q::R];
#pragma unroll
            for (int t = 0; t < Q::NB; ++t) {
                const int b = Q::bf(c.j, t);
#pragma unroll
                for (int r = 0; r < Q::R; ++r)
                    w4[t * Q::R + r] = (Q::FULL || b < Q::NBF) ? tw4_of(b + r * Q::NBF, c.col, c.o1, a)
                                                               : cconst<V>(1.0, 0.0);
            }
#pragma unroll
            for (int t = 0; t < Q::NB; ++t) {
                const int b = Q::bf(c.j, t);
                if (!Q::FULL && b >= Q::NBF) continue;
#pragma unroll
                for (int r = 0; r < Q::R; ++r) {
                    const int e = b + r * Q::NBF;
                    gstore(a.dst, c.base_out + (int64_t)e * es,
                           oscale(cmul(v[t * Q::R + r], w4[t * Q::R + r]), a));
                }
            }
            return;
        }
        if (c.split) {
            if constexpr (pairable_store<S>()) {
                if (((reinterpret_cast<uintptr_t>(c.ob) + c.ol) & (2 * IO::bytes - 1)) == 0) {
#pragma unroll
                    for (int t = 0; t < Q::NB; t += 2)
#pragma unroll
                        for (int r = 0; r < Q::R; ++r)
                            IO::st2_nt(c.ob + (int64_t)eoff<S>(t, r) * c.oes, c.ol, oscale(v[t * Q::R + r], a),
                                       oscale(v[(t + 1) * Q::R + r], a));
                    return;
                }
            }
            const float kxy2 = POISSON ? kxy2_of(c, a) : 0.f;
#pragma unroll
            for (int t = 0; t < Q::NB; ++t) {
                const int b = Q::bf(c.j, t);
                if (!Q::FULL && b >= Q::NBF) continue;
#pragma unroll
                for (int r = 0; r < Q::R; ++r)
                    st_out(c.ob + (int64_t)eoff<S>(t, r) * c.oes, c.ol,
                           finish(v[t * Q::R + r], b + r * Q::NBF, kxy2, a));
            }
            return;
        }
        if constexpr (pairable_store<S>()) {
            if (pair_aligned(a.dst, c.base_out)) {
#pragma unroll
                for (int t = 0; t < Q::NB; t += 2) {
                    const int b = Q::bf(c.j, t);
#pragma unroll
                    for (int r = 0; r < Q::R; ++r)
                        IO::store2_nt(a.dst, c.base_out + b + r * Q::NBF, oscale(v[t * Q::R + r], a),
                                      oscale(v[(t + 1) * Q::R + r], a));
                }
                return;
            }
        }
        const float kxy2 = POISSON ? kxy2_of(c, a) : 0.f;
#pragma unroll
        for (int t = 0; t < Q::NB; ++t) {
            const int b = Q::bf(c.j, t);
            if (!Q::FULL && b >= Q::NBF) continue;
#pragma unroll
            for (int r = 0; r < Q::R; ++r) {
                const int e = b + r * Q::NBF;
                gstore_out(a.dst, c.base_out + (int64_t)e * es, finish(v[t * Q::R + r], e, kxy2, a));
            }
        }
    }

    // Stages S .. NS-1; v holds the inputs of stage S.  lead0: the LDS may
    // still be read by earlier work of the tile before the first exchange
    // (later exchanges always synchronise first).
    template <int S>
    __device__ __forceinline__ static void stages(V* lds, V* v, const Ctx& c, const PassArgs& a,
                                                  const float2* tw, bool lead0 = C2R) {
        butterflies<S>(v, c.j, tw);
        if constexpr (S + 1 < NS) {
            V w[maxv()];
            exchange<S>(lds, v, w, c.p, c.j, S > 0 || lead0);
            stages<S + 1>(lds, w, c, a, tw, false);
        } else if constexpr (SOLVEZ) {
            solve_z<S>(lds, v, c, a);
        } else {
            store_last<S>(lds, v, c, a);
        }
    }

    // Thread context for tile t.
    __device__ __forceinline__ static Ctx make_ctx(const PassArgs& a, int64_t t) {
        const int tid = threadIdx.x;
        Ctx c;
        if constexpr (STRIDED) {
            const int wave = __builtin_amdgcn_readfirstlane(tid) >> 6;   // wave-uniform
            c.p = tid % P;
            c.j = tid / P;
            const int64_t ctiles = (a.C + P - 1) / P;
            const int64_t rest = t / ctiles;
            const int64_t col0 = (t - rest * ctiles) * P;
            c.col = col0 + c.p;
            c.o1 = rest % a.O1;
            const int64_t o2 = rest / a.O1;
            c.valid = c.col < a.C;
            // element offsets (before the o1, o2 terms) of the tile's first
            // column and of this lane's column; flattened columns step to the
            // next outer index every flat_c columns (cs_out = 1)
            int64_t in0 = col0, inp = c.col, out0 = col0 * a.cs_out, outp = c.col * a.cs_out;
            int64_t span = P;   // bound of the lane offsets within a row
            if (a.flat_c != 0) {
                const int64_t q0 = col0 / a.flat_c, qp = c.col / a.flat_c;
                in0 = col0 + q0 * (a.os1_in - a.flat_c);
                inp = c.col + qp * (a.os1_in - a.flat_c);
                out0 = col0 + q0 * (a.os1_out - a.flat_c);
                outp = c.col + qp * (a.os1_out - a.flat_c);
                // a tile spans at most P / flat_c + 2 outer indices
                span = P + (P / a.flat_c + 1) * (a.os1_in > a.os1_out ? a.os1_in : a.os1_out);
            }
            c.base_in = inp + c.o1 * a.os1_in + o2 * a.os2_in;
            c.base_out = outp + c.o1 * a.os1_out + o2 * a.os2_out;
            // the wave's lanes hold rows jw .. jw + JS - 1 (j grows with tid)
            constexpr int JS = (64 + P - 1) / P + 1;
            const int jw = (wave * 64) / P, jl = c.j - jw;
            c.ies = a.es_in * BI;
            c.oes = a.es_out * BO;
            c.ib = static_cast<const char*>(a.src) + (in0 + c.o1 * a.os1_in + o2 * a.os2_in + jw * a.es_in) * BI;
            c.ob = static_cast<char*>(a.dst) + (out0 + c.o1 * a.os1_out + o2 * a.os2_out + jw * a.es_out) * BO;
            c.il = (uint32_t)(((c.valid ? inp - in0 : 0) + jl * a.es_in) * BI);
            c.ol = (uint32_t)(((outp - out0) + jl * a.es_out) * BO);
            c.split = (span * BI + JS * c.ies) < (int64_t(1) << 32) &&
                      (span * a.cs_out * BO + JS * c.oes) < (int64_t(1) << 32);
        } else {
            c.j = tid % T;
            c.p = tid / T;
            c.col = t * P + c.p;
            c.o1 = 0;
            c.valid = c.col < a.C;
            c.base_in = c.col * a.os1_in;
            c.base_out = c.col * a.os1_out;
            // bases at the tile's first pencil
            constexpr int m0 = PAIRS ? St<0>::NB : 1, mL = PAIRS ? St<NS - 1>::NB : 1;
            c.ies = BI;
            c.oes = BO;
            c.ib = static_cast<const char*>(a.src) + t * P * a.os1_in * BI;
            c.ob = static_cast<char*>(a.dst) + t * P * a.os1_out * BO;
            c.il = (uint32_t)(((c.valid ? c.p : 0) * a.os1_in + c.j * m0) * BI);
            c.ol = (uint32_t)((c.p * a.os1_out + c.j * mL) * BO);
            c.split = (P * a.os1_in + N) * BI < (int64_t(1) << 32) && (P * a.os1_out + N) * BO < (int64_t(1) << 32);
        }
        return c;
    }

    // Whether the contiguous layout's first stage can move its inputs in
    // pairs (decided on the unpaired instance: the butterfly counts are the
    // same under both mappings).
    static constexpr bool pairs_help() {
        return !STRIDED && NT && !REALIN && St<0>::FULL && St<0>::NB % 2 == 0 && St<0>::NBF % 2 == 0;
    }

    // First-stage inputs straight from HBM.
    // Paired accesses: thread slots t and t+1 hold adjacent elements.
    template <int S> static constexpr bool pairable() {
        return PAIRS && NT && St<S>::FULL && St<S>::NB % 2 == 0 && St<S>::NBF % 2 == 0;
    }
    // the paired stores are streaming stores
    template <int S> static constexpr bool pairable_store() { return pairable<S>() && NTS; }
    __device__ __forceinline__ static bool pair_aligned(const void* p, int64_t base) {
        return ((reinterpret_cast<uintptr_t>(p) & (2 * IO::bytes - 1)) == 0) && (base % 2 == 0);
    }

    // Element offset of slot (t, r) of stage S relative to the lane's own
    // part: e = b + r*NBF with b = j + t*T (or j*NB + t when paired).
    template <int S> static constexpr int eoff(int t, int r) {
        return PAIRS ? t + r * St<S>::NBF : t * T + r * St<S>::NBF;
    }

    __device__ __forceinline__ static void load_first(V* v, const Ctx& c, const PassArgs& a) {
        using Q = St<0>;
        if (c.split) {
            if constexpr (pairable<0>()) {
                if (((reinterpret_cast<uintptr_t>(c.ib) + c.il) & (2 * IO::bytes - 1)) == 0) {
#pragma unroll
                    for (int t = 0; t < Q::NB; t += 2)
#pragma unroll
                        for (int r = 0; r < Q::R; ++r)
                            IO::ld2_nt(c.ib + (int64_t)eoff<0>(t, r) * c.ies, c.il, v[t * Q::R + r],
                                       v[(t + 1) * Q::R + r]);
                    return;
                }
            }
#pragma unroll
            for (int t = 0; t < Q::NB; ++t) {
                const int b = Q::bf(c.j, t);
                if (!Q::FULL && b >= Q::NBF) continue;
#pragma unroll
                for (int r = 0; r < Q::R; ++r) v[t * Q::R + r] = ld_in(c.ib + (int64_t)eoff<0>(t, r) * c.ies, c.il);
            }
            return;
        }
        if constexpr (pairable<0>()) {
            if (c.valid && pair_aligned(a.src, c.base_in)) {
#pragma unroll
                for (int t = 0; t < Q::NB; t += 2) {
                    const int b = Q::bf(c.j, t);
#pragma unroll
                    for (int r = 0; r < Q::R; ++r)
                        IO::load2_nt(a.src, c.base_in + b + r * Q::NBF, v[t * Q::R + r], v[(t + 1) * Q::R + r]);
                }
                return;
            }
        }
        const int64_t es = STRIDED ? a.es_in : 1;
#pragma unroll
        for (int t = 0; t < Q::NB; ++t) {
            const int b = Q::bf(c.j, t);
            if (!Q::FULL && b >= Q::NBF) continue;
#pragma unroll
            for (int r = 0; r < Q::R; ++r)
                v[t * Q::R + r] = c.valid ? gload_in(a.src, c.base_in + (int64_t)(b + r * Q::NBF) * es)
                                          : cconst<V>(0.0, 0.0);
        }
    }

    __device__ __forceinline__ static void scale_loaded(V* v, const PassArgs& a) {
        if constexpr (SCALE_IN) {
            using Q = St<0>;
#pragma unroll
            for (int i = 0; i < Q::NB * Q::R; ++i) v[i] = cscale(v[i], a.scale);
        }
    }

    // One tile; the caller owns the LDS and synchronises before reusing it.
    __device__ __forceinline__ static void run_tile(const PassArgs& a, int64_t t, V* lds) {
        const Ctx c = make_ctx(a, t);
        V v[maxv()];
        if constexpr (C2R) load_c2r(v, c, a, lds);
        else load_first(v, c, a);
        scale_loaded(v, a);
        stages<0>(lds, v, c, a, a.tw);
    }
    // The same, calling after_loads() once the tile's loads are issued.
    template <class H>
    __device__ __forceinline__ static void run_tile(const PassArgs& a, int64_t t, V* lds, H&& after_loads) {
        const Ctx c = make_ctx(a, t);
        V v[maxv()];
        load_first(v, c, a);
        after_loads();
        scale_loaded(v, a);
        stages<0>(lds, v, c, a, a.tw);
    }

    __device__ __forceinline__ static void run(const PassArgs& a0, const BatchTable& bt, V* lds) {
        // A merged batch launch first picks its array; both kinds of launch
        // then share one pipeline.
        PassArgs a = a0;
        int64_t t = a0.xcd_order ? xcd_tile(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
        if (bt.count != 0) {
            int i = 0;
            while (i + 1 < bt.count && t >= bt.d[i].tile_end) ++i;
            const ArrayDesc& d = bt.d[i];
            a.src = d.src;
            a.dst = d.dst;
            a.C = d.C;
            a.O1 = d.O1;
            a.es_in = a.es_out = d.es;
            a.os1_in = a.os1_out = d.os1;
            a.scale = d.scale;
            t -= i ? bt.d[i - 1].tile_end : 0;
        }
        run_tile(a, t, lds);
    }
};

template <int N, int T, int P, bool STRIDED, class IO, int SIGN, int FLAGS = 0, int K = 1, int PLAN = 0>
__global__ __launch_bounds__(T * P) void pencil_pass_kernel(PassArgs a, BatchTable bt) {
    using PP = PencilPass<N, T, P, STRIDED, IO, SIGN, FLAGS, K, PLAN>;
    extern __shared__ float2 lds_dyn[];
    PP::run(a, bt, reinterpret_cast<typename PP::V*>(lds_dyn));
}

}  // namespace wsfft
