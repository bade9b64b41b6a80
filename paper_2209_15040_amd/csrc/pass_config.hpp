// Launch geometry of the pencil passes.
//
//   T  threads per pencil          P  pencils (contiguous layout) or
//   K  LDS exchange rounds            columns (strided layout) per workgroup
//
// Rules measured on MI355X at N = 512 (512^3 arrays):
// * strided tiles of 32 columns: 256-byte rows for complex64, 128-byte rows
//   for the 4-byte types (these carry half the bytes and do better with
//   narrower tiles than with 64 columns);
// * strided complex64 tiles run best with radix <= 16 stages (plan 1), the
//   4-byte types with the fewest stages (plan 0);
// * 32 elements per thread, the exchange split into rounds of up to ~72 KB
//   of LDS, so two workgroups stay resident per CU and one's transform and
//   store drain overlap the other's loads;
// * contiguous pencils: N/16 threads each where the widest stage leaves
//   every thread a butterfly (512 points: 16 threads x 32 elements, radix
//   32 x 16, for complex64; 32 threads x 16 elements, radix 8 x 8 x 8, for
//   the 4-byte types), 256-thread workgroups (one wave for the 4-byte types
//   and for 1024-point complex64), and paired (two-element) first-stage
//   loads where the stage allows them;
// * non-temporal (streaming) loads and stores help every pass.
// FP16 storage with FP16 arithmetic (4-byte register and LDS values, argument
// vb = 4) holds half the state per element: strided tiles of 64 columns
// (256-byte rows) with twice the elements per thread, exchange rounds of at
// most ~36 KB, and 256-thread contiguous tiles.
#pragma once
#include "fft_device.hpp"

namespace wsfft {

constexpr int kLdsBytesMax = 160 * 1024;   // LDS per CU on gfx950
constexpr int kLdsRoundBudget = 36 * 1024; // LDS per exchange round, 256-thread strided tiles
constexpr int kPassFlags = kFlagNontemporal;

// Radix plan of the default contiguous kernel: the fewest stages, except
// that pencils of up to 32 points take radix <= 8 stages so that 4 threads
// share a pencil (cfg_T_contig), and the 4-byte storage types take radix
// <= 16 stages (512 points: 8 x 8 x 8 with 16 elements per thread, 185-188
// us per GiB against 197-208 us for 16 x 32).
constexpr int cfg_plan_contig(int N, int bytes = 8) { return N <= 32 ? 2 : (bytes == 4 ? 1 : 0); }

// Radix plan of the default strided kernel (see make_radices).
constexpr int cfg_plan_strided(int N, int bytes) {
    (void)N;
    return bytes == 8 ? 1 : 0;
}

// At least 4 threads per pencil where the radix plan allows: with one
// thread per pencil a wave's 64 lanes read 64 pencils, 64 cache lines per
// access.
constexpr int cfg_T_contig(int N, int plan = 0) {
    int t = N / 16;
    if (t < 4) t = 4;
    // every thread must own at least one butterfly of the widest stage
    const int tmax = N / max_radix(make_radices(N, plan));
    if (tmax >= 1 && t > tmax) t = tmax;
    return t > 1024 ? 1024 : t;
}
// Contiguous tiles: 256-thread workgroups for complex64; one wave for the
// 4-byte types, whose tiles carry half the bytes, so more workgroups (and
// more bytes in flight) fit per CU within the same FP32 LDS budget.  The
// 1024-point complex64 tile is one wave as well (two pencils, 17 KB of LDS:
// 355 us per GiB against 363-390 us for eight pencils in 256 threads).
constexpr int cfg_P_contig(int N, int plan = 0, int bytes = 8, int vb = 8) {
    const int p = ((bytes == 8 && N != 1024) || vb == 4 ? 256 : 64) / cfg_T_contig(N, plan);
    return p < 1 ? 1 : p;
}

constexpr bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
constexpr int pow2_floor(int n) {
    int p = 1;
    while (p * 2 <= n) p *= 2;
    return p;
}

// Elements per thread in the strided layout: 32 for powers of two (16 up to
// N = 128, so that tiles of these short lengths still have 256 threads and
// a CU holds 16 waves); radix-3 stages leave some threads idle, so fewer
// there to stay within registers.
// Past 512 threads per tile (32 columns x 16 threads) the elements per thread
// double instead: 1024-thread workgroups are held to 128 VGPRs and spill.
constexpr int cfg_T_strided(int N, int bytes, int plan = 0, int vb = 8) {
    (void)bytes;
    int e = is_pow2(N) ? (N <= 128 ? 16 : 32) : 24;
    if ((N + e - 1) / e > 16) e *= 2;
    if (vb == 4 && is_pow2(N) && N <= 512) e *= 2;   // longer or radix-3 pencils would spill
    int t = (N + e - 1) / e;
    const int tmax = N / max_radix(make_radices(N, plan));
    if (tmax >= 1 && t > tmax) t = tmax;
    return t < 1 ? 1 : t;
}
constexpr int cfg_P_strided(int N, int bytes, int plan = 0, int vb = 8) {
    (void)bytes;
    int p = 32;
    if (N <= 64 || (vb == 4 && is_pow2(N))) p = 64;   // one full wave of columns at least
    const int cap = pow2_floor(1024 / cfg_T_strided(N, bytes, plan, vb));
    return p > cap ? cap : p;
}
// Smallest K dividing N whose exchange round fits the LDS budget (twice the
// per-round budget for workgroups of up to 512 threads, two of which still
// fit per CU; four times at 1024 points); when that takes more than 8
// rounds, accept up to twice the budget instead.
constexpr int cfg_K_strided(int N, int bytes, int plan = 0, int vb = 8) {
    const int p = cfg_P_strided(N, bytes, plan, vb);
    // 1024-point tiles run best with two rounds and one workgroup per CU
    const int budget = vb == 4 ? kLdsRoundBudget
                       : N >= 1024 ? 4 * kLdsRoundBudget
                       : cfg_T_strided(N, bytes, plan) * p <= 512 ? 2 * kLdsRoundBudget : kLdsRoundBudget;
    int first = 0;
    for (int k = 1; k <= N && !first; ++k)
        if (N % k == 0 && (N / k) * (p + 1) * vb <= budget) first = k;
    if (first && first <= 8) return first;
    for (int k = 1; k <= N; ++k)
        if (N % k == 0 && (N / k) * (p + 1) * vb <= 2 * kLdsRoundBudget) return k;
    return first ? first : N;
}

// Longest pencil a single pass handles in each layout.
constexpr int kMaxContigN = 16384;   // one pencil of 16384 complex in LDS
constexpr int kMaxStridedN = 1024;

}  // namespace wsfft
