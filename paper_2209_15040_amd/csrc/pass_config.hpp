// Launch geometry of the pencil passes: threads per pencil (T) and pencils
// (contiguous layout) or columns (strided layout) per workgroup (P).
#pragma once
#include "fft_device.hpp"

namespace wsfft {

constexpr int kLdsBytesMax = 160 * 1024;   // LDS per CU on gfx950

constexpr int cfg_T_contig(int N) {
    const int t = N / max_radix(make_radices(N));
    return t < 1 ? 1 : (t > 1024 ? 1024 : t);
}
constexpr int cfg_P_contig(int N) {
    const int p = 256 / cfg_T_contig(N);
    return p < 1 ? 1 : p;
}

// Strided tiles want row segments of at least 128 bytes in storage:
// 16 columns of complex64, 32 columns of 4-byte complex.
constexpr int cfg_P_strided(int N, int bytes) {
    int p = bytes == 8 ? 16 : 32;
    const int t = N / max_radix(make_radices(N));
    if (t > 0 && t * p < 256) {            // small N: widen the tile
        const int want = 256 / t;
        p = want > 64 ? 64 : want;
    }
    while (p > 1 && N * (p + 1) * 8 > kLdsBytesMax) p /= 2;
    return p;
}
constexpr int cfg_T_strided(int N, int bytes) {
    const int p = cfg_P_strided(N, bytes);
    int t = N / max_radix(make_radices(N));
    if (t < 1) t = 1;
    const int cap = 1024 / p;
    return t > cap ? cap : t;
}

// Longest pencil a single pass handles in each layout (LDS capacity).
constexpr int kMaxContigN = 16384;
constexpr int kMaxStridedN = 1024;

}  // namespace wsfft
