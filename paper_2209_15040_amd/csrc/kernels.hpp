// Host-side registry of the compiled pencil-pass kernels.
#pragma once
#include <hip/hip_runtime.h>
#include "fft_device.hpp"

namespace wsfft {

enum StorageKind { kC64 = 0, kF16 = 1, kBF16 = 2, kF16Math = 3 };   // kF16Math: FP16 storage, FP16 arithmetic

struct PassKernel {
    int n;              // pencil length
    bool strided;       // layout: columns unit-stride (true) or pencils contiguous
    bool four_step;     // compiled with the split-axis first-pass features
    int variant;        // 0: default; 1: radix <= 8 plan; 2: half-width strided tiles
    int threads;        // workgroup size
    int per_block;      // pencils (contiguous) or columns (strided) per workgroup
    int lds_bytes;      // dynamic LDS per workgroup
    int plan;           // radix plan (make_radices)
    // bt == nullptr: one array described by the PassArgs; otherwise a merged
    // batch of direct passes (PassArgs supplies the shared fields)
    hipError_t (*launch)(const PassArgs&, const BatchTable* bt, dim3 grid, hipStream_t);
    hipError_t (*prepare)();   // one-time function attributes
    int fused;          // 0: plain pass; complex64 only: Poisson solve passes
                        // 1 real input, 2 times -1/|k|^2, 3 real output;
                        // 4 R2C x pass, 5 C2R x pass, 6 fused solve z pass,
                        // 7 pass with cached loads and stores,
                        // 8 fused x and y passes of whole planes,
                        // 9 contiguous pass with streaming loads and cached stores
    int n2;             // fused plane passes: the y length (n is the x length)
};

enum FusedKind {
    kFusedNone = 0, kFusedRealIn = 1, kFusedPoisson = 2, kFusedRealOut = 3,
    kFusedR2C = 4, kFusedC2R = 5, kFusedSolveZ = 6,
    kFusedCached = 7,  // a plain pass with cached (not streaming) loads and stores
    kFusedPlane = 8,   // the x and y transforms of whole xy-planes in LDS (plane.hip)
    kFusedCachedStore = 9   // a plain contiguous pass with streaming loads and cached stores
};

// NULL when no kernel of that length/layout/variant exists.
const PassKernel* find_pass_kernel(StorageKind kind, int sign, int n, bool strided, bool four_step,
                                   int variant = 0);
constexpr int kMaxVariants = 3;

#define WSFFT_DECLARE_FIND(NAME) const PassKernel* NAME(int n, bool strided, bool four_step, int variant);
WSFFT_DECLARE_FIND(find_pass_c64_neg)
WSFFT_DECLARE_FIND(find_pass_c64_pos)
WSFFT_DECLARE_FIND(find_pass_f16_neg)
WSFFT_DECLARE_FIND(find_pass_f16_pos)
WSFFT_DECLARE_FIND(find_pass_bf16_neg)
WSFFT_DECLARE_FIND(find_pass_bf16_pos)
WSFFT_DECLARE_FIND(find_pass_f16m_neg)
WSFFT_DECLARE_FIND(find_pass_f16m_pos)
#undef WSFFT_DECLARE_FIND
// Fused Poisson-solve kernels (complex64; real input and the multiplier with
// sign -1, real output with sign +1).  NULL when none exists for n.
const PassKernel* find_fused_c64_neg(int n, bool strided, int fused);
const PassKernel* find_fused_c64_pos(int n, bool strided, int fused);
// Real-data kernels (complex64): R2C x passes and fused solve z passes with
// sign -1 (_neg), C2R x passes with sign +1 (_pos); n is the pencil length of
// the complex transform (half the real length for the x passes).
const PassKernel* find_real_c64_neg(int n, bool strided, int fused);
const PassKernel* find_real_c64_pos(int n, bool strided, int fused);
// Passes that go through the caches (kind kFusedCached: cached loads and
// stores, both layouts, complex64 only; kFusedCachedStore: contiguous,
// streaming loads and cached stores, every storage type).  NULL when none
// exists.
const PassKernel* find_cached_kernel(StorageKind kind, int sign, int n, bool strided, int fused);
#define WSFFT_DECLARE_CACHED(NAME) const PassKernel* NAME(int n, bool strided, int fused);
WSFFT_DECLARE_CACHED(find_cached_c64_neg)
WSFFT_DECLARE_CACHED(find_cached_c64_pos)
WSFFT_DECLARE_CACHED(find_cached_f16_neg)
WSFFT_DECLARE_CACHED(find_cached_f16_pos)
WSFFT_DECLARE_CACHED(find_cached_bf16_neg)
WSFFT_DECLARE_CACHED(find_cached_bf16_pos)
WSFFT_DECLARE_CACHED(find_cached_f16m_neg)
WSFFT_DECLARE_CACHED(find_cached_f16m_pos)
#undef WSFFT_DECLARE_CACHED
// Fused x + y plane pass of complex64 nx x ny planes; NULL when none exists.
const PassKernel* find_plane_kernel(int nx, int ny, int sign);

}  // namespace wsfft
