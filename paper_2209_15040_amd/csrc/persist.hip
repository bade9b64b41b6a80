// One persistent launch for a whole batch of transforms.
//
// The work of a batch is a list of passes (one per array and superstep, in
// superstep-major order), each split into tiles.  Workgroups of a resident
// grid claim tiles in list order from a ticket counter; a tile of superstep
// L > 0 of an array first waits until every tile of superstep L-1 of the same
// array has been published.  Claim order makes this deadlock-free whether or
// not all workgroups are resident at once: a claimed tile depends only on
// tiles claimed earlier, by workgroups that are already running, whose own
// dependencies were claimed earlier still.  The wait is bounded; on timeout the
// launch records an error and finishes.  The last workgroup to leave resets
// the counters, so the next launch on the same counters starts from zero.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "pass_config.hpp"
#include "persist.hpp"

namespace wsfft {
namespace {

constexpr int kPT = kPersistThreads;
constexpr int kPersistFlags = kPassFlags;

// Geometry in the persistent kernel: one butterfly of the widest radix per
// thread and exactly kPersistThreads threads per workgroup.
template <int N, bool ST> struct PGeo {
    static constexpr int T = N / max_radix(make_radices(N, 0));
    static constexpr int P = kPT / T;
    static_assert(T * P == kPT, "persistent geometry must fill the workgroup");
    static constexpr int kfor() {
        if (!ST) return 1;
        for (int k = 1; k <= N; ++k)
            if (N % k == 0 && (N / k) * (P + 1) * 8 <= kLdsRoundBudget) return k;
        return N;
    }
    static constexpr int K = kfor();
    template <int SIGN> using PP = PencilPass<N, T, P, ST, IoC64, SIGN, kPersistFlags, K, 0>;
};

// The lengths of the uneven-batch workload (axes of 32, 64, 96, 128, 256) in
// both layouts.  Each branch inlines a full pass, and registers grow with the
// branch count, so the set is kept to what batches of such shapes need.
#define WSFFT_PERSIST_TYPES(X)                                                                   \
    X(0, 32, false) X(1, 32, true) X(2, 64, false) X(3, 64, true) X(4, 96, false) X(5, 96, true) \
    X(6, 128, false) X(7, 128, true) X(8, 256, false) X(9, 256, true)

constexpr int lds_max() {
    int m = 0;
#define WSFFT_LDS(I, N, ST) m = PGeo<N, ST>::PP<-1>::lds_bytes() > m ? PGeo<N, ST>::PP<-1>::lds_bytes() : m;
    WSFFT_PERSIST_TYPES(WSFFT_LDS)
#undef WSFFT_LDS
    return m;
}
constexpr int kPersistLds = lds_max();

template <int SIGN>
__device__ __forceinline__ void run_type(int type, const PassArgs& a, int64_t t, float2* lds) {
    switch (type) {
#define WSFFT_CASE(I, N, ST) \
    case I: PGeo<N, ST>::template PP<SIGN>::run_tile(a, t, lds); break;
        WSFFT_PERSIST_TYPES(WSFFT_CASE)
#undef WSFFT_CASE
        default: break;
    }
}

__device__ __forceinline__ unsigned load_acquire(const unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Control flow is kept wave-uniform: wave 0 claims (lane 0 issues the atomics,
// readfirstlane broadcasts), every other branch depends on values read back
// through readfirstlane, and one lane-0 region per iteration both publishes the
// previous tile and claims the next.  Two separate lane-0 regions, one at each
// end of the loop body, can be joined by the compiler across the back edge into
// a nested loop that leaves lane 0 parked while the other lanes keep cycling
// through the barriers.  The iteration cap bounds the loop whatever shape it
// is compiled to.
template <int SIGN>
__global__ __launch_bounds__(kPT) void persist_kernel(const PersistPass* __restrict__ passes, int npasses,
                                                      int64_t total, PersistCounters* ctr, unsigned spin_limit) {
    extern __shared__ float2 lds_dyn[];
    __shared__ int64_t s_item;
    __shared__ int s_pass;
    const bool wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x) < 64;   // wave-uniform
    const bool lane0 = threadIdx.x == 0;
    int prev = -1;                 // pass of the tile finished in the previous iteration
    for (int64_t iter = 0; iter <= total; ++iter) {
        if (wave0) {
            unsigned got = 0;
            if (lane0) {
                if (prev >= 0) __hip_atomic_fetch_add(&ctr->done[prev], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                got = atomicAdd(&ctr->ticket, 1u);
            }
            const int64_t item = (int64_t)(unsigned)__builtin_amdgcn_readfirstlane((int)got);
            int pi = -1;
            if (item < total) {   // the pass holding this item (passes sorted by `first`)
                int lo = 0, hi = npasses - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) / 2;
                    if (passes[mid].first <= item) lo = mid;
                    else hi = mid - 1;
                }
                pi = lo;
                const int dep = passes[pi].dep;
                if (dep >= 0) {   // bounded wait for the previous superstep of this array
                    const unsigned need = (unsigned)passes[dep].tiles;
                    for (unsigned spins = 0;; ++spins) {
                        const unsigned have = __builtin_amdgcn_readfirstlane(load_acquire(&ctr->done[dep]));
                        if (have >= need) break;
                        // give up after spin_limit polls, or at once after
                        // another workgroup has given up
                        const unsigned err = __builtin_amdgcn_readfirstlane(
                            __hip_atomic_load(&ctr->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                        if (err != 0u) break;
                        if (spins >= spin_limit) {
                            if (lane0) atomicOr(&ctr->error, 1u);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                }
            }
            if (lane0) {
                s_item = item;
                s_pass = pi;
            }
        }
        __syncthreads();
        const int pi = __builtin_amdgcn_readfirstlane(s_pass);
        if (pi < 0) break;
        const int64_t iv = s_item;   // broadcast through registers: the tile index stays wave-uniform
        const int64_t item = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(iv >> 32)) << 32) |
                                       (uint32_t)__builtin_amdgcn_readfirstlane((int)iv));
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // see the previous superstep
        const PersistPass& P = passes[pi];
        run_type<SIGN>(P.type, P.a, item - P.first, lds_dyn);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // this tile before its publication
        __syncthreads();                           // every thread's stores fenced; LDS free
        prev = pi;
    }
    // last workgroup out resets the counters for the next launch
    if (lane0) {
        const unsigned prevf = __hip_atomic_fetch_add(&ctr->finished, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prevf + 1 == gridDim.x) {
            for (int i = 0; i < npasses; ++i) ctr->done[i] = 0;
            ctr->ticket = 0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(&ctr->finished, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace

int persist_type(int n, bool strided) {
#define WSFFT_TYPE(I, N, ST) \
    if (n == N && strided == ST) return I;
    WSFFT_PERSIST_TYPES(WSFFT_TYPE)
#undef WSFFT_TYPE
    return -1;
}

int persist_per_block(int n, bool strided) {
#define WSFFT_PER(I, N, ST) \
    if (n == N && strided == ST) return PGeo<N, ST>::P;
    WSFFT_PERSIST_TYPES(WSFFT_PER)
#undef WSFFT_PER
    return 0;
}

int persist_lds_bytes() { return kPersistLds; }

hipError_t persist_prepare(int* blocks_per_cu) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&persist_kernel<-1>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kPersistLds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&persist_kernel<1>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kPersistLds);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, reinterpret_cast<const void*>(&persist_kernel<-1>),
                                                         kPT, kPersistLds);
    return e;
}

hipError_t persist_launch(int sign, const PersistPass* passes, int npasses, int64_t total, PersistCounters* ctr,
                          unsigned grid, unsigned spin_limit, hipStream_t s) {
    if (sign < 0)
        hipLaunchKernelGGL(persist_kernel<-1>, dim3(grid), dim3(kPT), kPersistLds, s, passes, npasses, total, ctr,
                           spin_limit);
    else
        hipLaunchKernelGGL(persist_kernel<1>, dim3(grid), dim3(kPT), kPersistLds, s, passes, npasses, total, ctr,
                           spin_limit);
    return hipGetLastError();
}

}  // namespace wsfft
