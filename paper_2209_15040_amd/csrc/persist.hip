// One persistent launch for a whole batch of transforms.
//
// The work of a batch is a list of passes (one per array and superstep), in
// superstep-major order, each split into tiles.  Workgroups of a resident
// grid claim tiles in list order from a ticket counter.  Synchronisation is
// per superstep level: a workgroup counts the tiles it finishes and publishes
// them (one release, one counter add) only when its next ticket belongs to a
// higher level or when it leaves; at its first tile of level L > 0 it waits
// until every tile of level L-1 has been published, then acquires once.  The
// cache-wide write-back and invalidate that release and acquire cost across
// the XCDs' separate L2s thus happen a few times per workgroup, not per tile.
// Claim order makes the wait deadlock-free whether or not all workgroups are
// resident at once: a workgroup waits only after publishing everything it
// holds, and every earlier tile belongs to a running workgroup that will
// publish it when it claims its next ticket or leaves.  The wait is bounded;
// on timeout the launch records an error and finishes.  The last workgroup to
// leave resets the counters, so the next launch on the same counters starts
// from zero: it moves a recorded error into a count of failed launches, which
// only the host reads and clears, so one timed-out launch never makes a
// later launch skip its waits.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "pass_config.hpp"
#include "persist.hpp"

namespace wsfft {
namespace {

constexpr int kPT = kPersistThreads;
constexpr int kPersistFlags = kPassFlags;

// Geometry in the persistent kernel: one butterfly of the widest radix per
// thread (two for strided 256-point tiles) and exactly kPersistThreads
// threads per workgroup.  Contiguous
// 32-point pencils take radix <= 8 stages, 4 threads per pencil: with one
// thread per pencil a wave's loads touch 64 cache lines each.
template <int N, bool ST> struct PGeo {
    static constexpr int PLAN = (!ST && N == 32) ? 2 : 0;
    // strided 256-point tiles: 8 threads per column, so that a tile spans
    // 32 columns (256-byte rows) rather than 16
    static constexpr int T = (ST && N == 256) ? 8 : N / max_radix(make_radices(N, PLAN));
    static constexpr int P = kPT / T;
    static_assert(T * P == kPT, "persistent geometry must fill the workgroup");
    static constexpr int kfor() {
        if (!ST) return 1;
        for (int k = 1; k <= N; ++k)
            if (N % k == 0 && (N / k) * (P + 1) * 8 <= kLdsRoundBudget) return k;
        return N;
    }
    static constexpr int K = kfor();
    template <int SIGN> using PP = PencilPass<N, T, P, ST, IoC64, SIGN, kPersistFlags, K, PLAN>;
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

template <int SIGN, class H>
__device__ __forceinline__ void run_type(int type, const PassArgs& a, int64_t t, float2* lds, H&& after_loads) {
    switch (type) {
#define WSFFT_CASE(I, N, ST) \
    case I: PGeo<N, ST>::template PP<SIGN>::run_tile(a, t, lds, after_loads); break;
        WSFFT_PERSIST_TYPES(WSFFT_CASE)
#undef WSFFT_CASE
        default: break;
    }
}

// A coherent (agent-scope) load of a counter without ordering: an acquire
// load would invalidate the caches at every poll.
__device__ __forceinline__ unsigned load_relaxed(const unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Control flow is kept wave-uniform: wave 0 claims (lane 0 issues the atomics,
// readfirstlane broadcasts) and every branch depends on values read back
// through readfirstlane.  Lane-0 regions hold no barrier and no back edge of
// the loop: two such regions at both ends of a loop body can be joined by the
// compiler across the back edge into a nested loop that parks lane 0 while
// the other lanes keep cycling through the barriers.  The iteration cap
// bounds the loop whatever shape it is compiled to.  Two workgroups per CU:
// held to three (168 VGPRs) the kernel runs 7% slower than with the 188 it
// takes at two (no spills either way).
template <int SIGN>
__global__ __launch_bounds__(kPT, 2) void persist_kernel(const PersistPass* __restrict__ passes, int npasses,
                                                      PersistLevels lv, PersistCounters* ctr, unsigned spin_limit) {
    extern __shared__ float2 lds_dyn[];
    __shared__ int64_t s_item;
    __shared__ int s_pass;
    __shared__ unsigned s_next;   // the ticket claimed during the previous tile
    const bool wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x) < 64;   // wave-uniform
    const bool lane0 = threadIdx.x == 0;
    const int64_t total = lv.end[lv.count - 1];
    int level = -1;          // level of the tiles finished since the last publication
    unsigned pending = 0;    // those tiles
    bool first = true;
    int cur = 0;             // wave 0: pass of the last item (items only grow)
    for (int64_t iter = 0; iter <= total; ++iter) {
        if (wave0) {
            unsigned got = 0;
            if (lane0) got = first ? atomicAdd(&ctr->ticket, 1u) : s_next;
            const int64_t item = (int64_t)(unsigned)__builtin_amdgcn_readfirstlane((int)got);
            int pi = -1;
            if (item < total) {
                // the pass holding this item (passes sorted by `first`)
                while (cur + 1 < npasses && passes[cur + 1].first <= item) ++cur;
                pi = cur;
            }
            if (lane0) {
                s_item = item;
                s_pass = pi;
            }
        }
        first = false;
        __syncthreads();
        const int pi = __builtin_amdgcn_readfirstlane(s_pass);
        const int L = pi < 0 ? kPersistMaxLevels : __builtin_amdgcn_readfirstlane(passes[pi].level);
        if (L != level) {
            if (pending != 0) {   // publish the finished tiles of `level`
                // Each wave waits for its own stores to reach the L2; then one
                // agent-scope release by wave 0 writes the XCD's L2 back for
                // the whole workgroup (the write-back is cache-wide, and the
                // barrier orders the other waves' stores before it), and the
                // count goes out after it.  A release per wave would repeat
                // the cache-wide write-back four times.
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                if (wave0) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    if (lane0)
                        __hip_atomic_fetch_add(&ctr->done[level], pending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                pending = 0;
            }
            if (L > 0 && L < kPersistMaxLevels) {   // bounded wait for the whole previous level
                if (wave0) {
                    const unsigned need = (unsigned)(lv.end[L - 1] - (L >= 2 ? lv.end[L - 2] : 0));
                    for (unsigned spins = 0;; ++spins) {
                        const unsigned have = __builtin_amdgcn_readfirstlane(load_relaxed(&ctr->done[L - 1]));
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
                    // the polls read the counter without ordering; one acquire
                    // after the last invalidates this CU's L1 and the XCD's L2
                    // for the whole workgroup, and the barrier orders the other
                    // waves' loads after it (an acquire per wave would repeat
                    // the cache-wide invalidation)
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
                __syncthreads();
            }
            level = L;
        }
        if (pi < 0) break;
        const int64_t iv = s_item;   // broadcast through registers: the tile index stays wave-uniform
        const int64_t item = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(iv >> 32)) << 32) |
                                       (uint32_t)__builtin_amdgcn_readfirstlane((int)iv));
        const PersistPass& P = passes[pi];
        // Claim the following ticket before this tile's loads and read it back
        // right after them: the wait for it is then not a wait for this or the
        // previous tile's stores (loads and stores share one in-order
        // counter).  A held ticket is never of a lower level than the current
        // one, so waiting for the previous level cannot depend on it.
        unsigned nxt = 0;
        if (lane0) nxt = atomicAdd(&ctr->ticket, 1u);
        run_type<SIGN>(P.type, P.a, item - P.first, lds_dyn, [&] {
            if (lane0) s_next = nxt;
        });
        __syncthreads();   // LDS and the shared slots free for the next tile
        ++pending;
    }
    // last workgroup out resets the counters for the next launch
    if (lane0) {
        // The tiles were written back at the last publication; waiting for
        // this lane's counter atomics to complete puts them before its count
        // (without a cache-wide write-back per workgroup).  Only the last
        // workgroup out needs the acquire.
        __builtin_amdgcn_s_waitcnt(0);
        const unsigned prevf = __hip_atomic_fetch_add(&ctr->finished, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (prevf + 1 == gridDim.x) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            for (int i = 0; i < kPersistMaxLevels; ++i) ctr->done[i] = 0;
            ctr->ticket = 0;
            if (__hip_atomic_load(&ctr->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                __hip_atomic_fetch_add(&ctr->failed, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&ctr->error, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
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

int persist_plan(int n, bool strided) {
#define WSFFT_PLAN(I, N, ST) \
    if (n == N && strided == ST) return PGeo<N, ST>::PLAN;
    WSFFT_PERSIST_TYPES(WSFFT_PLAN)
#undef WSFFT_PLAN
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

hipError_t persist_launch(int sign, const PersistPass* passes, int npasses, const PersistLevels& levels,
                          PersistCounters* ctr, unsigned grid, unsigned spin_limit, hipStream_t s) {
    if (sign < 0)
        hipLaunchKernelGGL(persist_kernel<-1>, dim3(grid), dim3(kPT), kPersistLds, s, passes, npasses, levels, ctr,
                           spin_limit);
    else
        hipLaunchKernelGGL(persist_kernel<1>, dim3(grid), dim3(kPT), kPersistLds, s, passes, npasses, levels, ctr,
                           spin_limit);
    return hipGetLastError();
}

}  // namespace wsfft
