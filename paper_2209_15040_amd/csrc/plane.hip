// The x and y supersteps of an array whose xy-plane fits in LDS, fused into
// one pass.  Supersteps may be grouped freely (paper, Section 1: the 1D
// transforms along each axis can be taken in any order); a workgroup loads a
// whole plane (nx * ny contiguous complex64 values, at most 128 KiB), runs
// every x transform and then every y transform of it in LDS, and stores it,
// so the array makes two HBM round trips (plane, then z) instead of three.
//
// Each transform is the same Stockham schedule as the pencil passes (stage
// s: radix R, sub-length Ns, butterfly b reads b + r*N/R and writes
// (b div Ns)*Ns*R + (b mod Ns) + r*Ns), with radix <= 16 stages.  A stage
// reads every butterfly's inputs from LDS into registers, synchronises, and
// writes the outputs back in place.
#include <hip/hip_runtime.h>

#include <mutex>
#include <set>
#include <utility>

#include "kernels.hpp"
#include "pass_config.hpp"
#include "plane.hpp"

namespace wsfft {
namespace {

// threads per workgroup: 1024 for planes above 8192 values (one such
// workgroup per CU: its LDS holds the whole plane), 512 for 4096 .. 8192,
// else 256 (a 32 x 32 plane gives 256 threads one butterfly each per stage)
constexpr int plane_threads(int values) { return values > 8192 ? 1024 : (values >= 4096 ? 512 : 256); }
constexpr int kPlaneRadixPlan = 1;   // stage twiddle block of radix plan 1 (radix <= 16)

template <int NX, int NY, int SIGN>
struct PlaneXY {
    static constexpr int E = NX * NY;
    static constexpr int kPlaneThreads = plane_threads(E);
    static_assert(E * 8 <= 128 * 1024, "a plane holds at most 16384 values");
    // LDS row pitch: 4 values (32 bytes) of padding per row, so the threads
    // of an x stage, which take 8 to 16 consecutive butterflies of each of
    // several rows, spread over all banks (rows NX * 8 bytes apart would all
    // start on the same bank); even, so two-value accesses stay 16-byte aligned
    static constexpr int LX = NX + 4;
    static constexpr int lds_bytes() { return NY * LX * (int)sizeof(float2); }

    // Stage S of length-N transforms over COUNT pencils; element e of pencil
    // q sits at lds[q * QS + e * ES].  ROWMAJOR: consecutive threads take
    // consecutive butterflies of one pencil (unit-stride pencils); else
    // consecutive pencils of one butterfly (pencils of stride LX, whose
    // neighbours sit next to each other in LDS).  GIN: the inputs come from
    // the plane in global memory (element e of pencil q at gin[q * NX + e])
    // instead of LDS; GOUT: the outputs go to global memory (element e of
    // pencil q at gout[e * NX + q], times scale) instead of LDS.
    template <int N, int COUNT, int QS, int ES, bool ROWMAJOR, int S, bool GIN, bool GOUT>
    __device__ __forceinline__ static void stage(float2* lds, const float2* tw, const char* gin, char* gout,
                                                 float scale) {
        constexpr Radices RD = make_radices(N, kPlaneRadixPlan);
        constexpr int R = RD.r[S];
        constexpr int Ns = stage_ns(RD, S);
        constexpr int NBF = N / R;
        constexpr int TOTAL = COUNT * NBF;
        constexpr int PER = (TOTAL + kPlaneThreads - 1) / kPlaneThreads;
        constexpr int off = stage_tw_offset(RD, S);
        float2 u[PER][R];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int g = (int)threadIdx.x + i * kPlaneThreads;
            if (TOTAL % kPlaneThreads != 0 && g >= TOTAL) continue;
            const int q = ROWMAJOR ? g / NBF : g % COUNT;
            const int b = ROWMAJOR ? g % NBF : g / COUNT;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if constexpr (GIN) {
                    const f32x2 v = __builtin_nontemporal_load(
                        gload_at<f32x2>(gin, (uint32_t)(q * NX + b + r * NBF) * 8u));
                    u[i][r] = make_float2(v.x, v.y);
                } else {
                    u[i][r] = lds[q * QS + (b + r * NBF) * ES];
                }
            }
            if constexpr (S > 0) {
                const int k = b % Ns;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const f32x2 w = *gload_at<f32x2>(reinterpret_cast<const char*>(tw),
                                                     (uint32_t)(off + (r - 1) * Ns + k) * 8u);
                    u[i][r] = cmul(u[i][r], make_float2(w.x, SIGN > 0 ? -w.y : w.y));
                }
            }
            Dft<R, SIGN>::run(u[i]);
        }
        if constexpr (!GIN && !GOUT) __syncthreads();   // in place in LDS: every read before any write
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int g = (int)threadIdx.x + i * kPlaneThreads;
            if (TOTAL % kPlaneThreads != 0 && g >= TOTAL) continue;
            const int q = ROWMAJOR ? g / NBF : g % COUNT;
            const int b = ROWMAJOR ? g % NBF : g / COUNT;
            const int o = (b / Ns) * Ns * R + b % Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if constexpr (GOUT) {
                    f32x2 v;
                    v.x = u[i][r].x * scale;
                    v.y = u[i][r].y * scale;
                    __builtin_nontemporal_store(v, gstore_at<f32x2>(gout, (uint32_t)((o + r * Ns) * NX + q) * 8u));
                } else {
                    lds[q * QS + (o + r * Ns) * ES] = u[i][r];
                }
            }
        }
        if constexpr (!GOUT) __syncthreads();
    }

    // all stages of one transform set; the first may read global memory, the
    // last may write it
    template <int N, int COUNT, int QS, int ES, bool ROWMAJOR, bool GIN, bool GOUT, int S = 0>
    __device__ __forceinline__ static void transform(float2* lds, const float2* tw, const char* gin, char* gout,
                                                     float scale) {
        constexpr Radices RD = make_radices(N, kPlaneRadixPlan);
        if constexpr (S < RD.n) {
            stage<N, COUNT, QS, ES, ROWMAJOR, S, GIN && S == 0, GOUT && S + 1 == RD.n>(lds, tw, gin, gout, scale);
            transform<N, COUNT, QS, ES, ROWMAJOR, GIN, GOUT, S + 1>(lds, tw, gin, gout, scale);
        }
    }

    // Plane t of an array: a.C planes of a.os1_in elements (= nx * ny) each,
    // in place or out of place; a.tw holds the x stage twiddles, a.tw4 the y
    // stage twiddles (radix plan 1 blocks); a.scale multiplies every store.
    // The first x stage reads the plane from HBM and the last y stage writes
    // it back, so LDS holds the plane only between stages.
    __device__ __forceinline__ static void run_plane(const PassArgs& a, int64_t t, float2* lds) {
        run(a.src, a.dst, a.tw, a.tw4, a.os1_in, a.os1_out, a.scale, t, lds);
    }
    __device__ __forceinline__ static void run(const void* src0, void* dst0, const float2* tw, const float2* tw4,
                                               int64_t stride_in, int64_t stride_out, float scale, int64_t t,
                                               float2* lds) {
        const char* src = reinterpret_cast<const char*>(static_cast<const float2*>(src0) + t * stride_in);
        char* dst = reinterpret_cast<char*>(static_cast<float2*>(dst0) + t * stride_out);
        transform<NX, NY, LX, 1, true, true, false>(lds, tw, src, nullptr, 1.0f);    // rows: pencils along x
        transform<NY, NX, 1, LX, false, false, true>(lds, tw4, nullptr, dst, scale);   // columns: along y
    }
};

template <int NX, int NY, int SIGN>
__global__ __launch_bounds__(plane_threads(NX * NY)) void plane_kernel(PassArgs a0, BatchTable bt) {
    extern __shared__ float2 lds_dyn[];
    PassArgs a = a0;
    int64_t t = blockIdx.x;
    if (bt.count != 0) {   // merged launch over several arrays: pick the array, as the pencil passes do
        int i = 0;
        while (i + 1 < bt.count && t >= bt.d[i].tile_end) ++i;
        const ArrayDesc& d = bt.d[i];
        a.src = d.src;
        a.dst = d.dst;
        a.C = d.C;
        a.os1_in = a.os1_out = d.os1;
        a.scale = d.scale;
        t -= i ? bt.d[i - 1].tile_end : 0;
    }
    PlaneXY<NX, NY, SIGN>::run_plane(a, t, lds_dyn);
}

template <int NX, int NY, int SIGN>
hipError_t plane_launch(const PassArgs& a, const BatchTable* bt, dim3 grid, hipStream_t s) {
    static const BatchTable kNone{};
    constexpr int lds = PlaneXY<NX, NY, SIGN>::lds_bytes();
    hipLaunchKernelGGL((plane_kernel<NX, NY, SIGN>), grid, dim3(plane_threads(NX * NY)), lds, s, a, bt ? *bt : kNone);
    return hipGetLastError();
}

template <int NX, int NY, int SIGN>
hipError_t plane_prepare() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&plane_kernel<NX, NY, SIGN>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, PlaneXY<NX, NY, SIGN>::lds_bytes());
}

// (nx, ny) pairs with a fused plane pass: the axis lengths of the uneven
// batch workload (32 .. 256) whose plane holds at most 16384 values (planes
// of up to 8192 values let two workgroups share a CU; the larger ones take
// one, and still beat the two passes they replace: 96 x 96 x 128 17 against
// 20 us, 128 x 128 x 256 31 against 42 us; 128 x 128 x 64, 21 against 18 us,
// is the exception among the batch's shapes)
#define WSFFT_PLANES(X)                                                                             \
    X(32, 32) X(32, 64) X(64, 32) X(32, 96) X(96, 32) X(32, 128) X(128, 32) X(32, 256) X(256, 32) \
    X(64, 64) X(64, 96) X(96, 64) X(64, 128) X(128, 64)                                           \
    X(96, 96) X(128, 96) X(96, 128) X(128, 128) X(64, 256) X(256, 64)

#define WSFFT_PLANE_ENTRY(NX, NY, SIGN)                                                                        \
    {NX, false, false, 0, plane_threads(NX * NY), 1, PlaneXY<NX, NY, SIGN>::lds_bytes(), kPlaneRadixPlan,     \
     &plane_launch<NX, NY, SIGN>, &plane_prepare<NX, NY, SIGN>, kFusedPlane, NY},
#define WSFFT_PLANE_NEG(NX, NY) WSFFT_PLANE_ENTRY(NX, NY, -1)
#define WSFFT_PLANE_POS(NX, NY) WSFFT_PLANE_ENTRY(NX, NY, 1)

const PassKernel kPlaneNeg[] = {WSFFT_PLANES(WSFFT_PLANE_NEG)};
const PassKernel kPlanePos[] = {WSFFT_PLANES(WSFFT_PLANE_POS)};

// Plane passes of several shapes in one launch.  A merged batch level would
// otherwise launch once per plane shape, and most of those launches are too
// small to fill the chip (a few hundred planes, some microseconds each, the
// start-up and the last partial wave of workgroups costing as much as the
// transform); one launch per class keeps the chip full from one shape's
// planes to the next.  A class groups the shapes that share a workgroup size
// and an LDS bracket, so a class launch keeps the residency of its shapes'
// own launches.
struct PlaneShape {
    int nx, ny;
};
#define WSFFT_PLANE_SHAPE(NX, NY) {NX, NY},
constexpr PlaneShape kPlaneShapes[] = {WSFFT_PLANES(WSFFT_PLANE_SHAPE)};
constexpr int kNumPlaneShapes = (int)(sizeof(kPlaneShapes) / sizeof(kPlaneShapes[0]));
// below 4096 values: 256 threads, at most 28 KB of LDS; 4096 .. 6144: 512
// threads, at most 53 KB; 8192: 512 threads, at most 74 KB; 9216 .. 16384:
// 1024 threads, at most 136 KB
constexpr int class_of(int values) { return values < 4096 ? 0 : (values <= 6144 ? 1 : (values <= 8192 ? 2 : 3)); }
constexpr int class_threads(int cls) { return cls == 0 ? 256 : (cls == 3 ? 1024 : 512); }
constexpr int shape_lds(int nx, int ny) { return ny * (nx + 4) * (int)sizeof(float2); }
constexpr int class_lds(int cls) {
    int m = 0;
    for (const PlaneShape& p : kPlaneShapes)
        if (class_of(p.nx * p.ny) == cls && shape_lds(p.nx, p.ny) > m) m = shape_lds(p.nx, p.ny);
    return m;
}
static_assert(kPlaneClasses == 4, "four plane classes");

template <int CLS, int SIGN, int S = 0>
__device__ __forceinline__ void run_shape(const PlaneEntry& e, int64_t t, float2* lds) {
    if constexpr (S < kNumPlaneShapes) {
        constexpr int NX = kPlaneShapes[S].nx, NY = kPlaneShapes[S].ny;
        if constexpr (class_of(NX * NY) == CLS) {
            static_assert(plane_threads(NX * NY) == class_threads(CLS), "a class shares one workgroup size");
            static_assert(PlaneXY<NX, NY, SIGN>::lds_bytes() == shape_lds(NX, NY), "LDS of a plane shape");
            if (e.shape == S) {
                PlaneXY<NX, NY, SIGN>::run(e.src, e.dst, e.tw, e.tw4, e.stride, e.stride, e.scale, t, lds);
                return;
            }
        }
        run_shape<CLS, SIGN, S + 1>(e, t, lds);
    }
}

template <int CLS, int SIGN>
__global__ __launch_bounds__(class_threads(CLS)) void plane_class_kernel(PlaneTable pt) {
    extern __shared__ float2 lds_dyn[];
    const int64_t b = blockIdx.x;
    int i = 0;
    while (i + 1 < pt.count && b >= pt.e[i].plane_end) ++i;
    run_shape<CLS, SIGN>(pt.e[i], b - (i ? pt.e[i - 1].plane_end : 0), lds_dyn);
}

template <int CLS, int SIGN>
hipError_t class_launch(const PlaneTable& t, unsigned planes, int lds, hipStream_t s) {
    hipLaunchKernelGGL((plane_class_kernel<CLS, SIGN>), dim3(planes), dim3(class_threads(CLS)), lds, s, t);
    return hipGetLastError();
}

template <int CLS, int SIGN>
hipError_t class_prepare() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&plane_class_kernel<CLS, SIGN>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, class_lds(CLS));
}

using ClassLaunch = hipError_t (*)(const PlaneTable&, unsigned, int, hipStream_t);
using ClassPrepare = hipError_t (*)();
const ClassLaunch kClassLaunch[2][kPlaneClasses] = {
    {&class_launch<0, -1>, &class_launch<1, -1>, &class_launch<2, -1>, &class_launch<3, -1>},
    {&class_launch<0, 1>, &class_launch<1, 1>, &class_launch<2, 1>, &class_launch<3, 1>}};
const ClassPrepare kClassPrepare[2][kPlaneClasses] = {
    {&class_prepare<0, -1>, &class_prepare<1, -1>, &class_prepare<2, -1>, &class_prepare<3, -1>},
    {&class_prepare<0, 1>, &class_prepare<1, 1>, &class_prepare<2, 1>, &class_prepare<3, 1>}};

}  // namespace

const PassKernel* find_plane_kernel(int nx, int ny, int sign) {
    for (const PassKernel& k : (sign < 0 ? kPlaneNeg : kPlanePos))
        if (k.n == nx && k.n2 == ny) return &k;
    return nullptr;
}

bool plane_shape_info(int nx, int ny, int* cls, int* shape, int* lds_bytes) {
    for (int i = 0; i < kNumPlaneShapes; ++i)
        if (kPlaneShapes[i].nx == nx && kPlaneShapes[i].ny == ny) {
            *cls = class_of(nx * ny);
            *shape = i;
            *lds_bytes = shape_lds(nx, ny);
            return true;
        }
    return false;
}

hipError_t plane_class_prepare(int cls, int sign) {
    if (cls < 0 || cls >= kPlaneClasses) return hipErrorInvalidValue;
    // once per kernel and device
    static std::mutex mu;
    static std::set<std::pair<int, int>> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const int key = (sign < 0 ? 0 : kPlaneClasses) + cls;
    std::lock_guard<std::mutex> lk(mu);
    if (done.count({dev, key})) return hipSuccess;
    e = kClassPrepare[sign < 0 ? 0 : 1][cls]();
    if (e == hipSuccess) done.insert({dev, key});
    return e;
}

hipError_t plane_class_launch(int cls, int sign, const PlaneTable& t, unsigned planes, int lds, hipStream_t s) {
    if (cls < 0 || cls >= kPlaneClasses || t.count < 1 || t.count > kMaxPlaneEntries || lds > class_lds(cls) ||
        planes != (unsigned)t.e[t.count - 1].plane_end)
        return hipErrorInvalidValue;
    return kClassLaunch[sign < 0 ? 0 : 1][cls](t, planes, lds, s);
}

}  // namespace wsfft
