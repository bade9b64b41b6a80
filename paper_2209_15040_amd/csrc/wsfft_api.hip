// C-ABI of the MI355X multidimensional FFT: plans, pass schedules, twiddle
// tables and the execute entry points.  The interface is declared and
// documented in include/wsfft.h.
//
// Schedule (paper, Section 1 and Section 2.2; redistribution as in Section
// 4.3, done here by addressing): one pencil pass per axis of length > 1.  An
// axis whose pencils are unit-stride runs in the contiguous layout, the others
// in the strided layout (tiles of adjacent columns).  An axis too long for one
// pass of its layout is split n = n1 * n2 (four-step, the decomposition the
// paper suggests for very long 1D transforms in Section 8) into two passes:
//   A: length-n1 DFTs over y1 of a[n2*y1 + y2], times W_n^(y2*k1),
//      written to position k1 + n1*y2
//   B: length-n2 DFTs over y2 of positions k1 + n1*y2, written in place,
//      which leaves X[k1 + n1*k2] at position k1 + n1*k2.
// Pass A cannot run in place, so split axes go first and read the input.
#include <hip/hip_runtime.h>

#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <set>
#include <sstream>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/wsfft.h"
#include "../../include/wsfft_pointwise.h"
#include "kernels.hpp"
#include "pass_config.hpp"
#include "persist.hpp"
#include "plane.hpp"

using namespace wsfft;

namespace {

thread_local wsfft_status_t g_last_error = WSFFT_SUCCESS;

std::mutex g_plans_mu;
std::unordered_set<const wsfft_plan_s*> g_plans;

struct Pass {
    const PassKernel* kern_neg;   // kernel with sign -1
    const PassKernel* kern_pos;   // kernel with sign +1
    PassArgs args;                // src/dst/scale filled per call
    int src_sel, dst_sel;         // 0 = caller input, 1 = caller output, 2 = work buffer
    int src_sel_ip, dst_sel_ip;   // the same when the caller passes in == out
    int axis;
    int64_t n;
    bool strided;
    int four_step;                // 0 direct, 1 pass A, 2 pass B
    int64_t tw_off, tw4_off;      // element offsets into the twiddle block (tw4: -1 none)
    float pass_scale;             // 2^-s_p
    float inv_scale;              // the pass's scale in wsfft_execute_inverse
    int outer_dim;                // count whose stride spans whole arrays: 0 = C, 1 = O1, 2 = O2
    int variant;                  // kernel launch variant (autotuner)
    dim3 grid;
    bool plane = false;           // fused x + y pass over whole planes (n = nx, n2 = ny;
    int64_t n2 = 0;               // tw_off / tw4_off: the x / y stage tables)
    // plane chunks (Infinity Cache policy): C per xy-plane (0: O1 counts the
    // planes) and the bytes per plane of the source and destination
    int64_t chunk_c = 0;
    int64_t plane_in = 0, plane_out = 0;
};

bool is_smooth23(int64_t n) {
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

bool direct_ok(int64_t n, bool strided) {
    return strided ? n <= kMaxStridedN : n <= kMaxContigN;
}

// Split n into n1 * n2 with both passes' lengths in the strided size range,
// n1 as close to sqrt(n) as possible.  Returns false if impossible.
bool split_axis(int64_t n, int64_t* n1, int64_t* n2) {
    int64_t best = 0;
    for (int64_t d = 2; d * d <= n; ++d) {
        if (n % d) continue;
        const int64_t e = n / d;
        if (d <= kMaxStridedN && e <= kMaxStridedN) best = d;
    }
    if (!best) return false;
    *n1 = best;            // the smaller factor, <= sqrt(n)
    *n2 = n / best;
    return true;
}

// Round x to a binary format with `mant` stored significand bits and
// smallest normal exponent `emin`, nearest-even (subnormals included).
double round_to_format(double x, int mant, int emin) {
    if (x == 0.0) return 0.0;
    int e2;
    std::frexp(x, &e2);              // |x| in [2^(e2-1), 2^e2)
    const int lead = std::max(e2 - 1, emin);
    const double ulp = std::ldexp(1.0, lead - mant);
    return std::nearbyint(x / ulp) * ulp;
}

// exp(-2*pi*i*m/n) in FP64, reduced to the first octant by exact integer
// symmetry so that values on the axes and diagonals come out exact.
void root_fp64(int64_t m, int64_t n, double* re, double* im) {
    m %= n;
    // angle = (pi/2) * (q + r/n) with integer quadrant q and 0 <= r < n
    const int64_t u = 4 * m;
    const int64_t q = u / n;
    const int64_t r = u - q * n;
    double c, s;
    if (2 * r <= n) {
        const double phi = (M_PI / 2) * (double)r / (double)n;
        c = std::cos(phi);
        s = std::sin(phi);
    } else {
        const double phi = (M_PI / 2) * (double)(n - r) / (double)n;
        c = std::sin(phi);
        s = std::cos(phi);
    }
    if (r == 0) { c = 1.0; s = 0.0; }
    double cr, sr;   // rotate (c, s) by q quarter turns
    switch (q & 3) {
        case 0: cr = c; sr = s; break;
        case 1: cr = -s; sr = c; break;
        case 2: cr = -c; sr = -s; break;
        default: cr = s; sr = -c; break;
    }
    *re = cr;
    *im = -sr;   // forward kernel exp(-i*angle)
}

StorageKind kind_of(wsfft_dtype_t d, unsigned flags) {
    if (d == WSFFT_C64) return kC64;
    if (d == WSFFT_C16_BF16) return kBF16;
    return (flags & WSFFT_FLAG_FP16_MATH) ? kF16Math : kF16;
}

int elem_bytes(wsfft_dtype_t d) { return d == WSFFT_C64 ? 8 : 4; }

}  // namespace

struct wsfft_plan_s {
    int64_t n[3];
    wsfft_dtype_t dtype;
    int sign;
    unsigned flags;
    int device;
    int scale_log2;
    std::vector<Pass> passes;     // c2c plans: the transform; real plans: the R2C passes
    bool real = false;            // created by wsfft_plan_create_real(_ex)
    int64_t half_pitch = 0;       // real plans: complex values per half-spectrum row
    std::vector<Pass> cpasses;    // real plans: the C2R passes (the x pass last)
    int nsplit = 0;               // axes split into two passes (four-step)
    float2* tw_dev = nullptr;     // all twiddle tables, one block
    void* work = nullptr;         // four-step work buffer (or null)
    int64_t work_bytes = 0;
    // Infinity Cache policy of x, y, z plans (WSFFT_FLAG_STREAMING):
    // 0 streaming, 1 cached loads and stores, 2 cached x stores, 3 two passes
    // in plane chunks of chunk_planes planes: passes[chunk_at] and the next
    int cache_mode = 0;
    int64_t chunk_planes = 0;
    int chunk_at = -1;
    std::string desc;
};

namespace {

bool plan_live(const wsfft_plan_s* p) {
    if (!p) return false;
    std::lock_guard<std::mutex> g(g_plans_mu);
    return g_plans.count(p) != 0;
}

wsfft_plan_t fail(wsfft_status_t st) {
    g_last_error = st;
    return nullptr;
}

// Geometry of one axis: `inner` = product of faster axes, `outer` = slower.
struct AxisGeo {
    int axis;
    int64_t n, inner, outer;
};

void set_direct(Pass& P, const AxisGeo& g) {
    PassArgs& a = P.args;
    std::memset(&a, 0, sizeof a);
    a.M = 1;
    a.scale = 1.0f;
    a.O1 = a.O2 = 1;
    if (g.inner == 1) {            // contiguous pencils
        P.strided = false;
        P.outer_dim = 0;
        a.C = g.outer;
        a.es_in = a.es_out = 1;
        a.os1_in = a.os1_out = g.n;
        a.cs_out = 1;
    } else {
        P.strided = true;
        P.outer_dim = 1;
        a.C = g.inner;
        a.O1 = g.outer;
        a.es_in = a.es_out = g.inner;
        a.os1_in = a.os1_out = g.inner * g.n;
        a.cs_out = 1;
    }
}

// Pass A and pass B of a split axis, see the file comment.
void set_four_step(Pass& A, Pass& B, const AxisGeo& g, int64_t n1, int64_t n2) {
    const int64_t I = g.inner, n = g.n;
    for (Pass* P : {&A, &B}) {
        std::memset(&P->args, 0, sizeof P->args);
        P->args.scale = 1.0f;
        P->args.M = n;
        P->strided = true;
    }
    A.outer_dim = B.outer_dim = (I == 1) ? 1 : 2;
    PassArgs& a = A.args;
    if (I == 1) {
        // columns y2 (unit stride), elements y1 at stride n2; output of
        // column y2 is the contiguous run k1 + n1*y2.
        a.C = n2; a.O1 = g.outer; a.O2 = 1;
        a.es_in = n2; a.os1_in = n;
        a.es_out = 1; a.cs_out = n1; a.os1_out = n;
        a.tw4_mode = 1;
        a.tstore = 1;
    } else {
        // columns are the faster axes (unit stride); y2 is outer index 1.
        a.C = I; a.O1 = n2; a.O2 = g.outer;
        a.es_in = n2 * I; a.os1_in = I; a.os2_in = I * n;
        a.es_out = I; a.cs_out = 1; a.os1_out = n1 * I; a.os2_out = I * n;
        a.tw4_mode = 2;
    }
    PassArgs& b = B.args;
    if (I == 1) {
        b.C = n1; b.O1 = g.outer; b.O2 = 1;
        b.es_in = b.es_out = n1; b.os1_in = b.os1_out = n; b.cs_out = 1;
    } else {
        b.C = I; b.O1 = n1; b.O2 = g.outer;
        b.es_in = b.es_out = n1 * I;
        b.os1_in = b.os1_out = I;
        b.os2_in = b.os2_out = I * n;
        b.cs_out = 1;
    }
}

int64_t blocks_for(const Pass& P, const PassKernel* k) {
    const PassArgs& a = P.args;
    if (P.strided) return ((a.C + k->per_block - 1) / k->per_block) * a.O1 * a.O2;
    return (a.C + k->per_block - 1) / k->per_block;
}

const char* kind_name(wsfft_dtype_t d, unsigned flags) {
    if (d == WSFFT_C16_FP16 && (flags & WSFFT_FLAG_FP16_MATH)) return "c16-fp16-math";
    return d == WSFFT_C64 ? "c64" : (d == WSFFT_C16_FP16 ? "c16-fp16" : "c16-bf16");
}

void describe_passes(std::string& out, const std::vector<Pass>& passes) {
    char buf[256];
    for (const Pass& P : passes) {
        const int fu = P.kern_neg->fused;
        const char* what = fu == kFusedR2C      ? "r2c"
                           : fu == kFusedC2R    ? "c2r"
                           : fu == kFusedCached ? "cached-"
                           : fu == kFusedCachedStore ? "cached-store-"
                                                : "";
        if (P.plane) {
            std::snprintf(buf, sizeof buf, " xy[plane %lldx%lld wg=%d lds=%d grid=%u]", (long long)P.n, (long long)P.n2,
                          P.kern_neg->threads, P.kern_neg->lds_bytes, P.grid.x);
            out += buf;
            continue;
        }
        std::snprintf(buf, sizeof buf, " %c%s[%s%s n=%lld v%d wg=%d per=%d lds=%d grid=%u%s]", "xyz"[P.axis],
                      P.four_step == 1 ? "A" : (P.four_step == 2 ? "B" : ""), what, P.strided ? "strided" : "contig",
                      (long long)P.n, P.variant, P.kern_neg->threads, P.kern_neg->per_block, P.kern_neg->lds_bytes,
                      P.grid.x, P.args.flat_c ? (P.args.xcd_order ? " flat xcd" : " flat") : (P.args.xcd_order ? " xcd" : ""));
        out += buf;
    }
}

void describe_plan(wsfft_plan_s* plan) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "%lldx%lldx%lld %s sign=%d S=%d:", (long long)plan->n[0], (long long)plan->n[1],
                  (long long)plan->n[2], plan->real ? "real-c64" : kind_name(plan->dtype, plan->flags), plan->sign,
                  plan->scale_log2);
    plan->desc = buf;
    if (plan->real && plan->half_pitch != plan->n[0] / 2 + 1) {
        std::snprintf(buf, sizeof buf, " (half-spectrum rows %lld apart)", (long long)plan->half_pitch);
        plan->desc.insert(plan->desc.size() - 1, buf);
    }
    describe_passes(plan->desc, plan->passes);
    if (plan->chunk_planes > 0) {
        std::snprintf(buf, sizeof buf, " (x, y in chunks of %lld planes)", (long long)plan->chunk_planes);
        plan->desc += buf;
    }
    if (plan->real) {
        plan->desc += " | c2r:";
        describe_passes(plan->desc, plan->cpasses);
    }
}

// WSFFT_LOG=1: print every created plan's schedule (passes, kernels, tiles)
// to stderr.
void log_plan(const std::string& desc) {
    const char* e = std::getenv("WSFFT_LOG");
    if (e && std::strcmp(e, "1") == 0) std::fprintf(stderr, "wsfft: plan %s\n", desc.c_str());
}

// Twiddle tables of a plan, one per distinct (kind, length, n1), laid out
// back to back in one device block:
//  kStage: the stage tables of the radix plans 0, 1, 2 of a pass length,
//          len entries each (stage_tw_offset); a pass uses the block of its
//          kernel's plan;
//  kPlain: entry m is W_len^m (inter-pass twiddles of strided split axes);
//  kMatrix: entry m is W_len^{(m div n1) * (m mod n1)}, the inter-pass
//          twiddle of output position k1 + n1*y2 of pass A of a unit-stride
//          split axis, so lanes that store consecutive outputs read
//          consecutive entries;
//  kHalf: entry m is W_len^m for m = 0 .. len/4, the recombination twiddles
//          of the half-spectrum passes of a real axis of len points;
//  kPair64: two FP64 tables (each entry two slots, 16-byte aligned),
//          W_len^j for j < 2^s and then W_len^(j * 2^s) for j < ceil(len / 2^s),
//          s = pair64_shift(len): the inter-pass twiddles of pass A of a
//          unit-stride split axis of complex64 plans, which the kernel
//          multiplies out in FP64 and rounds once.
enum { kStage = 0, kPlain = 1, kMatrix = 2, kHalf = 3, kPair64 = 4 };
// the smallest s with 2^s >= sqrt(len): both tables hold about sqrt(len) entries
int pair64_shift(int64_t len) {
    int s = 0;
    while ((int64_t(1) << (2 * s)) < len) ++s;
    return s;
}
struct TableSet {
    struct Table { int kind; int64_t len, n1, off; };
    std::vector<Table> tables;
    int64_t total = 0;
    int64_t get(int kind, int64_t len, int64_t n1 = 0) {
        for (auto& t : tables)
            if (t.kind == kind && t.len == len && t.n1 == n1) return t.off;
        if (kind == kPair64 && total % 2 != 0) ++total;   // 16-byte alignment
        tables.push_back({kind, len, n1, total});
        if (kind == kPair64) {
            const int64_t L = int64_t(1) << pair64_shift(len);
            total += 2 * (L + (len + L - 1) / L);
        } else {
            total += kind == kStage ? kTwPlans * len : (kind == kHalf ? len / 4 + 1 : len);
        }
        return tables.back().off;
    }
};

// Evaluates every table of `ts` in FP64, rounds each entry once (nearest even)
// to a format of `mant` stored significand bits and smallest normal exponent
// `emin`, and copies the block to a new device allocation.
wsfft_status_t upload_tables(const TableSet& ts, int mant, int emin, float2** dev) {
    std::vector<float2> host((size_t)std::max<int64_t>(ts.total, 1));
    auto put = [&](int64_t at, int64_t m, int64_t len) {
        double re, im;
        root_fp64(m, len, &re, &im);
        host[(size_t)at] = make_float2((float)round_to_format(re, mant, emin), (float)round_to_format(im, mant, emin));
    };
    for (auto& t : ts.tables) {
        if (t.kind == kStage) {
            // entry (r-1)*Ns + k of stage s: W_{Ns*R}^{k*r} = W_len^{k*r*len/(Ns*R)}
            for (int pl = 0; pl < kTwPlans; ++pl) {
                const Radices rd = make_radices((int)t.len, pl);
                const int64_t base = t.off + (int64_t)pl * t.len;
                for (int st = 1; st < rd.n; ++st) {
                    const int64_t R = rd.r[st], Ns = stage_ns(rd, st), tws = t.len / (Ns * R);
                    const int64_t off = stage_tw_offset(rd, st);
                    for (int64_t r = 1; r < R; ++r)
                        for (int64_t k = 0; k < Ns; ++k) put(base + off + (r - 1) * Ns + k, k * r * tws, t.len);
                }
            }
        } else if (t.kind == kHalf) {
            for (int64_t m = 0; m <= t.len / 4; ++m) put(t.off + m, m, t.len);
        } else if (t.kind == kPair64) {
            // FP64 entries, not rounded to the storage format
            const int64_t L = int64_t(1) << pair64_shift(t.len), H = (t.len + L - 1) / L;
            auto put64 = [&](int64_t slot, int64_t m) {
                double v[2];
                root_fp64(m % t.len, t.len, &v[0], &v[1]);
                std::memcpy(&host[(size_t)(t.off + 2 * slot)], v, sizeof v);
            };
            for (int64_t j = 0; j < L; ++j) put64(j, j);
            for (int64_t j = 0; j < H; ++j) put64(L + j, j * L);
        } else {
            for (int64_t m = 0; m < t.len; ++m) put(t.off + m, t.n1 > 0 ? (m / t.n1) * (m % t.n1) : m, t.len);
        }
    }
    if (hipMalloc(dev, host.size() * sizeof(float2)) != hipSuccess) return WSFFT_ERROR_OUT_OF_MEMORY;
    if (hipMemcpy(*dev, host.data(), host.size() * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(*dev);
        *dev = nullptr;
        return WSFFT_ERROR_HIP;
    }
    return WSFFT_SUCCESS;
}

// ---- autotuner -------------------------------------------------------------------
// Each pass of a hot length has several compiled launch variants (radix plan,
// tile width).  When tuning is requested (WSFFT_FLAG_TUNE or WSFFT_TUNE=1)
// the choice per pass geometry is read from a cache file, or measured at plan
// creation with HIP events on scratch buffers and appended to the cache.
// Without a request the cache is read only if $WSFFT_TUNE_CACHE names it.
// WSFFT_TUNE=0 disables both.  Cache: $WSFFT_TUNE_CACHE, else
// $HOME/.cache/wsfft_tune.txt, one "key variant microseconds" line per entry.

std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;
bool g_tune_loaded = false;

std::string tune_cache_path() {
    const char* e = std::getenv("WSFFT_TUNE_CACHE");
    if (e && *e) return e;
    const char* h = std::getenv("HOME");
    return std::string(h && *h ? h : "/tmp") + "/.cache/wsfft_tune.txt";
}

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    std::ifstream f(tune_cache_path());
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream ls(line);
        std::string key;
        int v = -1;
        if (ls >> key >> v && v >= 0 && v < kMaxVariants) g_tune_cache[key] = v;
    }
}

void tune_store_locked(const std::string& key, int v, double us) {
    g_tune_cache[key] = v;
    const std::string path = tune_cache_path();
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) (void)mkdir(path.substr(0, slash).c_str(), 0755);
    std::ofstream f(path, std::ios::app);
    if (f) f << key << " " << v << " " << us << "\n";
}

std::string tune_key(const wsfft_plan_s* plan, const Pass& P, const char* arch) {
    const PassArgs& a = P.args;
    char buf[320];
    std::snprintf(buf, sizeof buf, "%s|%s|s%d|n%lld|st%d|fs%d|C%lld|O%lld,%lld|es%lld|os%lld,%lld", arch,
                  kind_name(plan->dtype, plan->flags), plan->sign, (long long)P.n, (int)P.strided, P.four_step,
                  (long long)a.C, (long long)a.O1, (long long)a.O2, (long long)a.es_in, (long long)a.os1_in,
                  (long long)a.os2_in);
    return buf;
}

// The stage twiddles of the radix plan of P's kernel (kStage table block).
void set_stage_tw(const wsfft_plan_s* plan, Pass& P) {
    P.args.tw = plan->tw_dev + P.tw_off + (int64_t)P.kern_neg->plan * P.n;
}

bool use_variant(wsfft_plan_s* plan, Pass& P, int v) {
    const StorageKind kind = kind_of(plan->dtype, plan->flags);
    const PassKernel* kn = find_pass_kernel(kind, -1, (int)P.n, P.strided, P.four_step == 1, v);
    const PassKernel* kp = find_pass_kernel(kind, +1, (int)P.n, P.strided, P.four_step == 1, v);
    if (!kn || !kp || kn->prepare() != hipSuccess || kp->prepare() != hipSuccess) return false;
    const int64_t blocks = blocks_for(P, kn);
    if (blocks < 1 || blocks * kn->threads > 0xffffffffLL) return false;
    P.kern_neg = kn;
    P.kern_pos = kp;
    P.variant = v;
    P.grid = dim3((unsigned)blocks);
    set_stage_tw(plan, P);
    return true;
}

// Median-free best-of timing: microseconds per launch of pass P with variant v.
double time_variant(wsfft_plan_s* plan, Pass& P, int v, void* buf0, void* buf1, hipStream_t st) {
    Pass Q = P;
    if (!use_variant(plan, Q, v)) return -1.0;
    const PassKernel* k = plan->sign < 0 ? Q.kern_neg : Q.kern_pos;
    PassArgs a = Q.args;
    a.src = Q.src_sel == 0 ? buf0 : buf1;
    a.dst = Q.dst_sel == 0 ? buf0 : buf1;
    a.scale = Q.pass_scale;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.0;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.0;
    }
    double best = -1.0;
    bool ok = true;
    for (int i = 0; i < 2 && ok; ++i) ok = k->launch(a, nullptr, Q.grid, st) == hipSuccess;
    for (int rep = 0; rep < 3 && ok; ++rep) {
        ok = hipEventRecord(e0, st) == hipSuccess;
        for (int i = 0; i < 3 && ok; ++i) ok = k->launch(a, nullptr, Q.grid, st) == hipSuccess;
        ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.f;
        if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
            const double us = 1000.0 * ms / 3;
            if (best < 0 || us < best) best = us;
        }
    }
    (void)hipStreamSynchronize(st);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ok ? best : -1.0;
}

void tune_plan(wsfft_plan_s* plan, bool requested) {
    const char* force = std::getenv("WSFFT_TUNE_FORCE");   // diagnostic: one variant everywhere
    if (force && *force) {
        const int v = std::atoi(force);
        for (Pass& P : plan->passes) {
            Pass Q = P;
            if (!P.plane && P.kern_neg->fused == 0 && v >= 0 && v < kMaxVariants && use_variant(plan, Q, v)) P = Q;
        }
        (void)hipGetLastError();
        return;
    }
    const char* env = std::getenv("WSFFT_TUNE");
    if (env && std::strcmp(env, "0") == 0) return;
    requested = requested || (env && std::strcmp(env, "1") == 0);
    // the cache is consulted only when tuning is requested or a cache file is
    // named explicitly, so a plan made without either depends on its
    // arguments alone, whatever earlier processes recorded
    const char* named = std::getenv("WSFFT_TUNE_CACHE");
    if (!requested && !(named && *named)) return;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, plan->device) != hipSuccess) return;
    const char* arch = prop.gcnArchName;
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_load_locked();
    void* buf0 = nullptr;
    void* buf1 = nullptr;
    hipStream_t st = nullptr;
    const int64_t bytes = plan->n[0] * plan->n[1] * plan->n[2] * elem_bytes(plan->dtype);
    for (Pass& P : plan->passes) {
        // one kernel per plane shape; passes of the Infinity Cache policy keep
        // their cached kernels
        if (P.plane || P.kern_neg->fused != 0) continue;
        const StorageKind kind = kind_of(plan->dtype, plan->flags);
        int nvar = 0;
        for (int v = 0; v < kMaxVariants; ++v)
            if (find_pass_kernel(kind, plan->sign, (int)P.n, P.strided, P.four_step == 1, v)) ++nvar;
        if (nvar < 2) continue;
        const std::string key = tune_key(plan, P, arch);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            Pass Q = P;
            if (use_variant(plan, Q, it->second)) P = Q;
            continue;
        }
        if (!requested) continue;
        if (!buf0) {
            if (hipMalloc(&buf0, (size_t)bytes) != hipSuccess) { buf0 = nullptr; break; }
            if (hipMalloc(&buf1, (size_t)bytes) != hipSuccess) { buf1 = nullptr; break; }
            if (hipMemset(buf0, 0, (size_t)bytes) != hipSuccess || hipMemset(buf1, 0, (size_t)bytes) != hipSuccess ||
                hipStreamCreate(&st) != hipSuccess) {
                st = nullptr;
                break;
            }
        }
        int best_v = -1;
        double best_us = 0.0;
        for (int v = 0; v < kMaxVariants; ++v) {
            if (!find_pass_kernel(kind, plan->sign, (int)P.n, P.strided, P.four_step == 1, v)) continue;
            const double us = time_variant(plan, P, v, buf0, buf1, st);
            if (us > 0 && (best_v < 0 || us < best_us)) {
                best_v = v;
                best_us = us;
            }
        }
        if (best_v >= 0) {
            Pass Q = P;
            if (use_variant(plan, Q, best_v)) {
                P = Q;
                tune_store_locked(key, best_v, best_us);
            }
        }
    }
    if (st) (void)hipStreamDestroy(st);
    if (buf0) (void)hipFree(buf0);
    if (buf1) (void)hipFree(buf1);
    (void)hipGetLastError();
}

}  // namespace

namespace {
// A C caller may pass any int for an enum parameter; its bits are read as an
// int (loading an out-of-range value as the C++ enum type would be undefined).
template <class E> int enum_bits(const E& e) {
    static_assert(sizeof(E) == sizeof(int), "C enums are int-sized");
    int v;
    std::memcpy(&v, &e, sizeof v);
    return v;
}

}  // namespace

extern "C" {

const char* wsfft_status_string(wsfft_status_t st_in) {
    const int st = enum_bits(st_in);
    switch (st) {
        case WSFFT_SUCCESS: return "success";
        case WSFFT_ERROR_INVALID_VALUE: return "invalid value";
        case WSFFT_ERROR_UNSUPPORTED_SIZE: return "unsupported size";
        case WSFFT_ERROR_NULL_POINTER: return "null pointer";
        case WSFFT_ERROR_MISALIGNED: return "misaligned pointer";
        case WSFFT_ERROR_OUT_OF_MEMORY: return "out of device memory";
        case WSFFT_ERROR_NO_DEVICE: return "no HIP device";
        case WSFFT_ERROR_HIP: return "HIP runtime error";
        case WSFFT_ERROR_INVALID_PLAN: return "invalid plan";
        case WSFFT_ERROR_WRONG_DEVICE: return "current device is not the plan's device";
        case WSFFT_ERROR_EXCEEDS_SCRATCH: return "work exceeds the library's static scratch buffer";
    }
    return "unknown status";
}

wsfft_status_t wsfft_get_last_error(void) { return g_last_error; }

}  // extern "C"

namespace {
// Infinity Cache policy of a plan of three single passes x, y, z (see
// WSFFT_FLAG_STREAMING).  Measured on MI355X with complex64, by array size A:
//  * A <= 64 MiB: streaming throughout (16 MiB ties; at 32-64 MiB cached
//    passes win on 256 x 256 planes and lose on 512 x 512 ones);
//  * 64 MiB < A <= 128 MiB: every pass with cached loads and stores, so each
//    pass reads what the previous one left in the 256 MB Infinity Cache
//    (256^3: 136.6 us per transform against 154.8 streaming);
//  * 128 MiB < A <= 256 MiB: cached x stores only (512 x 512 x 128, x and y
//    passes: 176 against 194.5 us; caching every pass there: 212 us);
//  * A > 256 MiB: the x and y passes chunk by chunk over groups of planes of
//    at most 256 MiB, the x pass of a chunk with cached stores so that its y
//    pass reads the chunk from the cache (512^3: 4 chunks, 1107 against
//    1146 us; 1024^3: 32 chunks, 10.37 against 11.13 ms); chunks of a larger
//    share of the cache, or streaming x stores, lose it again.
// The 16-bit storage types have cached-store x kernels only (no cached
// loads), so they take the last two rules.  The cached kernels have the
// launch geometry of the default ones, so the results are bitwise equal and
// the grids unchanged.
bool use_cached(Pass& P, StorageKind kind, int fused) {
    const PassKernel* kn = find_cached_kernel(kind, -1, (int)P.n, P.strided, fused);
    const PassKernel* kp = find_cached_kernel(kind, +1, (int)P.n, P.strided, fused);
    if (!kn || !kp || kn->per_block != P.kern_neg->per_block || kn->threads != P.kern_neg->threads) return false;
    P.kern_neg = kn;
    P.kern_pos = kp;
    return true;
}

void apply_cache_policy(wsfft_plan_s* plan) {
    auto& ps = plan->passes;
    const int64_t nx = plan->n[0], ny = plan->n[1], nz = plan->n[2];
    const StorageKind kind = kind_of(plan->dtype, plan->flags);
    if (ps.size() != 3 || nz < 2) return;
    for (int i = 0; i < 3; ++i)
        if (ps[i].plane || ps[i].four_step != 0 || ps[i].axis != i || ps[i].strided != (i > 0)) return;
    constexpr int64_t kMiB = int64_t(1) << 20, kCache = 256 * kMiB;
    const int64_t plane = nx * ny * elem_bytes(plan->dtype), A = plane * nz;
    if (A <= 64 * kMiB) return;
    if (A <= 128 * kMiB) {
        Pass q[3] = {ps[0], ps[1], ps[2]};
        for (Pass& P : q)
            if (!use_cached(P, kind, kFusedCached)) return;
        for (int i = 0; i < 3; ++i) ps[i] = q[i];
        plan->cache_mode = 1;
        return;
    }
    if (A <= kCache) {
        if (use_cached(ps[0], kind, kFusedCachedStore)) plan->cache_mode = 2;
        return;
    }
    // the largest group of planes dividing nz that fits the cache; at most
    // 64 chunks
    int64_t zc = 0;
    for (int64_t z = nz - 1; z >= 1 && zc == 0; --z)
        if (nz % z == 0 && z * plane <= kCache) zc = z;
    if (zc == 0 || nz / zc > 64) return;
    if (!use_cached(ps[0], kind, kFusedCachedStore)) return;
    plan->cache_mode = 3;
    plan->chunk_planes = zc;
    plan->chunk_at = 0;
    ps[0].chunk_c = ny;                    // x: ny pencils per plane
    ps[1].chunk_c = 0;                     // y: planes are its outer index
    for (int i = 0; i < 2; ++i) ps[i].plane_in = ps[i].plane_out = plane;
}
}  // namespace

static wsfft_plan_t plan_create(int64_t nx, int64_t ny, int64_t nz, int dt, int sign, unsigned flags) {
    // ---- argument checks, no device calls -------------------------------
    if (nx < 1 || ny < 1 || nz < 1) return fail(WSFFT_ERROR_INVALID_VALUE);
    if (sign != 1 && sign != -1) return fail(WSFFT_ERROR_INVALID_VALUE);
    if (dt != WSFFT_C64 && dt != WSFFT_C16_FP16 && dt != WSFFT_C16_BF16) return fail(WSFFT_ERROR_INVALID_VALUE);
    const wsfft_dtype_t dtype = static_cast<wsfft_dtype_t>(dt);
    if (flags & ~(WSFFT_FLAG_FP32_TWIDDLES | WSFFT_FLAG_TUNE | WSFFT_FLAG_FP16_MATH | WSFFT_FLAG_NO_PLANE |
                  WSFFT_FLAG_STREAMING))
        return fail(WSFFT_ERROR_INVALID_VALUE);
    if ((flags & WSFFT_FLAG_FP16_MATH) && dtype != WSFFT_C16_FP16) return fail(WSFFT_ERROR_INVALID_VALUE);
    const int64_t dims[3] = {nx, ny, nz};
    for (int64_t d : dims)
        if (d > WSFFT_MAX_AXIS || !is_smooth23(d)) return fail(WSFFT_ERROR_UNSUPPORTED_SIZE);
    if (nx * ny > (int64_t(1) << 40) || nx * ny * nz > (int64_t(1) << 40))
        return fail(WSFFT_ERROR_UNSUPPORTED_SIZE);

    wsfft_plan_s* plan = new (std::nothrow) wsfft_plan_s();
    if (!plan) return fail(WSFFT_ERROR_OUT_OF_MEMORY);
    plan->n[0] = nx; plan->n[1] = ny; plan->n[2] = nz;
    plan->dtype = dtype;
    plan->sign = sign;
    plan->flags = flags;

    // ---- schedule --------------------------------------------------------
    const bool half = dtype != WSFFT_C64;
    std::vector<AxisGeo> direct, split;
    const AxisGeo geos[3] = {{0, nx, 1, ny * nz}, {1, ny, nx, nz}, {2, nz, nx * ny, 1}};
    for (const AxisGeo& g : geos) {
        if (g.n == 1) continue;
        if (direct_ok(g.n, g.inner != 1)) direct.push_back(g);
        else split.push_back(g);
    }
    std::vector<AxisGeo> order = split;   // split axes first: pass A reads the input
    order.insert(order.end(), direct.begin(), direct.end());

    TableSet ts;
    auto table_for = [&](int kind, int64_t len, int64_t n1 = 0) { return ts.get(kind, len, n1); };

    const StorageKind kind = kind_of(dtype, flags);
    int S = 0;
    // complex64 arrays whose x and y axes are both one pass and whose
    // xy-plane fits in LDS fuse the two into one plane pass (plane.hip)
    const bool plane = kind == kC64 && !(flags & WSFFT_FLAG_NO_PLANE) && nx > 1 && ny > 1 &&
                       direct_ok(nx, false) && direct_ok(ny, true) && find_plane_kernel((int)nx, (int)ny, -1) &&
                       find_plane_kernel((int)nx, (int)ny, +1);
    for (const AxisGeo& g : order) {
        const bool is_split = !direct_ok(g.n, g.inner != 1);
        const int sp = half ? (int)std::ceil(std::log2((double)g.n) / 2.0) : 0;
        S += sp;
        if (plane && g.axis == 1) continue;   // done by the plane pass
        if (plane && g.axis == 0) {
            Pass P{};
            set_direct(P, g);
            PassArgs& a = P.args;
            a.C = nz;                         // planes of nx * ny values
            a.es_in = a.es_out = 1;
            a.os1_in = a.os1_out = nx * ny;
            P.axis = 0; P.n = nx; P.n2 = ny; P.plane = true; P.four_step = 0;
            P.strided = false;
            P.outer_dim = 0;
            P.tw_off = table_for(kStage, nx);
            P.tw4_off = table_for(kStage, ny);
            P.pass_scale = 1.0f;
            plan->passes.push_back(P);
            continue;
        }
        if (!is_split) {
            Pass P{};
            set_direct(P, g);
            P.axis = g.axis; P.n = g.n; P.four_step = 0;
            P.tw_off = table_for(kStage, g.n); P.tw4_off = -1;
            P.pass_scale = std::ldexp(1.0f, -sp);
            // 16-bit storage with FP32 arithmetic, y axis (128-byte rows of
            // one plane): tiles that share DRAM pages meet in one XCD
            // (512^3: 234 -> 220 us; the z axis runs slower that way)
            if (g.axis == 1 && P.strided && half && !(flags & WSFFT_FLAG_FP16_MATH)) P.args.xcd_order = 1;
            plan->passes.push_back(P);
        } else {
            int64_t n1, n2;
            if (!split_axis(g.n, &n1, &n2)) { delete plan; return fail(WSFFT_ERROR_UNSUPPORTED_SIZE); }
            Pass A{}, B{};
            set_four_step(A, B, g, n1, n2);
            A.axis = B.axis = g.axis;
            A.n = n1; B.n = n2;
            A.four_step = 1; B.four_step = 2;
            A.tw_off = table_for(kStage, n1); B.tw_off = table_for(kStage, n2);
            if (A.args.tw4_mode == 1 && kind == kC64) {
                A.tw4_off = table_for(kPair64, g.n);
                A.args.tw4_shift = pair64_shift(g.n);
            } else {
                A.tw4_off = A.args.tw4_mode == 1 ? table_for(kMatrix, g.n, n1) : table_for(kPlain, g.n);
            }
            B.tw4_off = -1;
            // the axis scale 2^-sp is split between the two passes
            const int sa = sp / 2, sb = sp - sa;
            A.pass_scale = std::ldexp(1.0f, -sa);
            B.pass_scale = std::ldexp(1.0f, -sb);
            plan->passes.push_back(A);
            plan->passes.push_back(B);
        }
    }
    plan->scale_log2 = S;
    // wsfft_execute_inverse: complex64 plans fold 1/N into the last pass; the
    // 16-bit plans scale pass p by 2^s_p / n_p, about 1/sqrt(n_p) like the
    // forward 2^-s_p, so the inverse is 2^S/N times the opposite-sign sum
    // (the exact inverse of wsfft_execute) and stays within the FP16 range
    {
        const double N = (double)nx * (double)ny * (double)nz;
        for (Pass& P : plan->passes)
            P.inv_scale = half ? (float)(1.0 / ((double)P.pass_scale * (double)P.n)) : P.pass_scale;
        if (!half && !plan->passes.empty()) plan->passes.back().inv_scale = (float)((double)plan->passes.back().pass_scale / N);
    }

    // kernels
    for (Pass& P : plan->passes) {
        if (P.plane) {
            P.kern_neg = find_plane_kernel((int)P.n, (int)P.n2, -1);
            P.kern_pos = find_plane_kernel((int)P.n, (int)P.n2, +1);
        } else {
            P.kern_neg = find_pass_kernel(kind, -1, (int)P.n, P.strided, P.four_step == 1);
            P.kern_pos = find_pass_kernel(kind, +1, (int)P.n, P.strided, P.four_step == 1);
        }
        if (!P.kern_neg || !P.kern_pos) { delete plan; return fail(WSFFT_ERROR_UNSUPPORTED_SIZE); }
        // one grid dimension holds at most 2^32 - 1 work-items
        const int64_t blocks = blocks_for(P, P.kern_neg);
        if (blocks < 1 || blocks * P.kern_neg->threads > 0xffffffffLL) {
            delete plan;
            return fail(WSFFT_ERROR_UNSUPPORTED_SIZE);
        }
        P.grid = dim3((unsigned)blocks);
    }
    if (!(flags & WSFFT_FLAG_STREAMING)) apply_cache_policy(plan);

    // buffers: split passes read the caller's input (first) or, for a
    // second split axis, the work buffer
    int nsplit = 0;
    for (size_t i = 0; i < plan->passes.size(); ++i) {
        Pass& P = plan->passes[i];
        if (i == 0) { P.src_sel = 0; P.dst_sel = 1; }
        else { P.src_sel = 1; P.dst_sel = 1; }
        if (P.four_step == 1) {
            if (nsplit > 0) { P.src_sel = 1; P.dst_sel = 2; }
            ++nsplit;
        } else if (P.four_step == 2 && nsplit > 1) {
            P.src_sel = 2; P.dst_sel = 1;
        }
    }
    // In-place calls: the first split axis goes through the work buffer too
    // (its pass A reads the whole input before any of it may be overwritten).
    for (size_t i = 0; i < plan->passes.size(); ++i) {
        Pass& P = plan->passes[i];
        P.src_sel_ip = P.src_sel;
        P.dst_sel_ip = P.dst_sel;
        if (nsplit > 0 && i == 0 && P.four_step == 1) P.dst_sel_ip = 2;
        if (nsplit > 0 && i == 1 && P.four_step == 2) P.src_sel_ip = 2;
    }
    plan->nsplit = nsplit;
    const int64_t N = nx * ny * nz;
    if (nsplit > 0) plan->work_bytes = N * elem_bytes(dtype);

    // ---- device ------------------------------------------------------------
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) { delete plan; return fail(WSFFT_ERROR_NO_DEVICE); }
    if (hipGetDevice(&plan->device) != hipSuccess) { delete plan; return fail(WSFFT_ERROR_HIP); }

    // twiddles in FP64, rounded once to the table precision
    const bool tw32 = !half || (flags & WSFFT_FLAG_FP32_TWIDDLES);
    const int mant = tw32 ? 23 : (dtype == WSFFT_C16_FP16 ? 10 : 7);
    const int emin = tw32 ? -126 : (dtype == WSFFT_C16_FP16 ? -14 : -126);
    {
        const wsfft_status_t st = upload_tables(ts, mant, emin, &plan->tw_dev);
        if (st != WSFFT_SUCCESS) {
            delete plan;
            return fail(st);
        }
    }
    if (plan->work_bytes > 0 && hipMalloc(&plan->work, (size_t)plan->work_bytes) != hipSuccess) {
        (void)hipFree(plan->tw_dev);
        delete plan;
        return fail(WSFFT_ERROR_OUT_OF_MEMORY);
    }
    for (Pass& P : plan->passes) {
        set_stage_tw(plan, P);
        P.args.tw4 = P.tw4_off >= 0 ? plan->tw_dev + P.tw4_off : nullptr;
        // the plane pass's y stage table: the block of its kernel's radix plan
        if (P.plane) P.args.tw4 += (int64_t)P.kern_neg->plan * P.n2;
        if (P.kern_neg->prepare() != hipSuccess || P.kern_pos->prepare() != hipSuccess) {
            (void)hipFree(plan->tw_dev);
            if (plan->work) (void)hipFree(plan->work);
            delete plan;
            return fail(WSFFT_ERROR_HIP);
        }
    }
    tune_plan(plan, (flags & WSFFT_FLAG_TUNE) != 0);
    describe_plan(plan);
    log_plan(plan->desc);
    {
        std::lock_guard<std::mutex> g(g_plans_mu);
        g_plans.insert(plan);
    }
    g_last_error = WSFFT_SUCCESS;
    return plan;
}

extern "C" {

wsfft_plan_t wsfft_plan_create_ex(int64_t nx, int64_t ny, int64_t nz, wsfft_dtype_t dtype, int sign,
                                  unsigned flags) {
    return plan_create(nx, ny, nz, enum_bits(dtype), sign, flags);
}

wsfft_plan_t wsfft_plan_create(int64_t nx, int64_t ny, int64_t nz, wsfft_dtype_t dtype, int sign) {
    return plan_create(nx, ny, nz, enum_bits(dtype), sign, 0u);
}

// Real plans.  The forward transform of a real nx x ny x nz array keeps the
// bins kx = 0 .. nx/2 (the rest follow by Hermitian symmetry): an x pass of
// N = nx/2 complex points over the reals read in pairs, whose epilogue
// recombines the even and odd halves into the N + 1 bins, then c2c passes
// along y and z over the half spectrum (nx/2 + 1) x ny x nz.  The C2R
// transform runs the z and y passes first, in place on its input, and the x
// pass last, whose prologue undoes the recombination.
wsfft_plan_t wsfft_plan_create_real(int64_t nx, int64_t ny, int64_t nz, unsigned flags) {
    return wsfft_plan_create_real_ex(nx, ny, nz, flags, 0);
}

wsfft_plan_t wsfft_plan_create_real_ex(int64_t nx, int64_t ny, int64_t nz, unsigned flags, int64_t half_pitch) {
    if (nx < 1 || ny < 1 || nz < 1) return fail(WSFFT_ERROR_INVALID_VALUE);
    if (flags != 0u) return fail(WSFFT_ERROR_INVALID_VALUE);
    if (half_pitch != 0 && (nx < 2 || half_pitch < nx / 2 + 1 || half_pitch > WSFFT_MAX_AXIS))
        return fail(WSFFT_ERROR_INVALID_VALUE);
    const int64_t dims[3] = {nx, ny, nz};
    for (int64_t d : dims)
        if (d > WSFFT_MAX_AXIS || !is_smooth23(d)) return fail(WSFFT_ERROR_UNSUPPORTED_SIZE);
    if (nx % 2 != 0 || nx < 4 || nx / 2 > kMaxContigN) return fail(WSFFT_ERROR_UNSUPPORTED_SIZE);
    if (nx * ny > (int64_t(1) << 40) || nx * ny * nz > (int64_t(1) << 40)) return fail(WSFFT_ERROR_UNSUPPORTED_SIZE);

    wsfft_plan_s* plan = new (std::nothrow) wsfft_plan_s();
    if (!plan) return fail(WSFFT_ERROR_OUT_OF_MEMORY);
    plan->n[0] = nx; plan->n[1] = ny; plan->n[2] = nz;
    plan->dtype = WSFFT_C64;
    plan->sign = -1;
    plan->flags = flags;
    plan->real = true;
    const int64_t N = nx / 2, nxh = N + 1;
    // half-spectrum row pitch; rows of whole 128-byte lines are aligned
    const int64_t hp = half_pitch != 0 ? half_pitch : nxh;
    const bool aligned = hp % 16 == 0;
    plan->half_pitch = hp;
    TableSet ts;

    // the x pass, both directions
    Pass X{};
    std::memset(&X.args, 0, sizeof X.args);
    X.args.M = 1;
    X.args.scale = 1.0f;
    X.args.O1 = X.args.O2 = 1;
    X.args.C = ny * nz;
    X.args.es_in = X.args.es_out = 1;
    X.args.cs_out = 1;
    X.strided = false;
    X.outer_dim = 0;
    X.axis = 0;
    X.n = N;
    X.four_step = 0;
    X.tw_off = ts.get(kStage, N);
    X.tw4_off = ts.get(kHalf, nx);
    X.pass_scale = X.inv_scale = 1.0f;
    Pass XR = X, XC = X;
    XR.args.os1_in = N;            // 2N reals as N complex
    XR.args.os1_out = hp;
    // cached stores: the last line of each row is written in part, whatever
    // the pitch, and streaming partial-line writes cost twice the time
    XR.kern_neg = XR.kern_pos = find_real_c64_neg((int)N, false, kFusedR2C);
    XC.args.os1_in = hp;
    XC.args.os1_out = N;
    XC.kern_neg = XC.kern_pos = find_real_c64_pos((int)N, false, kFusedC2R);
    if (!XR.kern_neg || !XC.kern_neg) { delete plan; return fail(WSFFT_ERROR_UNSUPPORTED_SIZE); }

    // the y and z passes over the half spectrum, per axis: one direct pass or
    // a four-step pair
    std::vector<std::vector<Pass>> axes;
    const AxisGeo geos[2] = {{1, ny, hp, nz}, {2, nz, hp * ny, 1}};
    for (const AxisGeo& g : geos) {
        if (g.n == 1) continue;
        std::vector<Pass> ps;
        if (direct_ok(g.n, true)) {
            Pass P{};
            set_direct(P, g);
            P.axis = g.axis; P.n = g.n; P.four_step = 0;
            P.tw_off = ts.get(kStage, g.n); P.tw4_off = -1;
            // with padded rows the y and z passes transform whole rows (hp
            // columns): line-aligned tiles, the padding columns transformed
            // along with the spectrum
            ps.push_back(P);
        } else {
            int64_t n1, n2;
            if (!split_axis(g.n, &n1, &n2)) { delete plan; return fail(WSFFT_ERROR_UNSUPPORTED_SIZE); }
            Pass A{}, B{};
            set_four_step(A, B, g, n1, n2);
            A.axis = B.axis = g.axis;
            A.n = n1; B.n = n2;
            A.four_step = 1; B.four_step = 2;
            A.tw_off = ts.get(kStage, n1); B.tw_off = ts.get(kStage, n2);
            A.tw4_off = ts.get(kPlain, g.n);
            B.tw4_off = -1;
            ps.push_back(A);
            ps.push_back(B);
            ++plan->nsplit;
        }
        // compact rows of the half spectrum are (nx/2 + 1) * 8 bytes apart,
        // not cache-line aligned: a direct y pass reads and writes through the
        // caches and each XCD takes a contiguous range of tiles, so tiles that
        // share lines meet in one L2 (512^3: 238 against 418 us streaming).
        // Rows padded to whole lines stream (faster there than the cached
        // pass: 638 against 668 us per R2C + C2R transform at pitch 272).
        const bool misaligned = g.axis == 1 && !aligned;
        for (Pass& P : ps) {
            P.pass_scale = P.inv_scale = 1.0f;
            if (misaligned && P.four_step == 0) {
                P.kern_neg = find_cached_c64_neg((int)P.n, true, kFusedCached);
                P.kern_pos = find_cached_c64_pos((int)P.n, true, kFusedCached);
                P.args.xcd_order = 1;
            } else {
                P.kern_neg = find_pass_kernel(kC64, -1, (int)P.n, true, P.four_step == 1);
                P.kern_pos = find_pass_kernel(kC64, +1, (int)P.n, true, P.four_step == 1);
            }
            if (!P.kern_neg || !P.kern_pos) { delete plan; return fail(WSFFT_ERROR_UNSUPPORTED_SIZE); }
            // a direct pass whose columns leave a ragged tile at every outer
            // index runs its tiles on across the outer indices instead
            PassArgs& a = P.args;
            if (P.four_step == 0 && a.O1 > 1 && a.O2 == 1 && a.C % P.kern_neg->per_block != 0) {
                a.flat_c = a.C;
                a.C *= a.O1;
                a.O1 = 1;
            }
        }
        axes.push_back(ps);
    }
    // R2C: x (input -> output), then y, z in place on the output (a split
    // axis through the work buffer); C2R: z, y in place on the input, then x
    // (input -> output)
    XR.src_sel = 0; XR.dst_sel = 1;
    plan->passes.push_back(XR);
    for (auto& ps : axes)
        for (Pass P : ps) {
            P.src_sel = P.four_step == 2 ? 2 : 1;
            P.dst_sel = P.four_step == 1 ? 2 : 1;
            plan->passes.push_back(P);
        }
    for (auto it = axes.rbegin(); it != axes.rend(); ++it)
        for (Pass P : *it) {
            P.src_sel = P.four_step == 2 ? 2 : 0;
            P.dst_sel = P.four_step == 1 ? 2 : 0;
            plan->cpasses.push_back(P);
        }
    XC.src_sel = 0; XC.dst_sel = 1;
    plan->cpasses.push_back(XC);
    // wsfft_execute_c2r_inverse: 1/N in the last pass
    plan->cpasses.back().inv_scale = (float)(1.0 / ((double)nx * (double)ny * (double)nz));
    for (auto* list : {&plan->passes, &plan->cpasses})
        for (Pass& P : *list) {
            P.src_sel_ip = P.src_sel;
            P.dst_sel_ip = P.dst_sel;
            const int64_t blocks = blocks_for(P, P.kern_neg);
            if (blocks < 1 || blocks * P.kern_neg->threads > 0xffffffffLL) {
                delete plan;
                return fail(WSFFT_ERROR_UNSUPPORTED_SIZE);
            }
            P.grid = dim3((unsigned)blocks);
        }
    if (plan->nsplit > 0) plan->work_bytes = hp * ny * nz * 8;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) { delete plan; return fail(WSFFT_ERROR_NO_DEVICE); }
    if (hipGetDevice(&plan->device) != hipSuccess) { delete plan; return fail(WSFFT_ERROR_HIP); }
    {
        const wsfft_status_t st = upload_tables(ts, 23, -126, &plan->tw_dev);
        if (st != WSFFT_SUCCESS) {
            delete plan;
            return fail(st);
        }
    }
    if (plan->work_bytes > 0 && hipMalloc(&plan->work, (size_t)plan->work_bytes) != hipSuccess) {
        (void)hipFree(plan->tw_dev);
        delete plan;
        return fail(WSFFT_ERROR_OUT_OF_MEMORY);
    }
    for (auto* list : {&plan->passes, &plan->cpasses})
        for (Pass& P : *list) {
            set_stage_tw(plan, P);
            P.args.tw4 = P.tw4_off >= 0 ? plan->tw_dev + P.tw4_off : nullptr;
            if (P.kern_neg->prepare() != hipSuccess || P.kern_pos->prepare() != hipSuccess) {
                (void)hipFree(plan->tw_dev);
                if (plan->work) (void)hipFree(plan->work);
                delete plan;
                return fail(WSFFT_ERROR_HIP);
            }
        }
    describe_plan(plan);
    log_plan(plan->desc);
    {
        std::lock_guard<std::mutex> g(g_plans_mu);
        g_plans.insert(plan);
    }
    g_last_error = WSFFT_SUCCESS;
    return plan;
}

int wsfft_plan_scale_log2(wsfft_plan_t plan) { return plan_live(plan) ? plan->scale_log2 : -1; }

int wsfft_plan_num_passes(wsfft_plan_t plan) { return plan_live(plan) ? (int)plan->passes.size() : -1; }

int64_t wsfft_plan_work_bytes(wsfft_plan_t plan) { return plan_live(plan) ? plan->work_bytes : -1; }

wsfft_status_t wsfft_plan_describe(wsfft_plan_t plan, char* buf, size_t len) {
    if (!plan_live(plan)) return WSFFT_ERROR_INVALID_PLAN;
    if (!buf) return WSFFT_ERROR_NULL_POINTER;
    if (len == 0) return WSFFT_ERROR_INVALID_VALUE;
    std::snprintf(buf, len, "%s", plan->desc.c_str());
    return WSFFT_SUCCESS;
}

void wsfft_plan_destroy(wsfft_plan_t plan) {
    if (!plan) return;
    {
        std::lock_guard<std::mutex> g(g_plans_mu);
        if (!g_plans.erase(plan)) return;   // unknown or already destroyed
    }
    int cur = -1;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(plan->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(plan->tw_dev);
    if (plan->work) (void)hipFree(plan->work);
    if (cur >= 0) (void)hipSetDevice(cur);
    delete plan;
}

}  // extern "C"

// ---- execution -----------------------------------------------------------
namespace {

// mode: 0 = plan sign, 1 = opposite sign (adjoint), 2 = opposite sign / N
wsfft_status_t check_exec(const wsfft_plan_s* plan, const void* in, const void* out) {
    if (!plan_live(plan)) return WSFFT_ERROR_INVALID_PLAN;
    if (plan->real) return WSFFT_ERROR_INVALID_VALUE;   // real plans run wsfft_execute_r2c / _c2r
    if (!in || !out) return WSFFT_ERROR_NULL_POINTER;
    const uintptr_t al = (uintptr_t)elem_bytes(plan->dtype);
    if (((uintptr_t)in % al) || ((uintptr_t)out % al)) return WSFFT_ERROR_MISALIGNED;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return WSFFT_ERROR_HIP;
    if (cur != plan->device) return WSFFT_ERROR_WRONG_DEVICE;
    return WSFFT_SUCCESS;
}

// Whether a call on these buffers goes through the plan's work buffer: always
// with two split axes, and in place with one.
bool uses_work(const wsfft_plan_s* plan, const void* in, const void* out) {
    return plan->nsplit > 1 || (plan->nsplit == 1 && in == out);
}

// Arguments of a call on a real plan: in and out disjoint (identity checked),
// aligned to their element sizes (real FP32: 4 bytes, complex64: 8).
wsfft_status_t check_real(const wsfft_plan_s* plan, const void* in, const void* out, uintptr_t in_al,
                          uintptr_t out_al) {
    if (!plan_live(plan)) return WSFFT_ERROR_INVALID_PLAN;
    if (!plan->real) return WSFFT_ERROR_INVALID_VALUE;
    if (!in || !out) return WSFFT_ERROR_NULL_POINTER;
    if (((uintptr_t)in % in_al) || ((uintptr_t)out % out_al)) return WSFFT_ERROR_MISALIGNED;
    if (in == out) return WSFFT_ERROR_INVALID_VALUE;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return WSFFT_ERROR_HIP;
    if (cur != plan->device) return WSFFT_ERROR_WRONG_DEVICE;
    return WSFFT_SUCCESS;
}

// Enqueue pass index `pi` of a plan; returns false on a launch error.  Real
// plans: the R2C passes in mode 0, the C2R passes otherwise.
// With zc > 0, only planes [z0, z0 + zc) of the x or y pass (a plane chunk).
bool launch_pass(const wsfft_plan_s* plan, size_t pi, const void* in, void* out, int mode,
                 hipStream_t stream, int64_t batch = 1, int64_t z0 = 0, int64_t zc = 0) {
    const Pass& P = (plan->real && mode != 0) ? plan->cpasses[pi] : plan->passes[pi];
    PassArgs a = P.args;
    dim3 grid = P.grid;
    int64_t in_off = 0, out_off = 0;   // bytes
    if (zc > 0) {
        const int64_t per = P.kern_neg->per_block;
        if (P.chunk_c > 0) a.C = P.chunk_c * zc;   // C counts the planes' pencils or columns
        else a.O1 = zc;                           // the outer index counts planes
        const int64_t blocks = P.strided ? ((a.C + per - 1) / per) * a.O1 * a.O2 : (a.C + per - 1) / per;
        grid = dim3((unsigned)blocks);
        in_off = z0 * P.plane_in;
        out_off = z0 * P.plane_out;
    }
    if (batch > 1) {   // `batch` arrays back to back: one more factor on the outermost count
        int64_t blocks;
        const int64_t per = P.kern_neg->per_block;
        if (P.outer_dim == 0) a.C *= batch;
        else if (P.outer_dim == 1) a.O1 *= batch;
        else a.O2 *= batch;
        if (P.strided) blocks = ((a.C + per - 1) / per) * a.O1 * a.O2;
        else blocks = (a.C + per - 1) / per;
        if (blocks * P.kern_neg->threads > 0xffffffffLL) return false;
        grid = dim3((unsigned)blocks);
    }
    auto sel = [&](int s) -> void* {
        return s == 0 ? const_cast<void*>(in) : (s == 1 ? out : plan->work);
    };
    const bool ip = in == out;
    a.src = static_cast<const char*>(sel(ip ? P.src_sel_ip : P.src_sel)) + in_off;
    a.dst = static_cast<char*>(sel(ip ? P.dst_sel_ip : P.dst_sel)) + out_off;
    a.scale = mode == 2 ? P.inv_scale : P.pass_scale;
    const int sign = mode == 0 ? plan->sign : -plan->sign;
    const PassKernel* k = sign < 0 ? P.kern_neg : P.kern_pos;
    return k->launch(a, nullptr, grid, stream) == hipSuccess;
}

// A kernel's function attributes (its dynamic LDS limit), set once per kernel
// and device: the batched paths look kernels up on every call.
bool prepared(const PassKernel* k) {
    static std::mutex mu;
    static std::set<std::pair<int, const PassKernel*>> done;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> lk(mu);
    if (done.count({dev, k})) return true;
    if (k->prepare() != hipSuccess) return false;
    done.insert({dev, k});
    return true;
}

// Launch variants chosen for whole merged launches by wsfft_tune_batched,
// keyed by the launch's identity (kernel shape, storage, sign, twiddle
// precision and every member's geometry).
std::mutex g_batch_tune_mu;
std::map<std::string, int> g_batch_tune;

// Microseconds of the best of three runs of three launches of `launch`
// (after two warm-up launches), or -1 on a launch error.
template <class F> double time_launches(F&& launch, hipStream_t st) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.0;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.0;
    }
    double best = -1.0;
    bool ok = launch() && launch();
    for (int rep = 0; rep < 3 && ok; ++rep) {
        ok = hipEventRecord(e0, st) == hipSuccess;
        for (int i = 0; i < 3 && ok; ++i) ok = launch();
        ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.f;
        if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
            const double us = 1000.0 * ms / 3;
            if (best < 0 || us < best) best = us;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ok ? best : -1.0;
}

// Pass `pi` of every entry of a batch.  Direct passes that share a kernel and
// a twiddle precision go out as merged launches of up to kMaxBatchDescs
// arrays (one BatchTable each); split-axis passes launch one by one.  With
// `tune`, every merged launch is first timed in each compiled launch variant
// (synchronising) and the fastest is recorded for later calls.
bool launch_level_merged(int count, const wsfft_plan_t* plans, const void* const* in, void* const* out,
                         int mode, size_t pi, hipStream_t stream, bool tune = false) {
    // Entries whose passes differ only in the launch variant the tuner chose
    // for them alone share one launch: the launch runs the variant that
    // wsfft_tune_batched recorded for it, else the variant most of its
    // entries chose (ties: the lowest), so tuned plans never split a launch
    // that untuned ones would share.
    struct Group {
        const PassKernel* k0;          // any member's kernel (its shape and kind)
        StorageKind kind;
        int sign;
        unsigned twbits;
        int votes[kMaxVariants];
        std::vector<int> idx;
        const PassKernel* k;           // the kernel the group runs
    };
    std::vector<Group> groups;
    auto add_to_group = [&](int i) {
        const wsfft_plan_s* p = plans[i];
        const Pass& P = p->passes[pi];
        const int sign = mode == 0 ? p->sign : -p->sign;
        const PassKernel* k = sign < 0 ? P.kern_neg : P.kern_pos;
        const StorageKind kind = kind_of(p->dtype, p->flags);
        const unsigned twbits = (unsigned)p->dtype * 2u + (p->flags & WSFFT_FLAG_FP32_TWIDDLES ? 1u : 0u);
        Group* g = nullptr;
        for (Group& q : groups)
            if (q.k0->n == k->n && q.k0->n2 == k->n2 && q.k0->strided == k->strided && q.k0->fused == k->fused &&
                q.kind == kind && q.sign == sign && q.twbits == twbits)
                g = &q;
        if (!g) {
            groups.push_back({k, kind, sign, twbits, {}, {}, k});
            g = &groups.back();
        }
        if (k->variant >= 0 && k->variant < kMaxVariants) ++g->votes[k->variant];
        g->idx.push_back(i);
    };
    // plane passes by sign and plane class: a class that holds more than one
    // plane shape in this level goes out as mixed-shape launches
    std::vector<int> plane_bucket[2][kPlaneClasses];
    for (int i = 0; i < count; ++i) {
        const wsfft_plan_s* p = plans[i];
        if (pi >= p->passes.size()) continue;
        const Pass& P = p->passes[pi];
        if (P.four_step != 0) {
            if (!launch_pass(p, pi, in[i], out[i], mode, stream)) return false;
            continue;
        }
        int cls, shape, lds;
        if (P.plane && P.args.os1_in == P.args.os1_out && plane_shape_info((int)P.n, (int)P.n2, &cls, &shape, &lds)) {
            const int sign = mode == 0 ? p->sign : -p->sign;
            plane_bucket[sign < 0 ? 0 : 1][cls].push_back(i);
            continue;
        }
        add_to_group(i);
    }
    for (int sg = 0; sg < 2; ++sg)
        for (int cls = 0; cls < kPlaneClasses; ++cls) {
            const std::vector<int>& b = plane_bucket[sg][cls];
            bool mixed = false;
            for (int i : b) {
                const Pass& P0 = plans[b[0]]->passes[pi];
                const Pass& P = plans[i]->passes[pi];
                mixed = mixed || P.n != P0.n || P.n2 != P0.n2;
            }
            if (!mixed) {
                for (int i : b) add_to_group(i);
                continue;
            }
            if (plane_class_prepare(cls, sg == 0 ? -1 : 1) != hipSuccess) return false;
            for (size_t c0 = 0; c0 < b.size(); c0 += kMaxPlaneEntries) {
                const size_t c1 = std::min(b.size(), c0 + (size_t)kMaxPlaneEntries);
                PlaneTable t{};
                t.count = (int32_t)(c1 - c0);
                int64_t planes = 0;
                int lds_max = 0;
                for (size_t e = c0; e < c1; ++e) {
                    const int i = b[e];
                    const wsfft_plan_s* p = plans[i];
                    const Pass& P = p->passes[pi];
                    const bool ip = in[i] == out[i];
                    auto sel = [&](int s) -> void* {
                        return s == 0 ? const_cast<void*>(in[i]) : (s == 1 ? out[i] : p->work);
                    };
                    int c, shape, lds;
                    (void)plane_shape_info((int)P.n, (int)P.n2, &c, &shape, &lds);
                    PlaneEntry& d = t.e[e - c0];
                    d.src = sel(ip ? P.src_sel_ip : P.src_sel);
                    d.dst = sel(ip ? P.dst_sel_ip : P.dst_sel);
                    d.tw = P.args.tw;
                    d.tw4 = P.args.tw4;
                    d.stride = P.args.os1_in;
                    d.scale = mode == 2 ? P.inv_scale : P.pass_scale;
                    d.shape = shape;
                    planes += P.args.C;
                    d.plane_end = planes;
                    lds_max = std::max(lds_max, lds);
                }
                if (planes < 1 || planes > 0x7fffffffLL) return false;
                if (plane_class_launch(cls, sg == 0 ? -1 : 1, t, (unsigned)planes, lds_max, stream) != hipSuccess)
                    return false;
            }
        }
    for (Group& g : groups) {
        if (g.k0->fused != 0) continue;   // fused kernels have no variants
        int best = 0;
        for (int v = 1; v < kMaxVariants; ++v)
            if (g.votes[v] > g.votes[best]) best = v;
        const PassKernel* k = find_pass_kernel(g.kind, g.sign, g.k0->n, g.k0->strided, false, best);
        if (k && prepared(k)) g.k = k;
    }
    for (const Group& g : groups) {
        for (size_t c0 = 0; c0 < g.idx.size(); c0 += kMaxBatchDescs) {
            const size_t c1 = std::min(g.idx.size(), c0 + (size_t)kMaxBatchDescs);
            if (c1 - c0 == 1) {
                const int i = g.idx[c0];
                if (!launch_pass(plans[i], pi, in[i], out[i], mode, stream)) return false;
                continue;
            }
            // this launch's identity, and the variant recorded for it
            std::string key;
            {
                char buf[160];
                std::snprintf(buf, sizeof buf, "%d:%lld:%lld:%d:%d:%d:%u", g.k0->fused, (long long)g.k0->n,
                              (long long)g.k0->n2, g.k0->strided ? 1 : 0, (int)g.kind, g.sign, g.twbits);
                key = buf;
                for (size_t e = c0; e < c1; ++e) {
                    const PassArgs& a = plans[g.idx[e]]->passes[pi].args;
                    std::snprintf(buf, sizeof buf, "|%lld,%lld,%lld,%lld", (long long)a.C, (long long)a.O1,
                                  (long long)a.es_in, (long long)a.os1_in);
                    key += buf;
                }
            }
            const PassKernel* k = g.k;
            if (g.k0->fused == 0) {
                std::lock_guard<std::mutex> lk(g_batch_tune_mu);
                auto it = g_batch_tune.find(key);
                if (it != g_batch_tune.end()) {
                    const PassKernel* kv = find_pass_kernel(g.kind, g.sign, g.k0->n, g.k0->strided, false, it->second);
                    if (kv && prepared(kv)) k = kv;
                }
            }
            BatchTable bt{};
            bt.count = (int32_t)(c1 - c0);
            PassArgs shared{};
            for (size_t e = c0; e < c1; ++e) {
                const int i = g.idx[e];
                const wsfft_plan_s* p = plans[i];
                const Pass& P = p->passes[pi];
                const bool ip = in[i] == out[i];
                auto sel = [&](int s) -> void* {
                    return s == 0 ? const_cast<void*>(in[i]) : (s == 1 ? out[i] : p->work);
                };
                ArrayDesc& d = bt.d[e - c0];
                d.src = sel(ip ? P.src_sel_ip : P.src_sel);
                d.dst = sel(ip ? P.dst_sel_ip : P.dst_sel);
                d.C = P.args.C;
                d.O1 = P.args.O1;
                d.es = P.args.es_in;
                d.os1 = P.args.os1_in;
                d.scale = mode == 2 ? P.inv_scale : P.pass_scale;
                d.tile_end = 0;
                if (e == c0) shared = P.args;
            }
            // the tile ranges and stage twiddles of launch kernel kk
            auto fill = [&](const PassKernel* kk, PassArgs& sa) -> int64_t {
                int64_t tiles = 0;
                for (size_t e = c0; e < c1; ++e) {
                    const wsfft_plan_s* p = plans[g.idx[e]];
                    const Pass& P = p->passes[pi];
                    tiles += blocks_for(P, kk);
                    bt.d[e - c0].tile_end = tiles;
                    if (e == c0 && !P.plane) sa.tw = p->tw_dev + P.tw_off + (int64_t)kk->plan * P.n;
                }
                return tiles;
            };
            if (tune && g.k0->fused == 0) {
                int best_v = -1;
                double best_us = 0.0;
                for (int v = 0; v < kMaxVariants; ++v) {
                    const PassKernel* kv = find_pass_kernel(g.kind, g.sign, g.k0->n, g.k0->strided, false, v);
                    if (!kv || kv->prepare() != hipSuccess) continue;
                    PassArgs sa = shared;
                    const int64_t t = fill(kv, sa);
                    if (t * kv->threads > 0xffffffffLL) continue;
                    const double us = time_launches(
                        [&] { return kv->launch(sa, &bt, dim3((unsigned)t), stream) == hipSuccess; }, stream);
                    if (us > 0 && (best_v < 0 || us < best_us)) {
                        best_v = v;
                        best_us = us;
                        k = kv;
                    }
                }
                if (best_v >= 0) {
                    std::lock_guard<std::mutex> lk(g_batch_tune_mu);
                    g_batch_tune[key] = best_v;
                }
            }
            const int64_t tiles = fill(k, shared);
            if (tiles * k->threads > 0xffffffffLL) return false;
            if (k->launch(shared, &bt, dim3((unsigned)tiles), stream) != hipSuccess) return false;
        }
    }
    return true;
}

// Every pass of a list in order; passes `at` and `at + 1` (at >= 0) run
// chunk by chunk over groups of chunk_planes xy-planes, the two passes of a
// chunk back to back, so the second reads what the first left in the cache.
wsfft_status_t run_passes(const wsfft_plan_s* plan, size_t count, int at, const void* in, void* out, int mode,
                          hipStream_t stream) {
    for (size_t i = 0; i < count; ++i) {
        if (at >= 0 && plan->chunk_planes > 0 && i == (size_t)at) {
            const int64_t nz = plan->n[2], zc = plan->chunk_planes;
            for (int64_t z0 = 0; z0 < nz; z0 += zc)
                for (size_t k = i; k < i + 2; ++k)
                    if (!launch_pass(plan, k, in, out, mode, stream, 1, z0, zc)) return WSFFT_ERROR_HIP;
            ++i;
            continue;
        }
        if (!launch_pass(plan, i, in, out, mode, stream)) return WSFFT_ERROR_HIP;
    }
    return WSFFT_SUCCESS;
}

wsfft_status_t exec_plan(const wsfft_plan_s* plan, const void* in, void* out, int mode, hipStream_t stream) {
    if (plan->passes.empty()) {   // every axis has length 1: the DFT is the identity
        if (in != out &&
            hipMemcpyAsync(out, in, (size_t)elem_bytes(plan->dtype), hipMemcpyDeviceToDevice, stream) != hipSuccess)
            return WSFFT_ERROR_HIP;
        return WSFFT_SUCCESS;
    }
    return run_passes(plan, plan->passes.size(), plan->chunk_at, in, out, mode, stream);
}

}  // namespace

extern "C" {

wsfft_status_t wsfft_execute(wsfft_plan_t plan, const void* in, void* out, hipStream_t stream) {
    const wsfft_status_t st = check_exec(plan, in, out);
    return st != WSFFT_SUCCESS ? st : exec_plan(plan, in, out, 0, stream);
}

wsfft_status_t wsfft_execute_adjoint(wsfft_plan_t plan, const void* in, void* out, hipStream_t stream) {
    const wsfft_status_t st = check_exec(plan, in, out);
    return st != WSFFT_SUCCESS ? st : exec_plan(plan, in, out, 1, stream);
}

wsfft_status_t wsfft_execute_inverse(wsfft_plan_t plan, const void* in, void* out, hipStream_t stream) {
    const wsfft_status_t st = check_exec(plan, in, out);
    return st != WSFFT_SUCCESS ? st : exec_plan(plan, in, out, 2, stream);
}

// The solve on a real plan, over the half spectrum in five passes: the R2C
// x pass (f -> work), the forward y pass, one z pass that runs the forward
// transform, the multiplier and the inverse transform of every z pencil, the
// inverse y pass, and the C2R x pass (work -> u) with 1/N.
static wsfft_status_t poisson_real(const wsfft_plan_s* plan, const float* f, float* u, void* work,
                                   hipStream_t stream) {
    using namespace wsfft;
    const auto& ps = plan->passes;    // x (R2C), y, z
    const auto& cs = plan->cpasses;   // z, y, x (C2R)
    if (ps.size() != 3 || cs.size() != 3) return WSFFT_ERROR_UNSUPPORTED_SIZE;
    if (ps[1].four_step != 0 || ps[2].four_step != 0 || ps[1].axis != 1 || ps[2].axis != 2 || cs[1].axis != 1)
        return WSFFT_ERROR_UNSUPPORTED_SIZE;
    const int64_t nx = plan->n[0], ny = plan->n[1], nz = plan->n[2], nxh = nx / 2 + 1;
    const PassKernel* kz = find_real_c64_neg((int)nz, true, kFusedSolveZ);
    if (!kz || nxh * ny > INT32_MAX) return WSFFT_ERROR_UNSUPPORTED_SIZE;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return WSFFT_ERROR_HIP;
    if (cur != plan->device) return WSFFT_ERROR_WRONG_DEVICE;
    if (kz->prepare() != hipSuccess) return WSFFT_ERROR_HIP;
    auto go = [&](const Pass& P, const PassKernel* k, const void* src, void* dst, float scale) {
        PassArgs a = P.args;
        a.src = src;
        a.dst = dst;
        a.scale = scale;
        a.tw = plan->tw_dev + P.tw_off + (int64_t)k->plan * P.n;   // the stage tables of k's radix plan
        a.sym_nx = (int32_t)nxh;
        a.sym_ny = (int32_t)ny;
        a.sym_half = 1;
        return k->launch(a, nullptr, dim3((unsigned)blocks_for(P, k)), stream) == hipSuccess;
    };
    const double N = (double)nx * (double)ny * (double)nz;
    const bool ok = go(ps[0], ps[0].kern_neg, f, work, 1.0f) && go(ps[1], ps[1].kern_neg, work, work, 1.0f) &&
                    go(ps[2], kz, work, work, 1.0f) && go(cs[1], cs[1].kern_pos, work, work, 1.0f) &&
                    go(cs[2], cs[2].kern_pos, work, u, (float)(1.0 / N));
    return ok ? WSFFT_SUCCESS : WSFFT_ERROR_HIP;
}

wsfft_status_t wsfft_poisson_solve(wsfft_plan_t plan, const float* f, float* u, void* work, hipStream_t stream) {
    using namespace wsfft;
    if (!plan_live(plan)) return WSFFT_ERROR_INVALID_PLAN;
    if (!f || !u || !work) return WSFFT_ERROR_NULL_POINTER;
    if (((uintptr_t)f % 4) || ((uintptr_t)u % 4) || ((uintptr_t)work % 8)) return WSFFT_ERROR_MISALIGNED;
    if (work == (const void*)f || work == (void*)u) return WSFFT_ERROR_INVALID_VALUE;
    if (plan->real && plan->half_pitch != plan->n[0] / 2 + 1) return WSFFT_ERROR_INVALID_VALUE;
    if (plan->real) return poisson_real(plan, f, u, work, stream);
    if (plan->dtype != WSFFT_C64) return WSFFT_ERROR_UNSUPPORTED_SIZE;
    // three direct passes x (contiguous), y, z (strided), each with fused kernels
    const auto& ps = plan->passes;
    if (ps.size() != 3) return WSFFT_ERROR_UNSUPPORTED_SIZE;
    for (int i = 0; i < 3; ++i)
        if (ps[i].four_step != 0 || ps[i].axis != i || ps[i].strided != (i > 0)) return WSFFT_ERROR_UNSUPPORTED_SIZE;
    const int64_t nx = plan->n[0], ny = plan->n[1], nz = plan->n[2];
    const PassKernel* kin = find_fused_c64_neg((int)nx, false, kFusedRealIn);
    const PassKernel* ksym = find_fused_c64_neg((int)nz, true, kFusedPoisson);
    const PassKernel* kout = find_fused_c64_pos((int)nz, true, kFusedRealOut);
    if (!kin || !ksym || !kout || nx > INT32_MAX || ny > INT32_MAX) return WSFFT_ERROR_UNSUPPORTED_SIZE;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return WSFFT_ERROR_HIP;
    if (cur != plan->device) return WSFFT_ERROR_WRONG_DEVICE;
    if (kin->prepare() != hipSuccess || ksym->prepare() != hipSuccess || kout->prepare() != hipSuccess)
        return WSFFT_ERROR_HIP;
    auto go = [&](const Pass& P, const PassKernel* k, const void* src, void* dst, float scale) {
        PassArgs a = P.args;
        a.src = src;
        a.dst = dst;
        a.scale = scale;
        a.tw = plan->tw_dev + P.tw_off + (int64_t)k->plan * P.n;   // the stage tables of k's radix plan
        a.sym_nx = (int32_t)nx;
        a.sym_ny = (int32_t)ny;
        return k->launch(a, nullptr, dim3((unsigned)blocks_for(P, k)), stream) == hipSuccess;
    };
    const double N = (double)nx * (double)ny * (double)nz;
    const bool ok =
        // forward, sign -1: real input, then y, then z times -1/|k|^2
        go(ps[0], kin, f, work, ps[0].pass_scale) && go(ps[1], ps[1].kern_neg, work, work, ps[1].pass_scale) &&
        go(ps[2], ksym, work, work, ps[2].pass_scale) &&
        // inverse, sign +1: x, y, then z storing the real part times 1/N
        go(ps[0], ps[0].kern_pos, work, work, ps[0].pass_scale) &&
        go(ps[1], ps[1].kern_pos, work, work, ps[1].pass_scale) &&
        go(ps[2], kout, work, u, (float)((double)ps[2].pass_scale / N));
    return ok ? WSFFT_SUCCESS : WSFFT_ERROR_HIP;
}

}  // extern "C"

// ---- allocation-free Poisson solve ------------------------------------------------
// The work memory of wsfft_poisson_solve_noalloc: a file-scope device array
// of kScratchBytes that every GPU running the library holds until the
// process ends.  In host code its name is not a device address; each
// device's address comes from hipGetSymbolAddress at the first call on that
// device and is kept in g_scratch_ptr.
namespace {
constexpr size_t kScratchBytes = size_t(72) << 20;
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

extern "C" {

wsfft_status_t wsfft_poisson_solve_noalloc(wsfft_plan_t plan, const float* f, float* u, hipStream_t stream) {
    if (!plan_live(plan)) return WSFFT_ERROR_INVALID_PLAN;
    if (!f || !u) return WSFFT_ERROR_NULL_POINTER;
    if (((uintptr_t)f % 4) || ((uintptr_t)u % 4)) return WSFFT_ERROR_MISALIGNED;
    const int64_t nx = plan->n[0], ny = plan->n[1], nz = plan->n[2];
    const int64_t need = (plan->real ? nx / 2 + 1 : nx) * ny * nz * 8;
    if (need > (int64_t)kScratchBytes) return WSFFT_ERROR_EXCEEDS_SCRATCH;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return WSFFT_ERROR_HIP;
    if (cur != plan->device) return WSFFT_ERROR_WRONG_DEVICE;
    if (cur < 0 || cur >= kScratchDevices) return WSFFT_ERROR_UNSUPPORTED_SIZE;
    void* work = nullptr;
    {
        std::lock_guard<std::mutex> g(g_scratch_mu);
        if (!g_scratch_ptr[cur]) {
            void* p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return WSFFT_ERROR_HIP;
            g_scratch_ptr[cur] = p;
        }
        work = g_scratch_ptr[cur];
    }
    return wsfft_poisson_solve(plan, f, u, work, stream);
}

wsfft_status_t wsfft_execute_pass(wsfft_plan_t plan, int index, int mode, const void* in, void* out,
                                  hipStream_t stream) {
    const bool real = plan_live(plan) && plan->real;
    const wsfft_status_t st = real ? check_real(plan, in, out, 4, 4) : check_exec(plan, in, out);
    if (st != WSFFT_SUCCESS) return st;
    const size_t np = (real && mode != 0) ? plan->cpasses.size() : plan->passes.size();
    if (mode < 0 || mode > 2 || index < 0 || (size_t)index >= np) return WSFFT_ERROR_INVALID_VALUE;
    return launch_pass(plan, (size_t)index, in, out, mode, stream) ? WSFFT_SUCCESS : WSFFT_ERROR_HIP;
}

wsfft_status_t wsfft_execute_r2c(wsfft_plan_t plan, const float* in, void* out, hipStream_t stream) {
    const wsfft_status_t st = check_real(plan, in, out, 4, 8);
    if (st != WSFFT_SUCCESS) return st;
    for (size_t i = 0; i < plan->passes.size(); ++i)
        if (!launch_pass(plan, i, in, out, 0, stream)) return WSFFT_ERROR_HIP;
    return WSFFT_SUCCESS;
}

static wsfft_status_t exec_c2r(wsfft_plan_t plan, void* in, float* out, int mode, hipStream_t stream) {
    const wsfft_status_t st = check_real(plan, in, out, 8, 4);
    if (st != WSFFT_SUCCESS) return st;
    for (size_t i = 0; i < plan->cpasses.size(); ++i)
        if (!launch_pass(plan, i, in, out, mode, stream)) return WSFFT_ERROR_HIP;
    return WSFFT_SUCCESS;
}

wsfft_status_t wsfft_execute_c2r(wsfft_plan_t plan, void* in, float* out, hipStream_t stream) {
    return exec_c2r(plan, in, out, 1, stream);
}

wsfft_status_t wsfft_execute_c2r_inverse(wsfft_plan_t plan, void* in, float* out, hipStream_t stream) {
    return exec_c2r(plan, in, out, 2, stream);
}

int wsfft_plan_is_real(wsfft_plan_t plan) { return plan_live(plan) ? (plan->real ? 1 : 0) : -1; }

static wsfft_status_t batched(int count, const wsfft_plan_t* plans, const void* const* in, void* const* out,
                              int adjoint, hipStream_t stream, bool tune) {
    if (count < 0) return WSFFT_ERROR_INVALID_VALUE;
    if (count == 0) return WSFFT_SUCCESS;
    if (!plans || !in || !out) return WSFFT_ERROR_NULL_POINTER;
    size_t maxp = 0;
    for (int i = 0; i < count; ++i) {
        const wsfft_status_t st = check_exec(plans[i], in[i], out[i]);
        if (st != WSFFT_SUCCESS) return st;
        if (plans[i]->dtype != plans[0]->dtype) return WSFFT_ERROR_INVALID_VALUE;
        // entries run pass-major, so a plan's work buffer would be shared
        if (uses_work(plans[i], in[i], out[i])) return WSFFT_ERROR_INVALID_VALUE;
        maxp = std::max(maxp, plans[i]->passes.size());
    }
    const int mode = adjoint ? 1 : 0;
    // One plan over arrays spaced exactly one array apart, in and out alike:
    // the batch is one larger array whose slowest axis is not transformed.
    bool uniform = count > 1 && !plans[0]->passes.empty();
    const int64_t N = plans[0]->n[0] * plans[0]->n[1] * plans[0]->n[2];
    const intptr_t span = (intptr_t)(N * elem_bytes(plans[0]->dtype));
    for (int i = 1; uniform && i < count; ++i)
        uniform = plans[i] == plans[0] &&
                  (const char*)in[i] - (const char*)in[0] == (intptr_t)i * span &&
                  (const char*)out[i] - (const char*)out[0] == (intptr_t)i * span;
    if (uniform && (in[0] == out[0] || (const char*)out[0] >= (const char*)in[0] + span * count ||
                    (const char*)in[0] >= (const char*)out[0] + span * count)) {
        for (size_t pi = 0; pi < plans[0]->passes.size(); ++pi)
            if (!launch_pass(plans[0], pi, in[0], out[0], mode, stream, count)) return WSFFT_ERROR_HIP;
        return WSFFT_SUCCESS;
    }
    // identity plans first, then pass-major order over the batch
    for (int i = 0; i < count; ++i)
        if (plans[i]->passes.empty()) {
            const wsfft_status_t st = exec_plan(plans[i], in[i], out[i], mode, stream);
            if (st != WSFFT_SUCCESS) return st;
        }
    for (size_t pi = 0; pi < maxp; ++pi)
        if (!launch_level_merged(count, plans, in, out, mode, pi, stream, tune)) return WSFFT_ERROR_HIP;
    return WSFFT_SUCCESS;
}

wsfft_status_t wsfft_execute_batched(int count, const wsfft_plan_t* plans, const void* const* in,
                                     void* const* out, int adjoint, hipStream_t stream) {
    return batched(count, plans, in, out, adjoint, stream, false);
}

wsfft_status_t wsfft_tune_batched(int count, const wsfft_plan_t* plans, const void* const* in, void* const* out,
                                  int adjoint, hipStream_t stream) {
    const wsfft_status_t st = batched(count, plans, in, out, adjoint, stream, true);
    if (st != WSFFT_SUCCESS || count == 0) return st;
    return hipStreamSynchronize(stream) == hipSuccess ? WSFFT_SUCCESS : WSFFT_ERROR_HIP;
}

}  // extern "C"

namespace wsfft {

const PassKernel* find_pass_kernel(StorageKind kind, int sign, int n, bool strided, bool four_step, int v) {
    switch (kind) {
        case kC64:
            return sign < 0 ? find_pass_c64_neg(n, strided, four_step, v) : find_pass_c64_pos(n, strided, four_step, v);
        case kF16:
            return sign < 0 ? find_pass_f16_neg(n, strided, four_step, v) : find_pass_f16_pos(n, strided, four_step, v);
        case kBF16:
            return sign < 0 ? find_pass_bf16_neg(n, strided, four_step, v) : find_pass_bf16_pos(n, strided, four_step, v);
        case kF16Math:
            return sign < 0 ? find_pass_f16m_neg(n, strided, four_step, v) : find_pass_f16m_pos(n, strided, four_step, v);
    }
    return nullptr;
}

const PassKernel* find_cached_kernel(StorageKind kind, int sign, int n, bool strided, int fused) {
    switch (kind) {
        case kC64: return sign < 0 ? find_cached_c64_neg(n, strided, fused) : find_cached_c64_pos(n, strided, fused);
        case kF16: return sign < 0 ? find_cached_f16_neg(n, strided, fused) : find_cached_f16_pos(n, strided, fused);
        case kBF16: return sign < 0 ? find_cached_bf16_neg(n, strided, fused) : find_cached_bf16_pos(n, strided, fused);
        case kF16Math:
            return sign < 0 ? find_cached_f16m_neg(n, strided, fused) : find_cached_f16m_pos(n, strided, fused);
    }
    return nullptr;
}

}  // namespace wsfft

// ---- batch plans: one persistent launch per execution -----------------------------

struct wsfft_batch_plan_s {
    int device;
    int sign;                  // effective kernel sign of every pass
    int npasses;
    int64_t total;             // work items (tiles) of one execution
    wsfft::PersistLevels levels;
    unsigned grid;
    wsfft::PersistPass* d_passes = nullptr;
    wsfft::PersistCounters* d_ctr = nullptr;
    unsigned spin_limit = 1u << 22;   // polls before a dependency wait gives up
};

namespace {
std::mutex g_batch_mu;
std::unordered_set<const wsfft_batch_plan_s*> g_batches;
thread_local wsfft_status_t g_batch_error = WSFFT_SUCCESS;

wsfft_batch_plan_t batch_fail(wsfft_status_t st) {
    g_batch_error = st;
    return nullptr;
}
bool batch_live(const wsfft_batch_plan_s* b) {
    if (!b) return false;
    std::lock_guard<std::mutex> g(g_batch_mu);
    return g_batches.count(b) != 0;
}
}  // namespace

extern "C" {

wsfft_batch_plan_t wsfft_batch_plan_create(int count, const wsfft_plan_t* plans, const void* const* in,
                                           void* const* out, int adjoint) {
    using namespace wsfft;
    if (count < 1) return batch_fail(WSFFT_ERROR_INVALID_VALUE);
    if (!plans || !in || !out) return batch_fail(WSFFT_ERROR_NULL_POINTER);
    int sign = 0;
    size_t maxp = 0;
    // each plan's passes for the persistent kernel: a fused plane pass runs as
    // its x and y passes there (the kernel has no plane branch)
    std::vector<std::vector<Pass>> lists((size_t)count);
    for (int i = 0; i < count; ++i) {
        const wsfft_status_t st = check_exec(plans[i], in[i], out[i]);
        if (st != WSFFT_SUCCESS) return batch_fail(st);
        const wsfft_plan_s* p = plans[i];
        if (p->dtype != WSFFT_C64 || p->nsplit > 0) return batch_fail(WSFFT_ERROR_UNSUPPORTED_SIZE);
        const int s = adjoint ? -p->sign : p->sign;
        if (sign == 0) sign = s;
        if (s != sign) return batch_fail(WSFFT_ERROR_INVALID_VALUE);
        for (const Pass& P : p->passes) {
            if (!P.plane) {
                lists[i].push_back(P);
                continue;
            }
            const int64_t nx = p->n[0], ny = p->n[1], nz = p->n[2];
            Pass X{}, Y{};
            set_direct(X, AxisGeo{0, nx, 1, ny * nz});
            set_direct(Y, AxisGeo{1, ny, nx, nz});
            X.axis = 0; X.n = nx; X.tw_off = P.tw_off;
            Y.axis = 1; Y.n = ny; Y.tw_off = P.tw4_off;
            for (Pass* Q : {&X, &Y}) {
                Q->four_step = 0;
                Q->pass_scale = Q->inv_scale = 1.0f;
                Q->src_sel = Q->src_sel_ip = 1;
                Q->dst_sel = Q->dst_sel_ip = 1;
            }
            X.src_sel = P.src_sel; X.src_sel_ip = P.src_sel_ip;   // the plane pass's input
            lists[i].push_back(X);
            lists[i].push_back(Y);
        }
        for (const Pass& P : lists[i])
            if (P.four_step != 0 || persist_type((int)P.n, P.strided) < 0)
                return batch_fail(WSFFT_ERROR_UNSUPPORTED_SIZE);
        maxp = std::max(maxp, lists[i].size());
    }
    if (maxp > (size_t)kPersistMaxLevels) return batch_fail(WSFFT_ERROR_UNSUPPORTED_SIZE);
    // superstep-major list of passes
    std::vector<PersistPass> list;
    PersistLevels levels{};
    int64_t total = 0;
    for (size_t pi = 0; pi < maxp; ++pi) {
        for (int i = 0; i < count; ++i) {
            const wsfft_plan_s* p = plans[i];
            if (pi >= lists[i].size()) continue;
            const Pass& P = lists[i][pi];
            PersistPass q{};
            q.a = P.args;
            // the stage twiddles of the persistent branch's radix plan
            q.a.tw = p->tw_dev + P.tw_off + (int64_t)persist_plan((int)P.n, P.strided) * P.n;
            const bool ip = in[i] == out[i];
            const int ss = ip ? P.src_sel_ip : P.src_sel, ds = ip ? P.dst_sel_ip : P.dst_sel;
            q.a.src = ss == 0 ? in[i] : out[i];
            q.a.dst = ds == 0 ? const_cast<void*>(in[i]) : out[i];
            q.a.scale = P.pass_scale;
            const int64_t per = persist_per_block((int)P.n, P.strided);
            q.tiles = P.strided ? ((q.a.C + per - 1) / per) * q.a.O1 * q.a.O2 : (q.a.C + per - 1) / per;
            q.type = persist_type((int)P.n, P.strided);
            q.level = (int32_t)pi;
            q.first = total;
            total += q.tiles;
            list.push_back(q);
        }
        levels.end[pi] = total;
        levels.count = (int32_t)pi + 1;
    }
    // tickets are 32-bit and every workgroup draws one past the end
    if (list.empty() || total > 0x7fffffffLL) return batch_fail(WSFFT_ERROR_UNSUPPORTED_SIZE);
    wsfft_batch_plan_s* b = new (std::nothrow) wsfft_batch_plan_s();
    if (!b) return batch_fail(WSFFT_ERROR_OUT_OF_MEMORY);
    b->device = plans[0]->device;
    b->sign = sign;
    b->npasses = (int)list.size();
    b->total = total;
    b->levels = levels;
    int per_cu = 0, cus = 0;
    if (persist_prepare(&per_cu) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess) {
        delete b;
        return batch_fail(WSFFT_ERROR_HIP);
    }
    b->grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(total, (int64_t)std::max(1, per_cu) * cus));
    const size_t ctr_bytes = sizeof(PersistCounters);
    if (hipMalloc(&b->d_passes, sizeof(PersistPass) * list.size()) != hipSuccess) {
        delete b;
        return batch_fail(WSFFT_ERROR_OUT_OF_MEMORY);
    }
    if (hipMalloc(&b->d_ctr, ctr_bytes) != hipSuccess) {
        (void)hipFree(b->d_passes);
        delete b;
        return batch_fail(WSFFT_ERROR_OUT_OF_MEMORY);
    }
    if (hipMemcpy(b->d_passes, list.data(), sizeof(PersistPass) * list.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(b->d_ctr, 0, ctr_bytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(b->d_passes);
        (void)hipFree(b->d_ctr);
        delete b;
        return batch_fail(WSFFT_ERROR_HIP);
    }
    {
        std::lock_guard<std::mutex> g(g_batch_mu);
        g_batches.insert(b);
    }
    g_batch_error = WSFFT_SUCCESS;
    return b;
}

wsfft_status_t wsfft_batch_get_last_error(void) { return g_batch_error; }

wsfft_status_t wsfft_batch_execute(wsfft_batch_plan_t b, hipStream_t stream) {
    if (!batch_live(b)) return WSFFT_ERROR_INVALID_PLAN;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return WSFFT_ERROR_HIP;
    if (cur != b->device) return WSFFT_ERROR_WRONG_DEVICE;
    // a dependency wait gives up after spin_limit polls (by default 2^22, well
    // under a second per wait and far beyond any tile's duration): a bug
    // cannot hang the GPU
    return wsfft::persist_launch(b->sign, b->d_passes, b->npasses, b->levels, b->d_ctr, b->grid, b->spin_limit,
                                 stream) == hipSuccess
               ? WSFFT_SUCCESS
               : WSFFT_ERROR_HIP;
}

wsfft_status_t wsfft_batch_plan_set_spin_limit(wsfft_batch_plan_t b, unsigned polls) {
    if (!batch_live(b)) return WSFFT_ERROR_INVALID_PLAN;
    b->spin_limit = polls;
    return WSFFT_SUCCESS;
}

int64_t wsfft_batch_plan_tiles(wsfft_batch_plan_t b) { return batch_live(b) ? b->total : -1; }

wsfft_status_t wsfft_batch_plan_check(wsfft_batch_plan_t b, int* timed_out) {
    if (!batch_live(b)) return WSFFT_ERROR_INVALID_PLAN;
    if (!timed_out) return WSFFT_ERROR_NULL_POINTER;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return WSFFT_ERROR_HIP;
    if (cur != b->device) return WSFFT_ERROR_WRONG_DEVICE;
    // launches already enqueued must have finished before their count is read
    if (hipDeviceSynchronize() != hipSuccess) return WSFFT_ERROR_HIP;
    unsigned failed = 0;
    if (hipMemcpy(&failed, &b->d_ctr->failed, sizeof failed, hipMemcpyDeviceToHost) != hipSuccess)
        return WSFFT_ERROR_HIP;
    if (failed != 0 && hipMemset(&b->d_ctr->failed, 0, sizeof failed) != hipSuccess) return WSFFT_ERROR_HIP;
    *timed_out = failed != 0;
    return WSFFT_SUCCESS;
}

void wsfft_batch_plan_destroy(wsfft_batch_plan_t b) {
    if (!b) return;
    {
        std::lock_guard<std::mutex> g(g_batch_mu);
        if (!g_batches.erase(b)) return;
    }
    int cur = -1;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(b->d_passes);
    (void)hipFree(b->d_ctr);
    if (cur >= 0) (void)hipSetDevice(cur);
    delete b;
}

}  // extern "C"
