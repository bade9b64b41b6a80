// Host interface of the plane passes of several plane shapes in one launch
// (plane.hip): a merged batch level whose arrays have different xy-plane
// shapes runs them as one launch per plane class instead of one per shape.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace wsfft {

// One array of a mixed-shape plane launch: its planes (plane_end minus the
// previous entry's plane_end of them, `stride` complex64 values apart, in
// place or out of place), the x and y stage twiddle tables of its shape
// (radix plan 1 blocks, as the single-shape plane pass takes them), and a
// factor on every stored value.
struct PlaneEntry {
    const void* src;
    void* dst;
    const float2* tw;
    const float2* tw4;
    int64_t stride;
    int64_t plane_end;
    float scale;
    int32_t shape;      // index of (nx, ny) in the plane shape list
};
constexpr int kMaxPlaneEntries = 32;
struct PlaneTable {
    int32_t count;
    int32_t pad;
    PlaneEntry e[kMaxPlaneEntries];
};

// Plane shapes with a plane pass share a launch when they share a class
// (workgroup size and LDS bracket).  Returns false when (nx, ny) has no plane
// pass; else its class (0 .. kPlaneClasses-1), shape index and LDS bytes.
constexpr int kPlaneClasses = 4;
bool plane_shape_info(int nx, int ny, int* cls, int* shape, int* lds_bytes);
// Sets the class kernel's dynamic LDS limit (once per class and sign).
hipError_t plane_class_prepare(int cls, int sign);
// One workgroup per plane of every entry: grid = t.e[t.count - 1].plane_end
// workgroups, `lds` bytes of dynamic LDS (the largest of the entries' shapes).
hipError_t plane_class_launch(int cls, int sign, const PlaneTable& t, unsigned planes, int lds, hipStream_t s);

}  // namespace wsfft
