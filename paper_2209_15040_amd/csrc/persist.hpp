// Persistent batched launch (persist.hip): shared host/device types.
#pragma once
#include <hip/hip_runtime.h>
#include "fft_device.hpp"

namespace wsfft {

constexpr int kPersistThreads = 256;

constexpr int kPersistMaxLevels = 4;   // supersteps per array

// One superstep of one array.
struct PersistPass {
    PassArgs a;          // resolved arguments (buffers, geometry, scale)
    int64_t first;       // index of its first tile in the launch's work list
    int64_t tiles;
    int32_t type;        // kernel branch (persist_type)
    int32_t level;       // superstep index; the work list is level-major
};

// Tiles of each level: level L holds work items [end[L-1], end[L]).
struct PersistLevels {
    int64_t end[kPersistMaxLevels];
    int32_t count;
    int32_t pad;
};

// Device-resident counters owned by one batch plan.
struct PersistCounters {
    unsigned ticket;     // next work item
    unsigned finished;   // workgroups that left
    unsigned error;      // nonzero: a dependency wait of the running launch timed out
    unsigned failed;     // launches that ended with `error` set (kept until the host clears it)
    unsigned done[kPersistMaxLevels];   // tiles published per level
};

int persist_type(int n, bool strided);        // -1: no persistent kernel for it
int persist_per_block(int n, bool strided);   // pencils or columns per workgroup
int persist_plan(int n, bool strided);        // radix plan of that branch (its stage twiddle table)
int persist_lds_bytes();
hipError_t persist_prepare(int* blocks_per_cu);
hipError_t persist_launch(int sign, const PersistPass* passes, int npasses, const PersistLevels& levels,
                          PersistCounters* ctr, unsigned grid, unsigned spin_limit, hipStream_t s);

}  // namespace wsfft
