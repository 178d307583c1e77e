// Internal interface of the persistent batch kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pstereo_internal.h"

namespace pstereo {

// A run of tasks of one (frame, phase) in claim order.
struct BatchSeg {
    int frame;
    int phase;  // 0 block statistics, 1 region grouping, 2 depth filter, 3 warp
    int first;  // index of the first task
    int ntask;  // tasks in the run
    int items;  // tiles (phases 0, 2), rows (phase 3) or 1 (phase 1)
    int gx;     // tiles per tile row (phases 0, 2)
};

struct BatchDesc {
    const FrameDesc* frames;  // [nframes]
    const BatchSeg* segs;     // [4 * nframes] in claim order
    const int* need;          // [4 * nframes]: tasks of (frame, phase)
    uint32_t* ctr;            // [0]: next task; [1 + 4 f + p]: finished tasks of (frame f, phase p)
    int nframes;
    int ntask;
};

int batch_tasks(const FrameDesc& f, int phase, int* items, int* gx);
bool batch_width_ok(int w);
hipError_t prepare_batch_kernels();
hipError_t launch_batch(const BatchDesc& bd, int r, int grid, hipStream_t s);

}  // namespace pstereo
