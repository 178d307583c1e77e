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

// The fused kernel's work is split into kXcds queues, one per XCD: every
// frame belongs to one queue, and only the workgroups running on that XCD
// (read from the hardware's XCC id) claim its tasks, so a task and the tasks
// it depends on run on one XCD and share its L2.
constexpr int kXcds = 8;

struct BatchDesc {
    const FrameDesc* frames;  // [nframes]
    const BatchSeg* segs;     // [4 * nframes]: queue q's segments are [qseg[q], qseg[q + 1]), in claim order
    const int* need;          // [4 * nframes]: tasks of (frame, phase)
    uint32_t* ctr;            // [q]: next task of queue q; [kXcds + 4 f + p]: finished tasks of (frame f,
                              // phase p); [kXcds + 4 nframes]: abort word (a dependency wait timed out)
    int nframes;
    int qseg[kXcds + 1];
    int qntask[kXcds];        // tasks of each queue
};

// Launch plan of the staged form: per-stage workgroup counts and the warp
// launches, one per distinct (lanes, quads per lane) shape among the frames.
constexpr int kMaxWarpClasses = 24;
struct StagedPlan {
    int n = 0;
    int tiles_bs = 0, tiles_cbf = 0;
    size_t regions_lds = 0;
    int r = 2;
    bool k2 = false;    // blocks of 2 px (shared by every frame of the batch)
    int warp_rows = 1;  // image rows per warp workgroup
    int bs_rows = 0;    // block-statistics tile rows (0 = each block size's default)
    int nclass = 0;
    int cls_threads[kMaxWarpClasses];
    int cls_q[kMaxWarpClasses];
    size_t cls_lds[kMaxWarpClasses];
    int cls_rows[kMaxWarpClasses];  // workgroups of each warp launch
};

// d_first: (2 + nclass) tables of n + 1 ints: first workgroup of each frame in
// the block-statistics launch, the depth-filter launch, then each warp launch.
hipError_t launch_staged(const FrameDesc* d_frames, const int* d_first, const StagedPlan& plan, hipStream_t s);

// Device scratch of one job: block tables (gw * gh entries each) and the
// filtered-depth image (w * h bytes).
struct JobScratch {
    uint32_t* stats;
    uint2* binfo;
    int32_t* labels;
    uint8_t* df;
};

// Scratch bytes of one job of size w x h with blocks K (tables then depth,
// each 256-byte aligned); carve() lays such a region out.
size_t job_scratch_bytes(int w, int h, int K);
JobScratch job_scratch_carve(uint8_t* base, int w, int h, int K);

// Stage `phase` (0 block statistics, 1 grouping, 2 filter, 3 warp) of frame
// f: its items (tiles, or rows for the warp) and tile columns, and the
// fused kernel's tasks for them; bs_rows: the block-statistics tile height
// (0 = each block size's default, which the fused kernel uses).
int batch_tasks(const FrameDesc& f, int phase, int* items, int* gx, int bs_rows = 0);
bool batch_width_ok(int w);
hipError_t prepare_batch_kernels();
hipError_t launch_batch(const BatchDesc& bd, int r, int grid, hipStream_t s);

}  // namespace pstereo

struct pstereo_batch;

namespace pstereo {

// Batch objects for a caller that brings each job's scratch (the server):
// own_scratch = false allocates only the task tables; prepare then takes one
// JobScratch per job and, with check_ptrs = false, trusts the caller to have
// validated the job's device pointers.
int batch_create_internal(pstereo_ctx* ctx, int max_jobs, int64_t max_pixels, bool own_scratch, pstereo_batch** out);
int batch_prepare_internal(pstereo_batch* b, const pstereo_job* jobs, int n, const pstereo_params* p,
                           const JobScratch* scratch, bool check_ptrs);

}  // namespace pstereo
