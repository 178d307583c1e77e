// Internal interface between the C ABI layer and the gfx950 kernels.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pstereo.h"

namespace pstereo {

// Everything one frame's kernels need, passed by value as a kernel argument.
struct FrameDesc {
    const uint8_t* frame;    // RGB24 [h][w][3]
    uint8_t* out_l;          // RGB24 outputs, any may be null
    uint8_t* out_r;
    uint8_t* out_a;
    const uint8_t* depth_in; // external depth map (u8 [h][w]) or null
    uint8_t* out_df;         // optional filtered-depth dump
    uint8_t* out_d0;         // optional raw-depth dump
    uint8_t* out_h;          // optional half side-by-side frame, RGB24 [h][w][3]
    uint32_t* stats;         // per block: mean R | G << 8 | B << 16 | edge << 24
    uint2* binfo;            // per block: {stats, region depth}
    int32_t* labels;         // per block: region label
    uint8_t* df;             // filtered depth scratch, u8 [h][w] (4-byte aligned)
    // strip-parallel region grouping (rstrip > 0): strip-local components are
    // merged across strip boundaries through a table of slots; binfo then
    // holds {statistics, slot of the block's component} until resolved
    uint2* rent;             // per slot: {strip-local label, non-edge count}
    uint32_t* rrow;          // per slot: lowest block row + 1
    uint32_t* rfin;          // per slot: final label << 9 | background << 8 | depth
    uint2* rbnd;             // boundary join candidates: {block above the strip, slot below}
    uint32_t* rctl;          // [0]: slots taken, [1]: 1 if the merge fell back to one workgroup,
                             // [2]: boundary candidates
    int rstrip;              // block rows per strip, 0 = single-workgroup grouping
    int w, h;
    int K, gw, gh;           // depth block size and grid
    int B, T, g, tau, r;     // method parameters
    int aligned;             // w % 4 == 0 and every RGB24 pointer 4-byte aligned
    int gather;              // reconstruct by the Fig. 3 gather instead of the warp and fill
    // block-iterative inpainting (ipc != null): the warp leaves, per view, the
    // warped colour and a fill tag (0 landed, 0xFFFF hole, s = filled by sweep
    // s) for the sweeps and the final composition
    uint32_t* ipc;           // colours, [2][h][w]
    uint16_t* ipt;           // tags, [2][h][w]
    uint32_t* ipn;           // pixels filled per sweep, [kMaxSweeps + 1]
    // end-of-depth-map signal (pipelined calls): the grouping's last kernel
    // stores sig_value to *sig when it is done (null: no signal)
    unsigned long long* sig;
    unsigned long long sig_value;
    // start-of-filter mark (pipelined calls): the depth filter stores
    // mark_value to *mark as it starts, i.e. once everything before it on
    // its stream is done (null: no mark)
    unsigned long long* mark;
    unsigned long long mark_value;
    // start-of-warp mark (three-stage pipelined calls): the warp stores
    // wmark_value to *wmark as it starts (null: no mark)
    unsigned long long* wmark;
    unsigned long long wmark_value;
};

// Launch shape of the warp kernel (one image row per workgroup).
struct WarpShape {
    int threads;        // workgroup size (multiple of 64, <= 1024)
    int quads;          // quads (4 px) per lane: 1, 2 or 4
    size_t lds_bytes;   // dynamic LDS per workgroup
};

// One kernel launch of a frame: every kernel takes a single FrameDesc.
struct LaunchSpec {
    const void* func;
    dim3 grid, block;
    size_t lds;
};

// Launch specifications (kernels_depth.hip, kernels_render.hip); func is null
// for an unsupported combination.
bool warp_shape(int w, WarpShape* out);
// The fewest quads per lane (1, 2, 4) that keep the lanes of a row within
// cap (else four quads per lane, up to 1024 lanes).
bool warp_shape_cap(int w, int cap, WarpShape* out);
LaunchSpec spec_blockstats(const FrameDesc& f);
LaunchSpec spec_regions(const FrameDesc& f);
// Strip-parallel grouping: strips, merge, per-block resolution.
int strip_rows(int gw);
constexpr int kRegionSlots = 4096;
constexpr int kBoundSlots = 8192;
LaunchSpec spec_rg_strip(const FrameDesc& f);
LaunchSpec spec_rg_merge(const FrameDesc& f);
LaunchSpec spec_rg_final(const FrameDesc& f);
LaunchSpec spec_cbf(const FrameDesc& f);
LaunchSpec spec_warp(const FrameDesc& f, const WarpShape& ws);
// Block-iterative inpainting: counter reset, one Jacobi sweep, composition.
constexpr int kMaxSweeps = 4096;
hipError_t launch_inpaint_reset(const FrameDesc& f, hipStream_t s);
hipError_t launch_inpaint_sweep(const FrameDesc& f, int sweep, hipStream_t s);
hipError_t launch_inpaint_final(const FrameDesc& f, hipStream_t s);
// Fig. 3 gather in place of the warp and the fill (one row per workgroup).
bool gather_fits(int w);
LaunchSpec spec_gather(const FrameDesc& f);

// Launch one spec on a stream (hipSuccess or the launch error).
inline hipError_t launch(const LaunchSpec& ls, const FrameDesc& f, hipStream_t s) {
    if (!ls.func) return hipErrorInvalidValue;
    FrameDesc arg = f;
    void* args[] = {&arg};
    return hipLaunchKernel(ls.func, ls.grid, ls.block, args, ls.lds, s);
}
// The same with the kernel's own start and stop times recorded into two
// events (timestamps of the dispatch itself, no marker packets around it).
inline hipError_t launch_timed(const LaunchSpec& ls, const FrameDesc& f, hipStream_t s, hipEvent_t start,
                               hipEvent_t stop) {
    if (!ls.func) return hipErrorInvalidValue;
    FrameDesc arg = f;
    void* args[] = {&arg};
    return hipExtLaunchKernel(ls.func, ls.grid, ls.block, args, ls.lds, s, start, stop, 0);
}
size_t regions_lds_bytes(int nb);
// Zero n words with a kernel (no memset node, so it can sit in a captured graph).
hipError_t launch_clear_words(uint32_t* p, int n, hipStream_t s);
// Store v to *p (system-scope release) once everything before it on s is done.
hipError_t launch_signal(unsigned long long* p, unsigned long long v, hipStream_t s);
// Concurrency probe of two idle streams: a bounded wait on wait_on for a
// store of token to w[0] from post_on; w[1] receives 1 if the store was seen
// while waiting, 2 if not (the streams ran one after the other).
hipError_t launch_probe(unsigned long long* w, unsigned long long token, hipStream_t wait_on, hipStream_t post_on);
hipError_t prepare_depth_kernels();
hipError_t prepare_render_kernels();

// Accessors of the opaque context for the other C ABI files: its device, the
// batch object it keeps for pstereo_synthesize_batch, and its last-error text.
int ctx_device(const pstereo_ctx* c);
pstereo_batch** ctx_batch(pstereo_ctx* c);
void ctx_set_error(pstereo_ctx* c, const char* msg);

}  // namespace pstereo
