// Batched forms: many frames of uneven size per launch.
//
// Fused form: one persistent kernel.
// Every workgroup (1024 lanes, one per CU) loops: claim the next task from
// its XCD's queue (the next one is claimed while the current one runs), wait
// until the task's inputs are complete, run it, count it done.  Each frame
// belongs to one of the eight queues (the host balances their pixels), and
// each queue's tasks are numbered in a topological order:
//   for each of its frames: the block-statistics tasks, then the region task;
//   then for each: the depth-filter tasks, then the warp tasks.
// A task is four 256-px-wide block-statistics tiles or four 64 x 32 filter
// tiles (four 256-lane groups), 1024/G image rows (warp: groups of G lanes),
// or the whole frame (region grouping: all 1024 lanes).  The smallest
// unfinished claimed task depends only on finished tasks and is some
// workgroup's current task, so the loop cannot deadlock whatever the number
// of resident workgroups.
// A task and the tasks it waits for run on one XCD, whose L2 all its CUs
// share: a producer waits until its stores are acknowledged (s_waitcnt 0)
// before counting, and a consumer invalidates its CU's L1 after seeing the
// count -- no agent-scope release or acquire, which on this part would write
// back or invalidate the whole L2 at every task.  A dependency wait is also
// bounded in wall-clock time: should one ever exceed it, the workgroup raises
// the abort word and every workgroup leaves its loop at its next claim or
// wait.
//
// Staged form (below the fused kernel): one launch per stage, each over all
// frames of the batch.
#include <hip/hip_runtime.h>

#include "body_depth.h"
#include "body_render.h"
#include "pstereo_batch.h"

namespace pstereo {

constexpr int kBatchThreads = 1024;
// task-index broadcast slot at the end of the dynamic LDS
constexpr size_t kBatchLdsBytes = kMaxLds;
constexpr size_t kBatchSlotOffset = kMaxLds - 16;

// Longest dependency wait, in ticks of the 100 MHz constant clock (1 s; a
// whole 64-frame batch takes a few milliseconds).
constexpr uint64_t kWaitLimitTicks = 100000000ull;

__device__ __forceinline__ uint32_t load_acquire(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t load_relaxed(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Lanes per row group and quads per lane of the warp stage for a row width.
// At most two quads per lane below 8K: the fused kernel runs 1024-lane
// workgroups, which caps a lane at 128 VGPRs for all stages together.
__host__ __device__ inline void warp_group(int w, int& group, int& quads) {
    const int q4 = (w + 3) / 4;
    if (q4 <= 256) { group = 256; quads = 1; }
    else if (q4 <= 512) { group = 256; quads = 2; }
    else if (q4 <= 1024) { group = 512; quads = 2; }
    else if (q4 <= 2048) { group = 1024; quads = 2; }
    else { group = 1024; quads = 4; }
}

// One task of each stage, as separate (not inlined) functions: each gets its
// own register allocation instead of the union of all four stages.
__device__ __noinline__ void task_blockstats(const FrameDesc* fp, int k, int items, int gx, uint32_t* lds) {
    const FrameDesc f = *fp;
    const int tid = threadIdx.x;
    const int g = tid >> 8, t = tid & 255;
    const int item = 4 * k + g;
    const bool active = item < items;
    const int tx = active ? item % gx : 0, ty = active ? item / gx : 0;
    switch (f.K) {
        case 2: bs_tile_k2(f, tx, ty, t, active); break;
        case 4: bs_tile<4, true>(f, tx, ty, t, lds + g * BsTile<4>::kLdsWords, active); break;
        case 8: bs_tile<8, true>(f, tx, ty, t, lds + g * BsTile<8>::kLdsWords, active); break;
        case 16: bs_tile<16, true>(f, tx, ty, t, lds + g * BsTile<16>::kLdsWords, active); break;
        case 32: bs_tile<32, true>(f, tx, ty, t, lds + g * BsTile<32>::kLdsWords, active); break;
        default: bs_tile<64, true>(f, tx, ty, t, lds + g * BsTile<64>::kLdsWords, active); break;
    }
}

__device__ __noinline__ void task_regions(const FrameDesc* fp, uint32_t* lds) {
    const FrameDesc f = *fp;
    regions_body(f, lds);
}

template <int R>
__device__ __noinline__ void task_cbf(const FrameDesc* fp, int k, int items, int gx, uint32_t* lds) {
    const FrameDesc f = *fp;
    const int tid = threadIdx.x;
    const int g = tid >> 8, t = tid & 255;
    const int item = 4 * k + g;
    const bool active = item < items;
    const int tx = active ? item % gx : 0, ty = active ? item / gx : 0;
    if (f.K == 2) cbf_tile<R, true, true>(f, tx, ty, t, lds + g * CbfTile<R>::kLdsWords, active);
    else cbf_tile<R, true>(f, tx, ty, t, lds + g * CbfTile<R>::kLdsWords, active);
}

__device__ __noinline__ void task_warp(const FrameDesc* fp, int k, uint32_t* lds) {
    const FrameDesc f = *fp;
    const int tid = threadIdx.x;
    int group, quads;
    warp_group(f.w, group, quads);
    const int per = kBatchThreads / group;
    const int g = tid / group, t = tid - g * group;
    const int y = per * k + g;
    const bool active = y < f.h;
    const size_t stride = (warp_lds_bytes(f.w, group, quads) + 15) / 16 * 16;
    uint32_t* l = reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(lds) + g * stride);
    if (quads == 1) warp_row<true, 1>(f, active ? y : 0, t, group, l, active);
    else if (quads == 2) warp_row<true, 2>(f, active ? y : 0, t, group, l, active);
    else warp_row<true, 4>(f, active ? y : 0, t, group, l, active);
}

template <int R>
__global__ void __launch_bounds__(kBatchThreads) k_batch(BatchDesc bd) {
    extern __shared__ uint32_t lds[];
    int* slot = reinterpret_cast<int*>(reinterpret_cast<uint8_t*>(lds) + kBatchSlotOffset);
    const int tid = threadIdx.x;
    // this workgroup's XCD, from the hardware register: it serves that XCD's
    // queue only
    const int q = (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kXcds - 1));
    const int ntask = bd.qntask[q];
    uint32_t* abort_word = bd.ctr + kXcds + 4 * bd.nframes;
    int seg = bd.qseg[q];
    // the next task is claimed while the current one runs
    if (tid == 0) slot[0] = (int)atomicAdd(&bd.ctr[q], 1u);
    __syncthreads();
    int task = slot[0];
    while (true) {
        __syncthreads();  // every lane has read slot[0]
        if (task >= ntask) break;
        uint32_t next = 0;
        if (tid == 0) next = load_relaxed(abort_word) ? (uint32_t)ntask : atomicAdd(&bd.ctr[q], 1u);
        while (task >= bd.segs[seg].first + bd.segs[seg].ntask) ++seg;
        const BatchSeg sg = bd.segs[seg];
        const FrameDesc* fp = bd.frames + sg.frame;
        const int k = task - sg.first;  // task index inside the segment
        // wait for the inputs of this phase of this frame: written on this
        // XCD by tasks that waited for their stores before counting, so they
        // are in this XCD's L2; this CU's L1 is invalidated before reading
        if (sg.phase > 0) {
            if (tid == 0) {
                const uint32_t* dep = &bd.ctr[kXcds + 4 * sg.frame + sg.phase - 1];
                const uint32_t need = (uint32_t)bd.need[4 * sg.frame + sg.phase - 1];
                const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
                int ok = 1;
                while (load_relaxed(dep) < need) {
                    if (load_relaxed(abort_word) || __builtin_amdgcn_s_memrealtime() - t0 > kWaitLimitTicks) {
                        __hip_atomic_store(abort_word, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                slot[1] = ok;
            }
            __syncthreads();
            if (!slot[1]) break;
            asm volatile("buffer_inv sc0" ::: "memory");
        }
        if (sg.phase == 0) task_blockstats(fp, k, sg.items, sg.gx, lds);
        else if (sg.phase == 1) task_regions(fp, lds);
        else if (sg.phase == 2) task_cbf<R>(fp, k, sg.items, sg.gx, lds);
        else task_warp(fp, k, lds);
        // publish: every lane's stores acknowledged by the L2, then one count
        // (warp tasks have no dependent task -- their outputs are read after
        // the kernel -- so their stores need not drain here)
        if (sg.phase < 3) __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) {
            if (sg.phase < 3)
                __hip_atomic_fetch_add(&bd.ctr[kXcds + 4 * sg.frame + sg.phase], 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            slot[0] = (int)next;
        }
        __syncthreads();
        task = slot[0];
    }
}

__global__ void k_batch_reset(uint32_t* ctr, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) ctr[i] = 0;
}

// ---------------------------------------------------------------------------
// Staged form: one launch per stage over the tiles (rows) of every frame of
// the batch.  first[] holds, per frame, the index of its first workgroup in
// the launch (non-decreasing, n + 1 entries); a workgroup finds its frame by
// binary search over that table (uniform, so scalar loads), then its tile.
// Kernel boundaries order the stages, so no workgroup ever waits on another.

__device__ __forceinline__ int frame_of(const int* first, int n, int idx) {
    int lo = 0, hi = n - 1;  // last f with first[f] <= idx
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= idx) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// LDS of the largest block-statistics tile over the block sizes and tile
// heights the staged form runs.
constexpr int kBsLdsMax = [] {
    const int w[] = {BsTile<4, 4>::kLdsWords,  BsTile<4, 8>::kLdsWords,   BsTile<4, 16>::kLdsWords,
                     BsTile<8, 4>::kLdsWords,  BsTile<8, 8>::kLdsWords,   BsTile<8, 16>::kLdsWords,
                     BsTile<16, 4>::kLdsWords, BsTile<16, 8>::kLdsWords,  BsTile<16, 16>::kLdsWords,
                     BsTile<32, 8>::kLdsWords, BsTile<32, 16>::kLdsWords, BsTile<64, 16>::kLdsWords};
    int m = 1;
    for (int x : w) m = x > m ? x : m;
    return m;
}();

// A block-statistics tile of rows th (16, 32 or 64, at least K).
template <int K>
__device__ __forceinline__ void bs_tile_rows_of(const FrameDesc& f, int th, int tx, int ty, uint32_t* lds) {
    if constexpr (K <= 16) {
        if (th == 16) {
            bs_tile<K, true, 4>(f, tx, ty, threadIdx.x, lds, true);
            return;
        }
    }
    if constexpr (K <= 32) {
        if (th == 32) {
            bs_tile<K, true, 8>(f, tx, ty, threadIdx.x, lds, true);
            return;
        }
    }
    bs_tile<K, true, 16>(f, tx, ty, threadIdx.x, lds, true);
}

// bs_rows: the tuned tile height (0 = each block size's default).
__global__ void __launch_bounds__(256) k_mf_blockstats(const FrameDesc* frames, const int* first, int n, int bs_rows) {
    __shared__ uint32_t lds[kBsLdsMax];
    const int idx = xcd_tile(blockIdx.x, gridDim.x);
    const int fi = frame_of(first, n, idx);
    const FrameDesc f = frames[fi];
    const int local = idx - first[fi];
    const int gx = (f.w + kBsTileW - 1) / kBsTileW;
    const int tx = local % gx, ty = local / gx;
    const int th = bs_tile_rows_tuned(f.K, bs_rows);
    switch (f.K) {
        case 2: bs_tile_k2(f, tx, ty, threadIdx.x, true); break;
        case 4: bs_tile_rows_of<4>(f, th, tx, ty, lds); break;
        case 8: bs_tile_rows_of<8>(f, th, tx, ty, lds); break;
        case 16: bs_tile_rows_of<16>(f, th, tx, ty, lds); break;
        case 32: bs_tile_rows_of<32>(f, th, tx, ty, lds); break;
        default: bs_tile_rows_of<64>(f, th, tx, ty, lds); break;
    }
}

__global__ void __launch_bounds__(kRegionThreads) k_mf_regions(const FrameDesc* frames) {
    extern __shared__ uint32_t lds[];
    const FrameDesc f = frames[blockIdx.x];
    regions_body(f, lds);
}

// K2: every frame of the batch has blocks of 2 px (the block size is shared).
template <int R, bool K2>
__global__ void __launch_bounds__(256) k_mf_cbf(const FrameDesc* frames, const int* first, int n) {
    __shared__ uint32_t lds[CbfTile<R>::kLdsWords];
    const int idx = xcd_tile(blockIdx.x, gridDim.x);
    const int fi = frame_of(first, n, idx);
    const FrameDesc f = frames[fi];
    const int local = idx - first[fi];
    const int gx = (f.w + kTileW - 1) / kTileW;
    cbf_tile<R, true, K2>(f, local % gx, local / gx, threadIdx.x, lds, true);
}

// `rows` consecutive image rows per workgroup, each row's loads issued
// during the previous one (four quads per lane: one row after another).
template <int Q>
__global__ void __launch_bounds__(1024) k_mf_warp(const FrameDesc* frames, const int* first, int n, int rows) {
    extern __shared__ uint32_t lds[];
    const int idx = blockIdx.x;
    const int fi = frame_of(first, n, idx);
    const FrameDesc f = frames[fi];
    const int y0 = (idx - first[fi]) * rows;
    if constexpr (Q < 4) {
        warp_rows<true, Q>(f, y0, min(y0 + rows, f.h), 1, threadIdx.x, blockDim.x, lds);
    } else {
        // the LDS state prepared once (each row restores it); lane offsets
        // recomputed per row rather than held across rows
        warp_prepare(f, f.w, threadIdx.x, blockDim.x, lds);
        __syncthreads();
        WarpRowIn<true, Q> in, unused;
        for (int k = 0; k < rows; ++k) {
            const int y = y0 + k;
            if (y >= f.h) break;
            const int t = opaque((int)threadIdx.x);
            warp_load<true, Q>(f, y, t, blockDim.x, in);
            warp_row_body<true, Q>(f, y, t, blockDim.x, lds, true, in, -1, unused);
        }
    }
}

// ---------------------------------------------------------------------------
// host side

hipError_t launch_staged(const FrameDesc* d_frames, const int* d_first, const StagedPlan& pl, hipStream_t s) {
    const int n = pl.n;
    const int* first_bs = d_first;
    const int* first_cbf = d_first + (n + 1);
    hipLaunchKernelGGL(k_mf_blockstats, dim3(pl.tiles_bs), dim3(256), 0, s, d_frames, first_bs, n, pl.bs_rows);
    hipLaunchKernelGGL(k_mf_regions, dim3(n), dim3(kRegionThreads), pl.regions_lds, s, d_frames);
    const void* cbf_fn;
    switch (pl.r) {
        case 0: cbf_fn = pl.k2 ? (const void*)&k_mf_cbf<0, true> : (const void*)&k_mf_cbf<0, false>; break;
        case 1: cbf_fn = pl.k2 ? (const void*)&k_mf_cbf<1, true> : (const void*)&k_mf_cbf<1, false>; break;
        case 2: cbf_fn = pl.k2 ? (const void*)&k_mf_cbf<2, true> : (const void*)&k_mf_cbf<2, false>; break;
        default: cbf_fn = pl.k2 ? (const void*)&k_mf_cbf<3, true> : (const void*)&k_mf_cbf<3, false>; break;
    }
    {
        void* args[] = {const_cast<FrameDesc**>(&d_frames), const_cast<int**>(&first_cbf), const_cast<int*>(&n)};
        hipError_t e = hipLaunchKernel(cbf_fn, dim3(pl.tiles_cbf), dim3(256), args, 0, s);
        if (e != hipSuccess) return e;
    }
    for (int c = 0; c < pl.nclass; ++c) {
        const int* fw = d_first + (size_t)(2 + c) * (n + 1);
        const dim3 g(pl.cls_rows[c]), b(pl.cls_threads[c]);
        switch (pl.cls_q[c]) {
            case 1: hipLaunchKernelGGL(k_mf_warp<1>, g, b, pl.cls_lds[c], s, d_frames, fw, n, pl.warp_rows); break;
            case 2: hipLaunchKernelGGL(k_mf_warp<2>, g, b, pl.cls_lds[c], s, d_frames, fw, n, pl.warp_rows); break;
            default: hipLaunchKernelGGL(k_mf_warp<4>, g, b, pl.cls_lds[c], s, d_frames, fw, n, pl.warp_rows); break;
        }
    }
    return hipGetLastError();
}

int batch_tasks(const FrameDesc& f, int phase, int* items, int* gx, int bs_rows) {
    switch (phase) {
        case 0: {
            const int th = bs_tile_rows_tuned(f.K, bs_rows);
            *gx = (f.w + kBsTileW - 1) / kBsTileW;
            *items = *gx * ((f.h + th - 1) / th);
            return (*items + 3) / 4;
        }
        case 1:
            *gx = 1;
            *items = 1;
            return 1;
        case 2:
            *gx = (f.w + kTileW - 1) / kTileW;
            *items = *gx * ((f.h + kTileH - 1) / kTileH);
            return (*items + 3) / 4;
        default: {
            int group, quads;
            warp_group(f.w, group, quads);
            const int per = kBatchThreads / group;
            *gx = 1;
            *items = f.h;
            return (f.h + per - 1) / per;
        }
    }
}

bool batch_width_ok(int w) {
    int group, quads;
    warp_group(w, group, quads);
    if ((w + 3) / 4 > group * quads) return false;
    return (size_t)(kBatchThreads / group) * ((warp_lds_bytes(w, group, quads) + 15) / 16 * 16) <= kBatchSlotOffset;
}

hipError_t prepare_batch_kernels() {
    hipError_t e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mf_regions), hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mf_warp<1>), hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mf_warp<2>), hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mf_warp<4>), hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch<0>), hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBatchLdsBytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch<1>), hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBatchLdsBytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch<2>), hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBatchLdsBytes)) != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch<3>), hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBatchLdsBytes);
}

hipError_t launch_batch(const BatchDesc& bd, int r, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(256), 0, s, bd.ctr, kXcds + 1 + 4 * bd.nframes);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (r) {
        case 0: hipLaunchKernelGGL(k_batch<0>, dim3(grid), dim3(kBatchThreads), kBatchLdsBytes, s, bd); break;
        case 1: hipLaunchKernelGGL(k_batch<1>, dim3(grid), dim3(kBatchThreads), kBatchLdsBytes, s, bd); break;
        case 2: hipLaunchKernelGGL(k_batch<2>, dim3(grid), dim3(kBatchThreads), kBatchLdsBytes, s, bd); break;
        default: hipLaunchKernelGGL(k_batch<3>, dim3(grid), dim3(kBatchThreads), kBatchLdsBytes, s, bd); break;
    }
    return hipGetLastError();
}

}  // namespace pstereo
