// gfx950 kernels of the stereo rendering (one frame per launch): the depth
// filter on 64 x 32 tiles and the per-row warp; the bodies live in
// body_render.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

#include "body_render.h"

namespace pstereo {

// The warp's start mark (three-stage pipelined calls), stored by the first
// lane of the first workgroup: the kernel runs only once all earlier work on
// its stream is done.
__device__ __forceinline__ void warp_start_mark(const FrameDesc& f) {
    if (f.wmark && blockIdx.x == 0 && threadIdx.x == 0)
        __hip_atomic_store(f.wmark, f.wmark_value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <int R, bool ALIGNED, bool K2>
__global__ void __launch_bounds__(256) k_cbf(FrameDesc f) {
    __shared__ uint32_t lds[CbfTile<R>::kLdsWords];
    // the start mark of a pipelined call: this kernel runs only once all
    // earlier work on its stream is done (a system-scope store that a
    // stream's wait-value packet polls; it publishes no data)
    if (f.mark && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0)
        __hip_atomic_store(f.mark, f.mark_value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    const int gx = gridDim.x;
    const int tile = xcd_tile(blockIdx.y * gx + blockIdx.x, gx * gridDim.y);
    const int ty = tile / gx;
    cbf_tile<R, ALIGNED, K2>(f, tile - ty * gx, ty, threadIdx.x, lds, true);
}

// Rows blockIdx.x, blockIdx.x + gridDim.x, ...: a grid of at most a few
// workgroups per CU walks the rows, loading each next row during the current
// one.
template <bool ALIGNED, int Q>
__global__ void __launch_bounds__(512) k_warp(FrameDesc f) {
    extern __shared__ uint32_t lds[];
    warp_start_mark(f);
    warp_rows<ALIGNED, Q>(f, blockIdx.x, f.h, gridDim.x, threadIdx.x, blockDim.x, lds);
}

// Rows needing four quads per lane (wider than 4096 px): one row per
// workgroup of up to 1024 lanes (a second row's prefetched share would not
// fit the register budget).
template <bool ALIGNED>
__global__ void __launch_bounds__(1024) k_warp_wide(FrameDesc f) {
    extern __shared__ uint32_t lds[];
    warp_start_mark(f);
    warp_row<ALIGNED, 4>(f, blockIdx.x, threadIdx.x, blockDim.x, lds, true);
}

template <bool ALIGNED>
__global__ void __launch_bounds__(256) k_gather(FrameDesc f) {
    extern __shared__ uint32_t lds[];
    warp_start_mark(f);
    gather_row<ALIGNED>(f, blockIdx.x, threadIdx.x, blockDim.x, lds);
}

__global__ void k_inpaint_reset(FrameDesc f) {
    for (int i = threadIdx.x; i <= kMaxSweeps; i += blockDim.x) f.ipn[i] = i == 0 ? 1u : 0u;
}

// Sweep `sweep` over both views (blockIdx.y); nothing to do once the
// previous sweep filled no pixel.
__global__ void __launch_bounds__(256) k_inpaint_sweep(FrameDesc f, int sweep) {
    if (f.ipn[sweep - 1] == 0) return;
    const int W = f.w;
    const int q = blockIdx.x * 256 + threadIdx.x;
    const int qw = (W + 3) >> 2;
    int filled = 0;
    if (q < qw * f.h) {
        const int y = q / qw, x0 = 4 * (q - y * qw);
        for (int j = 0; j < 4 && x0 + j < W; ++j) filled += inpaint_pixel(f, blockIdx.y, x0 + j, y, sweep);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) filled += __shfl_xor(filled, o);
    if ((threadIdx.x & 63) == 0 && filled) atomicAdd(&f.ipn[sweep], (uint32_t)filled);
}

// The views from the inpainted colours (pixels never filled keep their own
// source pixel), then the anaglyph and the half side-by-side frame.
template <bool ALIGNED>
__global__ void __launch_bounds__(256) k_inpaint_final(FrameDesc f) {
    const int W = f.w;
    const int q = blockIdx.x * 256 + threadIdx.x;
    const int qw = (W + 3) >> 2;
    if (q >= qw * f.h) return;
    const int y = q / qw, x0 = 4 * (q - y * qw);
    const size_t plane = (size_t)W * f.h;
    uint32_t cl[4] = {0, 0, 0, 0}, cr[4] = {0, 0, 0, 0};
    for (int j = 0; j < 4 && x0 + j < W; ++j) {
        const size_t o = (size_t)y * W + x0 + j;
        const uint8_t* sp = f.frame + o * 3;
        const uint32_t src = sp[0] | ((uint32_t)sp[1] << 8) | ((uint32_t)sp[2] << 16);
        cl[j] = f.ipt[o] == 0xFFFF ? src : f.ipc[o];
        cr[j] = f.ipt[plane + o] == 0xFFFF ? src : f.ipc[plane + o];
    }
    store_quad_views<ALIGNED>(f, y, x0, cl, cr);
}

// ---------------------------------------------------------------------------
// host-side launch helpers

// The plain path: up to 512 lanes per row (two quads per lane from 2048 px)
// before four quads per lane.
bool warp_shape(int w, WarpShape* out) { return warp_shape_cap(w, 512, out); }

bool warp_shape_cap(int w, int cap, WarpShape* out) {
    const int quads = (w + 3) / 4;
    int q = 1;
    while (q < 4 && (quads + q - 1) / q > cap) q *= 2;
    int threads = ((quads + q - 1) / q + 63) / 64 * 64;
    if (threads > 1024) return false;
    const size_t lds = warp_lds_bytes(w, threads, q);
    if (lds > kMaxLds) return false;
    out->threads = threads;
    out->quads = q;
    out->lds_bytes = lds;
    return true;
}

template <int R, bool A>
static LaunchSpec cbf_spec(const FrameDesc& f) {
    // blocks of 2 px take their raw depth per pixel from global memory (an
    // external depth map needs no block lookups at all)
    const void* fn = (f.K == 2 && !f.depth_in) ? reinterpret_cast<const void*>(&k_cbf<R, A, true>)
                                                 : reinterpret_cast<const void*>(&k_cbf<R, A, false>);
    return {fn, dim3((f.w + kTileW - 1) / kTileW, (f.h + kTileH - 1) / kTileH), dim3(256), 0};
}

template <bool A>
static LaunchSpec cbf_r(const FrameDesc& f) {
    switch (f.r) {
        case 0: return cbf_spec<0, A>(f);
        case 1: return cbf_spec<1, A>(f);
        case 2: return cbf_spec<2, A>(f);
        case 3: return cbf_spec<3, A>(f);
        default: return {nullptr, dim3(), dim3(), 0};
    }
}

LaunchSpec spec_cbf(const FrameDesc& f) { return f.aligned ? cbf_r<true>(f) : cbf_r<false>(f); }

// VGPRs per lane of k_warp<aligned, quads 1 / 2>, read at preparation (every
// context stores the same values).
static std::atomic<int> g_warp_vgprs[2][2] = {{128, 128}, {128, 128}};

template <bool A>
static LaunchSpec warp_q(const FrameDesc& f, const WarpShape& ws) {
    if (ws.quads == 4)
        return {reinterpret_cast<const void*>(&k_warp_wide<A>), dim3(f.h), dim3(ws.threads), ws.lds_bytes};
    const void* fn = ws.quads == 1 ? reinterpret_cast<const void*>(&k_warp<A, 1>)
                   : ws.quads == 2 ? reinterpret_cast<const void*>(&k_warp<A, 2>) : nullptr;
    // resident workgroups per CU by LDS, lanes and registers (512 VGPRs per
    // SIMD lane in steps of 8, at most 8 waves per SIMD, a workgroup's waves
    // spread over the 4 SIMDs), times 256 CUs; every workgroup gets a row
    const int regs = (g_warp_vgprs[A ? 1 : 0][ws.quads == 1 ? 0 : 1].load(std::memory_order_relaxed) + 7) / 8 * 8;
    const int waves_simd = std::min(8, 512 / std::max(regs, 8));
    const int by_regs = std::max(1, waves_simd / ((ws.threads / 64 + 3) / 4));
    const int by_lds = std::max(1, (int)(kMaxLds / std::max<size_t>(ws.lds_bytes, 1)));
    const int by_lanes = std::max(1, 2048 / ws.threads);
    const int resident = std::min(std::min(by_lds, by_lanes), by_regs) * 256;
    return {fn, dim3(std::min(f.h, resident)), dim3(ws.threads), ws.lds_bytes};
}

LaunchSpec spec_warp(const FrameDesc& f, const WarpShape& ws) { return f.aligned ? warp_q<true>(f, ws) : warp_q<false>(f, ws); }

bool gather_fits(int w) { return gather_lds_bytes(w) <= kMaxLds; }

static dim3 quad_grid(const FrameDesc& f, int views) {
    const long long quads = (long long)((f.w + 3) / 4) * f.h;
    return dim3((unsigned)((quads + 255) / 256), views);
}

hipError_t launch_inpaint_reset(const FrameDesc& f, hipStream_t s) {
    hipLaunchKernelGGL(k_inpaint_reset, dim3(1), dim3(256), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_inpaint_sweep(const FrameDesc& f, int sweep, hipStream_t s) {
    hipLaunchKernelGGL(k_inpaint_sweep, quad_grid(f, 2), dim3(256), 0, s, f, sweep);
    return hipGetLastError();
}

hipError_t launch_inpaint_final(const FrameDesc& f, hipStream_t s) {
    if (f.aligned) hipLaunchKernelGGL(k_inpaint_final<true>, quad_grid(f, 1), dim3(256), 0, s, f);
    else hipLaunchKernelGGL(k_inpaint_final<false>, quad_grid(f, 1), dim3(256), 0, s, f);
    return hipGetLastError();
}

LaunchSpec spec_gather(const FrameDesc& f) {
    const void* fn = f.aligned ? reinterpret_cast<const void*>(&k_gather<true>)
                               : reinterpret_cast<const void*>(&k_gather<false>);
    return {fn, dim3(f.h), dim3(256), gather_lds_bytes(f.w)};
}

template <bool A>
static hipError_t allow_lds_wide() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_warp_wide<A>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
}

template <bool A, int Q>
static hipError_t allow_lds() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_warp<A, Q>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
}

template <bool A, int Q>
static hipError_t read_warp_vgprs() {
    hipFuncAttributes a;
    const hipError_t e = hipFuncGetAttributes(&a, reinterpret_cast<const void*>(&k_warp<A, Q>));
    if (e == hipSuccess && a.numRegs > 0)
        g_warp_vgprs[A ? 1 : 0][Q == 1 ? 0 : 1].store(a.numRegs, std::memory_order_relaxed);
    return e;
}

hipError_t prepare_render_kernels() {
    hipError_t e;
    if ((e = read_warp_vgprs<true, 1>()) != hipSuccess) return e;
    if ((e = read_warp_vgprs<true, 2>()) != hipSuccess) return e;
    if ((e = read_warp_vgprs<false, 1>()) != hipSuccess) return e;
    if ((e = read_warp_vgprs<false, 2>()) != hipSuccess) return e;
    if ((e = allow_lds<true, 1>()) != hipSuccess) return e;
    if ((e = allow_lds<true, 2>()) != hipSuccess) return e;
    if ((e = allow_lds<false, 1>()) != hipSuccess) return e;
    if ((e = allow_lds<false, 2>()) != hipSuccess) return e;
    if ((e = allow_lds_wide<true>()) != hipSuccess) return e;
    if ((e = allow_lds_wide<false>()) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gather<true>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds)) != hipSuccess)
        return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gather<false>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
}

}  // namespace pstereo
