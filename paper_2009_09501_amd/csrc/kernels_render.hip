// gfx950 kernels of the stereo rendering (one frame per launch): the depth
// filter on 64 x 32 tiles and the per-row warp; the bodies live in
// body_render.h.
#include <hip/hip_runtime.h>

#include "body_render.h"

namespace pstereo {

template <int R, bool ALIGNED>
__global__ void __launch_bounds__(256) k_cbf(FrameDesc f) {
    __shared__ uint32_t lds[CbfTile<R>::kLdsWords];
    cbf_tile<R, ALIGNED>(f, blockIdx.x, blockIdx.y, threadIdx.x, lds, true);
}

template <bool ALIGNED, int Q>
__global__ void __launch_bounds__(1024) k_warp(FrameDesc f) {
    extern __shared__ uint32_t lds[];
    warp_row<ALIGNED, Q>(f, blockIdx.x, threadIdx.x, blockDim.x, lds, true);
}

// ---------------------------------------------------------------------------
// host-side launch helpers

bool warp_shape(int w, WarpShape* out) { return warp_shape_cap(w, 256, out); }

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
    return {reinterpret_cast<const void*>(&k_cbf<R, A>), dim3((f.w + kTileW - 1) / kTileW, (f.h + kTileH - 1) / kTileH),
            dim3(256), 0};
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

template <bool A>
static LaunchSpec warp_q(const FrameDesc& f, const WarpShape& ws) {
    const void* fn = ws.quads == 1 ? reinterpret_cast<const void*>(&k_warp<A, 1>)
                   : ws.quads == 2 ? reinterpret_cast<const void*>(&k_warp<A, 2>)
                   : ws.quads == 4 ? reinterpret_cast<const void*>(&k_warp<A, 4>) : nullptr;
    return {fn, dim3(f.h), dim3(ws.threads), ws.lds_bytes};
}

LaunchSpec spec_warp(const FrameDesc& f, const WarpShape& ws) { return f.aligned ? warp_q<true>(f, ws) : warp_q<false>(f, ws); }

template <bool A, int Q>
static hipError_t allow_lds() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_warp<A, Q>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
}

hipError_t prepare_render_kernels() {
    hipError_t e;
    if ((e = allow_lds<true, 1>()) != hipSuccess) return e;
    if ((e = allow_lds<true, 2>()) != hipSuccess) return e;
    if ((e = allow_lds<true, 4>()) != hipSuccess) return e;
    if ((e = allow_lds<false, 1>()) != hipSuccess) return e;
    if ((e = allow_lds<false, 2>()) != hipSuccess) return e;
    return allow_lds<false, 4>();
}

}  // namespace pstereo
