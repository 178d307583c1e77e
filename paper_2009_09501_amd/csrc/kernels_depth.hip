// gfx950 kernels of the depth map: block statistics and region grouping (one
// frame per launch); the stage bodies live in body_depth.h.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "body_depth.h"

namespace pstereo {

template <int K, bool ALIGNED>
__global__ void __launch_bounds__(256) k_blockstats(FrameDesc f) {
    __shared__ uint32_t lds[BsTile<K>::kLdsWords];
    const int gx = gridDim.x;
    const int tile = xcd_tile(blockIdx.y * gx + blockIdx.x, gx * gridDim.y);
    const int ty = tile / gx;
    bs_tile<K, ALIGNED>(f, tile - ty * gx, ty, threadIdx.x, lds, true);
}

__global__ void __launch_bounds__(256) k_blockstats_k2(FrameDesc f) {
    bs_tile_k2(f, blockIdx.x, blockIdx.y, threadIdx.x, true);
}

// The signal of a finished depth map (pipelined calls; the kernel is one
// workgroup): every wave waits until its stores are acknowledged, then one
// lane's system-scope release store (which writes the L2 back first) sets the
// word a stream's wait-value packet polls, so the kernels that packet releases
// read the whole depth map from any XCD.
__device__ __forceinline__ void signal_done(const FrameDesc& f) {
    if (!f.sig) return;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(f.sig, f.sig_value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void __launch_bounds__(kRegionThreads) k_regions(FrameDesc f) {
    extern __shared__ uint32_t lds[];
    regions_body(f, lds);
    signal_done(f);
}

__global__ void __launch_bounds__(kStripLanes) k_rg_strip(FrameDesc f) {
    __shared__ uint32_t lds[rg_strip_lds_words()];
    rg_strip_body(f, blockIdx.x, lds);
}

__global__ void __launch_bounds__(kStripLanes) k_rg_merge(FrameDesc f) {
    extern __shared__ uint32_t lds[];
    rg_merge_body(f, lds);
    signal_done(f);
}

__global__ void __launch_bounds__(256) k_rg_final(FrameDesc f) { rg_final_block(f, blockIdx.x * 256 + threadIdx.x); }

__global__ void __launch_bounds__(64) k_clear_words(uint32_t* p, int n) {
    for (int i = threadIdx.x; i < n; i += 64) p[i] = 0u;
}

// Whether two streams run beside each other.  k_probe_wait, launched on one
// stream, waits -- bounded in wall-clock time (s_memrealtime counts at
// 100 MHz) and in iterations, so it always ends -- for k_probe_post, launched
// on the other stream after it, to store `token` to w[0]; it then stores 1 to
// w[1] if it saw that store, 2 if its time ran out.  Streams that share a
// hardware queue run the two one after the other, so the wait runs out.
__global__ void __launch_bounds__(64) k_probe_wait(unsigned long long* w, unsigned long long token,
                                                   unsigned long long limit_ticks) {
    if (threadIdx.x != 0) return;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    unsigned long long seen = 2;
    for (int i = 0; i < (1 << 16); ++i) {
        if (__hip_atomic_load(&w[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) == token) {
            seen = 1;
            break;
        }
        if (__builtin_amdgcn_s_memrealtime() - t0 > limit_ticks) break;
        __builtin_amdgcn_s_sleep(2);
    }
    __hip_atomic_store(&w[1], seen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void __launch_bounds__(64) k_probe_post(unsigned long long* w, unsigned long long token) {
    if (threadIdx.x == 0) __hip_atomic_store(&w[0], token, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The end of the kernels before it on its stream, as a word a wait-value
// packet polls: it runs once they are done and their stores written back.
__global__ void __launch_bounds__(64) k_signal(unsigned long long* p, unsigned long long v) {
    if (threadIdx.x == 0) __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ---------------------------------------------------------------------------
// host-side launch helpers

template <int K, bool A>
static LaunchSpec bs_spec(const FrameDesc& f) {
    return {reinterpret_cast<const void*>(&k_blockstats<K, A>),
            dim3((f.w + kBsTileW - 1) / kBsTileW, (f.h + BsTile<K>::TH - 1) / BsTile<K>::TH), dim3(256), 0};
}

template <bool A>
static LaunchSpec bs_k(const FrameDesc& f) {
    switch (f.K) {
        case 2:
            return {reinterpret_cast<const void*>(&k_blockstats_k2),
                    dim3((f.w + kBsTileW - 1) / kBsTileW, (f.h + 63) / 64), dim3(256), 0};
        case 4: return bs_spec<4, A>(f);
        case 8: return bs_spec<8, A>(f);
        case 16: return bs_spec<16, A>(f);
        case 32: return bs_spec<32, A>(f);
        case 64: return bs_spec<64, A>(f);
        default: return {nullptr, dim3(), dim3(), 0};
    }
}

LaunchSpec spec_blockstats(const FrameDesc& f) { return f.aligned ? bs_k<true>(f) : bs_k<false>(f); }

size_t regions_lds_bytes(int nb) { return regions_lds_bytes_c(nb); }

LaunchSpec spec_regions(const FrameDesc& f) {
    return {reinterpret_cast<const void*>(&k_regions), dim3(1), dim3(kRegionThreads), regions_lds_bytes(f.gw * f.gh)};
}

// Rows per strip: about one block per lane (two for rows wider than the
// workgroup), 0 when a row does not fit a strip.
int strip_rows(int gw) {
    if (gw < 1 || gw > kStripBlocks) return 0;
    return gw <= kStripLanes ? kStripLanes / gw : 1;
}

LaunchSpec spec_rg_strip(const FrameDesc& f) {
    return {reinterpret_cast<const void*>(&k_rg_strip), dim3((f.gh + f.rstrip - 1) / f.rstrip), dim3(kStripLanes), 0};
}

LaunchSpec spec_rg_merge(const FrameDesc& f) {
    const size_t lds = std::max(rg_merge_lds_words() * 4, regions_lds_bytes(f.gw * f.gh));
    return {reinterpret_cast<const void*>(&k_rg_merge), dim3(1), dim3(kStripLanes), lds};
}

LaunchSpec spec_rg_final(const FrameDesc& f) {
    return {reinterpret_cast<const void*>(&k_rg_final), dim3((f.gw * f.gh + 255) / 256), dim3(256), 0};
}

hipError_t launch_clear_words(uint32_t* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_probe(unsigned long long* w, unsigned long long token, hipStream_t wait_on, hipStream_t post_on) {
    // 300 us: far beyond the start-up latency of a kernel on an idle stream
    hipLaunchKernelGGL(k_probe_wait, dim3(1), dim3(64), 0, wait_on, w, token, 30000ull);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_probe_post, dim3(1), dim3(64), 0, post_on, w, token);
    return hipGetLastError();
}

hipError_t launch_signal(unsigned long long* p, unsigned long long v, hipStream_t s) {
    hipLaunchKernelGGL(k_signal, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

hipError_t prepare_depth_kernels() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_regions),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rg_merge), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kMaxLds);
}

}  // namespace pstereo
