// Device helpers shared by the gfx950 kernels of the pseudo-stereo pipeline.
#pragma once

#include <hip/hip_runtime.h>

#include "pstereo_internal.h"

namespace pstereo {

// Range weights of the cross-bilateral filter: round(255 exp(-d^2 / (2 * 12^2)))
// for a luma difference d = 0..42, zero for larger d (range sigma 12).
__host__ __device__ constexpr uint32_t range_w(int d) {
    constexpr uint16_t t[43] = {255, 254, 251, 247, 241, 234, 225, 215, 204, 192, 180, 168, 155, 142, 129,
                                117, 105, 93,  83,  73,  64,  55,  47,  41,  35,  29,  24,  20,  17,  14,
                                11,  9,   7,   6,   5,   4,   3,   2,   2,   1,   1,   1,   1};
    return d < 43 ? t[d] : 0u;
}

// Spatial weights round(255 exp(-k / (2 * 1.5^2))) by squared distance k.
__host__ __device__ constexpr uint32_t spatial_w(int k) {
    return k == 0 ? 255 : k == 1 ? 204 : k == 2 ? 164 : k == 3 ? 131 : k == 4 ? 105
         : k == 5 ? 84 : k == 6 ? 67 : k == 7 ? 54 : k == 8 ? 43 : k == 9 ? 35
         : k == 10 ? 28 : k == 11 ? 22 : k == 12 ? 18 : k == 13 ? 14 : k == 14 ? 11
         : k == 15 ? 9 : k == 16 ? 7 : k == 17 ? 6 : 5;
}

// Luma guide: Q8 BT.601 weights summing to 256, rounded half up.
__device__ __forceinline__ int luma(int r, int g, int b) {
    return (77 * r + 150 * g + 29 * b + 128) >> 8;
}

// Exact floor(num / den) for num < 2^31, 0 < den < 2^22 and a quotient below
// 2^8: a single-precision reciprocal estimate is within 1 of the quotient,
// and one integer correction step makes it exact.
__device__ __forceinline__ uint32_t div_small_quotient(uint32_t num, uint32_t den) {
    const float qf = (float)num * __builtin_amdgcn_rcpf((float)den);
    int q = (int)qf;
    const int rem = (int)num - q * (int)den;
    if (rem < 0) --q;
    else if (rem >= (int)den) ++q;
    return (uint32_t)q;
}

// Row ramp of the region depth: 0 (far) at block row 0, 255 (near) at the
// bottom block row, rounded half up (quotient <= 255, so the reciprocal
// division above is exact).
__device__ __forceinline__ int ramp(int row, int gh) {
    return gh > 1 ? (int)div_small_quotient((uint32_t)(255 * row + (gh - 1) / 2), (uint32_t)(gh - 1)) : 0;
}

__device__ __forceinline__ int iabs(int v) { return v < 0 ? -v : v; }

// Four RGB24 pixels starting at p.  ALIGNED: the frame width is divisible by 4
// and the buffer is 4-byte aligned, so p is 4-byte aligned and all four pixels
// exist; otherwise n (0..4) pixels exist and are read bytewise.
template <bool ALIGNED>
__device__ __forceinline__ void load_quad(const uint8_t* p, int n, int (&r)[4], int (&g)[4], int (&b)[4]) {
    if constexpr (ALIGNED) {
        const uint3 v = *reinterpret_cast<const uint3*>(p);
        r[0] = v.x & 255;         g[0] = (v.x >> 8) & 255;  b[0] = (v.x >> 16) & 255;
        r[1] = v.x >> 24;         g[1] = v.y & 255;         b[1] = (v.y >> 8) & 255;
        r[2] = (v.y >> 16) & 255; g[2] = v.y >> 24;         b[2] = v.z & 255;
        r[3] = (v.z >> 8) & 255;  g[3] = (v.z >> 16) & 255; b[3] = v.z >> 24;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (j < n) { r[j] = p[3 * j]; g[j] = p[3 * j + 1]; b[j] = p[3 * j + 2]; }
            else { r[j] = g[j] = b[j] = 0; }
        }
    }
}

constexpr size_t kMaxLds = 160 * 1024;

// The value of v, opaque to the optimiser: indices derived from it are
// recomputed where they are used (or in each loop iteration) instead of being
// held in registers across the whole kernel.
__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Workgroups are dispatched to the 8 XCDs round-robin by linear workgroup id.
// Tile for workgroup bid of n: each XCD gets one contiguous run of tiles in
// raster order, so neighbouring tiles -- sharing halo rows and the 128-byte
// lines across tile borders -- meet in the same L2.  A bijection on [0, n).
__device__ __forceinline__ int xcd_tile(int bid, int n) {
    constexpr int X = 8;
    const int q = n / X, r = n - q * X;
    const int xcd = bid % X, idx = bid / X;
    return xcd * q + min(xcd, r) + idx;
}

}  // namespace pstereo
