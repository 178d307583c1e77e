// gfx950 kernels of the depth map: block statistics and region grouping.
//
// The depth map follows the paper's conversion scheme (Section 3, Fig. 1:
// the depth map is the first of the six components; Section 4: it is the
// "iterative" stage) built from block colour and edge cues (Section 2 and
// Table 1: edge / region-boundary information, block processing).  The exact
// cues, thresholds and region-depth rule are the library's readings.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace pstereo {

// ---------------------------------------------------------------------------
// k_blockstats: per K x K block, rounded mean colour and edge flag.
// Grid (ceil(ceil(w/4) / 256), gh), 256 lanes; lane q owns pixels 4q..4q+3 of
// the block row (K % 4 == 0, so a quad never straddles blocks) and walks the
// K rows, plus the first row of the next block row for the vertical steps.
// The K/4 lanes of one block combine by cross-lane xor reduction.
template <int K, bool ALIGNED>
__global__ void __launch_bounds__(256) k_blockstats(FrameDesc f) {
    const int W = f.w, H = f.h;
    const int by = blockIdx.y;
    const int q = blockIdx.x * 256 + threadIdx.x;
    const int x0 = 4 * q;
    const int yb = by * K;
    const int ye = min(yb + K, H);
    const int n = min(4, W - x0);
    uint32_t sr = 0, sg = 0, sb = 0;
    int edge = 0;
    if (x0 < W) {
        int prev[4] = {0, 0, 0, 0};
        // rows past the image bottom are predicated off (no break), so the
        // loop unrolls and all K+1 row loads are in flight together
#pragma unroll
        for (int i = 0; i <= K; ++i) {
            const int y = yb + i;
            if (y >= H) continue;
            const uint8_t* p = f.frame + ((size_t)y * W + x0) * 3;
            int r[4], g[4], b[4], Y[4];
            load_quad<ALIGNED>(p, n, r, g, b);
#pragma unroll
            for (int j = 0; j < 4; ++j) Y[j] = luma(r[j], g[j], b[j]);
            if (i > 0) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (j < n && iabs(Y[j] - prev[j]) > f.g) edge = 1;
            }
            if (i < K) {
                int ynext = 0;
                if (x0 + 4 < W) ynext = luma(p[12], p[13], p[14]);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (j < n) {
                        sr += r[j]; sg += g[j]; sb += b[j];
                        if (x0 + j + 1 < W) {
                            const int yn = j < 3 ? Y[j + 1] : ynext;
                            if (iabs(yn - Y[j]) > f.g) edge = 1;
                        }
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) prev[j] = Y[j];
        }
    }
    constexpr int G = K / 4;
#pragma unroll
    for (int o = G / 2; o >= 1; o >>= 1) {
        sr += __shfl_xor(sr, o);
        sg += __shfl_xor(sg, o);
        sb += __shfl_xor(sb, o);
        edge |= __shfl_xor(edge, o);
    }
    if (x0 < W && (q % G) == 0) {
        const int bx = q / G;
        if (bx < f.gw) {
            const int cnt = (min(bx * K + K, W) - bx * K) * (ye - yb);
            const uint32_t mr = (sr + cnt / 2) / cnt;
            const uint32_t mg = (sg + cnt / 2) / cnt;
            const uint32_t mb = (sb + cnt / 2) / cnt;
            f.stats[by * f.gw + bx] = mr | (mg << 8) | (mb << 16) | ((uint32_t)edge << 24);
        }
    }
}

// ---------------------------------------------------------------------------
// k_regions: region grouping, one workgroup of 1024 lanes per frame.
//
// Links join right / down neighbours that are both non-edge blocks and whose
// mean colours differ by at most tau (sum of absolute channel differences).
// A region is a connected component of the link graph; its label is its
// smallest block index.  Lane t owns the 32 contiguous blocks [32t, 32t+32).
//
//  1. link and edge bits of every block into LDS bitmaps;
//  2. row segments (maximal runs of right-linked blocks): a block-wide prefix
//     max of segment starts gives each block its segment; the parent array
//     starts as one star per segment;
//  3. lock-free union-find over the down links, only where the pair of
//     segments changes along the row; roots hook by a fixed pseudo-random
//     priority, so trees stay shallow whatever the order of the unions;
//  4. the smallest block index of every tree (atomic minimum at its root) is
//     the label; the parent array is then reused as the per-label block
//     count / background key and as the per-label lowest block row.
constexpr int kRegionThreads = 1024;
constexpr int kRegionPer = PSTEREO_MAX_BLOCKS / kRegionThreads;  // 32 blocks per lane

__device__ __forceinline__ uint32_t lds_load(const uint32_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
__device__ __forceinline__ void lds_store(uint32_t* p, uint32_t v) { __atomic_store_n(p, v, __ATOMIC_RELAXED); }

// Bijective 32-bit mix: distinct blocks get distinct hooking priorities.
__device__ __forceinline__ uint32_t hook_prio(uint32_t x) {
    x *= 0x9E3779B1u;
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    return x;
}

__device__ __forceinline__ int mean_l1(uint32_t s, uint32_t n) {
    return iabs((int)(s & 255) - (int)(n & 255)) + iabs((int)((s >> 8) & 255) - (int)((n >> 8) & 255)) +
           iabs((int)((s >> 16) & 255) - (int)((n >> 16) & 255));
}

// LDS index of block b in the parent array: one pad word every 32 blocks, so
// the 64 lanes of a wave, each at its own run of 32 blocks, hit 64 distinct
// banks instead of one.
__device__ __forceinline__ uint32_t pidx(uint32_t b) { return b + (b >> 5); }

__device__ __forceinline__ uint32_t uf_find_s(uint32_t* parent, uint32_t x) {
    while (true) {
        const uint32_t p = lds_load(&parent[pidx(x)]);
        if (p == x) return x;
        const uint32_t gp = lds_load(&parent[pidx(p)]);
        if (gp != p) lds_store(&parent[pidx(x)], gp);
        x = gp;
    }
}

__device__ __forceinline__ void uf_unite_s(uint32_t* parent, uint32_t a, uint32_t b) {
    while (true) {
        a = uf_find_s(parent, a);
        b = uf_find_s(parent, b);
        if (a == b) return;
        if (hook_prio(a) > hook_prio(b)) { const uint32_t t = a; a = b; b = t; }
        if (atomicCAS(&parent[pidx(a)], a, b) == a) return;
    }
}

__global__ void __launch_bounds__(kRegionThreads) k_regions(FrameDesc f) {
    extern __shared__ uint32_t lds[];
    const int gw = f.gw, gh = f.gh, nb = gw * gh;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    constexpr int NW = kRegionThreads / 64;
    uint32_t* parent = lds;                           // pidx(nb) words
    uint32_t* lrb = parent + pidx((uint32_t)nb) + 1;  // right-link bits, word j = blocks 32j..32j+31
    uint32_t* ldb = lrb + kRegionThreads;             // down-link bits
    uint32_t* eb = ldb + kRegionThreads;              // edge bits
    uint32_t* scan = eb + kRegionThreads;             // NW words
    uint32_t* misc = scan + NW;                       // [0]: background key

    // 1. link / edge bits, strided over the blocks so the loads coalesce; a
    // wave's 64 bits go to two bitmap words through ballots
#pragma unroll 8
    for (int i = 0; i < kRegionPer; ++i) {
        const int b = i * kRegionThreads + t;
        bool e = true, lr = false, ld = false;
        if (b < nb) {
            const uint32_t s = f.stats[b];
            parent[pidx(b)] = b;
            const int bx = b % gw;
            e = (s >> 24) != 0;
            if (!e && bx + 1 < gw) {
                const uint32_t n = f.stats[b + 1];
                lr = !(n >> 24) && mean_l1(s, n) <= f.tau;
            }
            if (!e && b + gw < nb) {
                const uint32_t n = f.stats[b + gw];
                ld = !(n >> 24) && mean_l1(s, n) <= f.tau;
            }
        }
        const unsigned long long mr = __ballot(lr), md = __ballot(ld), me = __ballot(e);
        if (lane == 0) {
            const int w0 = (i * kRegionThreads + wave * 64) >> 5;
            lrb[w0] = (uint32_t)mr; lrb[w0 + 1] = (uint32_t)(mr >> 32);
            ldb[w0] = (uint32_t)md; ldb[w0 + 1] = (uint32_t)(md >> 32);
            eb[w0] = (uint32_t)me; eb[w0 + 1] = (uint32_t)(me >> 32);
        }
    }
    if (t == 0) misc[0] = 0;
    __syncthreads();

    // from here on lane t owns the 32 contiguous blocks [32t, 32t+32)
    const int b0 = t * kRegionPer;
    const int nown = max(0, min(kRegionPer, nb - b0));
    const int bx0 = b0 % gw, by0 = b0 / gw;
    const uint32_t lr = lrb[t], ld = ldb[t], emask = eb[t];

    // 2. segments: start(b) = b is not right-linked from b - 1 (a row's first
    // block never is: the last block of a row has no right link)
    const uint32_t prev_lr = t > 0 ? lrb[t - 1] : 0u;
    const uint32_t linked_from_left = (lr << 1) | (prev_lr >> 31);
    const uint32_t own_mask = nown >= 32 ? 0xFFFFFFFFu : ((1u << nown) - 1u);
    const uint32_t starts = ~linked_from_left & own_mask;
    const int last_start = starts ? b0 + 31 - __clz(starts) : -1;
    int incl = last_start;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o);
        if (lane >= o) incl = max(incl, v);
    }
    if (lane == 63) scan[wave] = (uint32_t)(incl + 1);
    __syncthreads();
    int carry = __shfl_up(incl, 1);
    if (lane == 0) carry = -1;
    for (int v = 0; v < wave; ++v) carry = max(carry, (int)scan[v] - 1);
    uint32_t node[kRegionPer];  // segment, then root, then label of each owned block
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i) {
        if ((starts >> i) & 1u) carry = b0 + i;
        node[i] = (uint32_t)carry;
    }
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i)
        if (i < nown) parent[pidx(b0 + i)] = node[i];
    __syncthreads();

    // 3. unions across rows where the segment pair changes
    for (int i = 0; i < nown; ++i) {
        if (!((ld >> i) & 1u)) continue;
        const int b = b0 + i;
        if (i > 0 && ((ld >> (i - 1)) & 1u) && ((lr >> (i - 1)) & 1u)) {
            // b - 1 and b share a segment and both link down; skip when the
            // blocks below are right-linked too (same lower segment)
            const int c = b + gw - 1;
            if ((lrb[c >> 5] >> (c & 31)) & 1u) continue;
        }
        uf_unite_s(parent, (uint32_t)b, (uint32_t)(b + gw));
    }
    __syncthreads();

#pragma unroll
    for (int i = 0; i < kRegionPer; ++i)
        if (i < nown) node[i] = uf_find_s(parent, b0 + i);
    __syncthreads();

    // 4. label = smallest block index of the tree, kept at the root as 0x10000 | min
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i)
        if (i < nown && node[i] == (uint32_t)(b0 + i)) parent[pidx(b0 + i)] = 0xFFFFFFFFu;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i)
        if (i < nown && (i == 0 || node[i] != node[i - 1]))
            atomicMin(&parent[pidx(node[i])], 0x10000u | (uint32_t)(b0 + i));
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i)
        if (i < nown) node[i] = parent[pidx(node[i])] & 0xFFFFu;
    __syncthreads();

    // background key per label: (non-edge block count << 16) | (0xFFFF - label);
    // the largest key is the largest region, ties to the smaller label
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i)
        if (i < nown) parent[pidx(b0 + i)] = 0;
    __syncthreads();
    {
        uint32_t run = 0;
#pragma unroll
        for (int i = 0; i < kRegionPer; ++i) {
            if (i >= nown) break;
            if (!((emask >> i) & 1u)) ++run;
            const bool flush = i + 1 == nown || i + 1 == kRegionPer || node[i + 1 < kRegionPer ? i + 1 : i] != node[i];
            if (flush && run) {
                atomicAdd(&parent[pidx(node[i])], run << 16);
                atomicOr(&parent[pidx(node[i])], 0xFFFFu - node[i]);
            }
            if (flush) run = 0;
        }
    }
    __syncthreads();
    uint32_t best = 0;
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i)
        if (i < nown) best = max(best, parent[pidx(b0 + i)]);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) best = max(best, (uint32_t)__shfl_xor((int)best, o));
    if (lane == 0 && best) atomicMax(&misc[0], best);
    __syncthreads();
    const uint32_t bgkey = misc[0];
    const int bg = bgkey ? (int)(0xFFFFu - (bgkey & 0xFFFFu)) : -1;

    // lowest block row (+1) per label
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i)
        if (i < nown) parent[pidx(b0 + i)] = 0;
    __syncthreads();
    {
        int by = by0, bx = bx0;
#pragma unroll
        for (int i = 0; i < kRegionPer; ++i) {
            if (i >= nown) break;
            if (!((emask >> i) & 1u)) atomicMax(&parent[pidx(node[i])], (uint32_t)(by + 1));
            if (++bx == gw) { bx = 0; ++by; }
        }
    }
    __syncthreads();

    // region depth: background and edge blocks follow the row ramp, any other
    // region sits at the ramp of its lowest block row (ground contact)
    {
        int by = by0, bx = bx0;
#pragma unroll
        for (int i = 0; i < kRegionPer; ++i) {
            if (i >= nown) break;
            const int b = b0 + i;
            int d;
            if (((emask >> i) & 1u) || (int)node[i] == bg) d = ramp(by, gh);
            else d = ramp((int)parent[pidx(node[i])] - 1, gh);
            f.binfo[b] = make_uint2(f.stats[b], (uint32_t)d);
            f.labels[b] = (int32_t)node[i];
            if (++bx == gw) { bx = 0; ++by; }
        }
    }
}

// ---------------------------------------------------------------------------
// host-side launch helpers

template <int K, bool A>
static hipError_t bs_launch(const FrameDesc& f, hipStream_t s) {
    dim3 grid(((f.w + 3) / 4 + 255) / 256, f.gh);
    hipLaunchKernelGGL((k_blockstats<K, A>), grid, dim3(256), 0, s, f);
    return hipGetLastError();
}

template <bool A>
static hipError_t bs_dispatch(const FrameDesc& f, hipStream_t s) {
    switch (f.K) {
        case 4: return bs_launch<4, A>(f, s);
        case 8: return bs_launch<8, A>(f, s);
        case 16: return bs_launch<16, A>(f, s);
        case 32: return bs_launch<32, A>(f, s);
        case 64: return bs_launch<64, A>(f, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_blockstats(const FrameDesc& f, hipStream_t s) {
    return f.aligned ? bs_dispatch<true>(f, s) : bs_dispatch<false>(f, s);
}

size_t regions_lds_bytes(int nb) {
    return (size_t)(nb + nb / 32 + 1 + 3 * kRegionThreads + kRegionThreads / 64 + 4) * 4;
}

hipError_t launch_regions(const FrameDesc& f, hipStream_t s) {
    const int nb = f.gw * f.gh;
    hipLaunchKernelGGL(k_regions, dim3(1), dim3(kRegionThreads), regions_lds_bytes(nb), s, f);
    return hipGetLastError();
}

hipError_t prepare_depth_kernels() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_regions),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
}

}  // namespace pstereo
