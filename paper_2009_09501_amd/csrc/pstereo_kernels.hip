// gfx950 kernels of the pseudo-stereo DIBR pipeline.
//
// Three kernels per frame, all integer arithmetic:
//   k_blockstats  block means + edge flags of the depth cues (one pass over
//                 the frame, quads of 4 pixels per lane, lane-group reduction)
//   k_regions     region grouping (connected components of linked blocks by
//                 lock-free union-find in LDS), region sizes, background pick
//                 and region depth, in one workgroup
//   k_render      fused row renderer: luma + pixel depth into an LDS ring of
//                 2r+1 rows, cross-bilateral filter, depth -> shift table,
//                 z-buffered forward warp of both views with LDS atomics on
//                 packed (depth, source x) keys, hole fill by workgroup
//                 prefix / suffix scans, anaglyph composition and RGB24 stores
//
// The stage definitions follow the paper's conversion scheme (Section 3,
// Fig. 1; Section 4, seven steps) and the depth -> shift rule of the Fig. 3
// code; the constants the paper leaves open are the library's readings and
// are stated at their point of use.
#include <hip/hip_runtime.h>

#include <climits>

#include "pstereo_internal.h"

namespace pstereo {

// Range weights of the cross-bilateral filter: round(255 exp(-d^2 / (2 * 12^2)))
// for a luma difference d = 0..42, zero for larger d (range sigma 12).
__constant__ uint16_t c_range_w[43] = {
    255, 254, 251, 247, 241, 234, 225, 215, 204, 192, 180, 168, 155, 142, 129,
    117, 105, 93,  83,  73,  64,  55,  47,  41,  35,  29,  24,  20,  17,  14,
    11,  9,   7,   6,   5,   4,   3,   2,   2,   1,   1,   1,   1};

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

// Row ramp of the region depth: 0 (far) at block row 0, 255 (near) at the
// bottom block row, rounded half up.
__device__ __forceinline__ int ramp(int row, int gh) {
    return gh > 1 ? (255 * row + (gh - 1) / 2) / (gh - 1) : 0;
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

template <bool ALIGNED>
__device__ __forceinline__ void store_quad(uint8_t* p, int n, const int (&r)[4], const int (&g)[4], const int (&b)[4]) {
    if constexpr (ALIGNED) {
        uint3 v;
        v.x = r[0] | (g[0] << 8) | (b[0] << 16) | (r[1] << 24);
        v.y = g[1] | (b[1] << 8) | (r[2] << 16) | (g[2] << 24);
        v.z = b[2] | (r[3] << 8) | (g[3] << 16) | (b[3] << 24);
        *reinterpret_cast<uint3*>(p) = v;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (j < n) { p[3 * j] = r[j]; p[3 * j + 1] = g[j]; p[3 * j + 2] = b[j]; }
        }
    }
}

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
#pragma unroll
        for (int i = 0; i <= K; ++i) {
            const int y = yb + i;
            if (y >= H) break;
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
// k_regions: one workgroup of 1024 lanes per frame.
//
// Links: right / down neighbours that are both non-edge blocks and whose mean
// colours differ by at most tau (sum of absolute channel differences).
// Components: lock-free union-find in LDS, always hooking the larger root
// under the smaller, so every component's final root is its smallest block
// index (the region label), whatever the order of the unions.  The parent
// array then serves as the per-label block counter and afterwards as the
// per-label lowest block row.
constexpr int kRegionThreads = 1024;
constexpr int kRegionPer = PSTEREO_MAX_BLOCKS / kRegionThreads;  // blocks per lane

__device__ __forceinline__ uint32_t lds_load(const uint32_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
__device__ __forceinline__ void lds_store(uint32_t* p, uint32_t v) { __atomic_store_n(p, v, __ATOMIC_RELAXED); }

__device__ __forceinline__ uint32_t uf_find(uint32_t* parent, uint32_t x) {
    // path halving; every write stores an ancestor, so the forest stays valid
    while (true) {
        const uint32_t p = lds_load(&parent[x]);
        if (p == x) return x;
        const uint32_t gp = lds_load(&parent[p]);
        if (gp != p) lds_store(&parent[x], gp);
        x = gp;
    }
}

__device__ __forceinline__ void uf_unite(uint32_t* parent, uint32_t a, uint32_t b) {
    while (true) {
        a = uf_find(parent, a);
        b = uf_find(parent, b);
        if (a == b) return;
        if (a < b) { const uint32_t t = a; a = b; b = t; }
        if (atomicCAS(&parent[a], a, b) == a) return;
    }
}

__device__ __forceinline__ int mean_l1(uint32_t s, uint32_t n) {
    return iabs((int)(s & 255) - (int)(n & 255)) + iabs((int)((s >> 8) & 255) - (int)((n >> 8) & 255)) +
           iabs((int)((s >> 16) & 255) - (int)((n >> 16) & 255));
}

__global__ void __launch_bounds__(kRegionThreads) k_regions(FrameDesc f) {
    extern __shared__ uint32_t lds[];
    const int gw = f.gw, gh = f.gh, nb = gw * gh;
    const int t = threadIdx.x;
    uint32_t* parent = lds;                    // nb words
    uint32_t* links = parent + nb;             // 2 bits per block, 16 blocks per word
    uint32_t* misc = links + (nb + 15) / 16;   // [0]: background key
    const int nlw = (nb + 15) / 16;

    uint32_t st[kRegionPer];
    uint32_t lab[kRegionPer];
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i) {
        const int b = t + i * kRegionThreads;
        st[i] = b < nb ? f.stats[b] : (1u << 24);
        if (b < nb) parent[b] = b;
    }
    for (int i = t; i < nlw; i += kRegionThreads) links[i] = 0;
    if (t == 0) misc[0] = 0;
    __syncthreads();

#pragma unroll
    for (int i = 0; i < kRegionPer; ++i) {
        const int b = t + i * kRegionThreads;
        if (b >= nb || (st[i] >> 24)) continue;
        const int bx = b % gw, by = b / gw;
        uint32_t bits = 0;
        if (bx + 1 < gw) {
            const uint32_t nbr = f.stats[b + 1];
            if (!(nbr >> 24) && mean_l1(st[i], nbr) <= f.tau) bits |= 1;
        }
        if (by + 1 < gh) {
            const uint32_t nbr = f.stats[b + gw];
            if (!(nbr >> 24) && mean_l1(st[i], nbr) <= f.tau) bits |= 2;
        }
        if (bits) atomicOr(&links[b >> 4], bits << ((b & 15) * 2));
    }
    __syncthreads();

#pragma unroll
    for (int i = 0; i < kRegionPer; ++i) {
        const int b = t + i * kRegionThreads;
        if (b >= nb) continue;
        const uint32_t bits = (links[b >> 4] >> ((b & 15) * 2)) & 3;
        if (bits & 1) uf_unite(parent, b, b + 1);
        if (bits & 2) uf_unite(parent, b, b + gw);
    }
    __syncthreads();

#pragma unroll
    for (int i = 0; i < kRegionPer; ++i) {
        const int b = t + i * kRegionThreads;
        lab[i] = b < nb ? uf_find(parent, b) : 0;
    }
    __syncthreads();

    // block count per label (non-edge blocks only)
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i) {
        const int b = t + i * kRegionThreads;
        if (b < nb) parent[b] = 0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i) {
        const int b = t + i * kRegionThreads;
        if (b < nb && !(st[i] >> 24)) atomicAdd(&parent[lab[i]], 1u);
    }
    __syncthreads();

    // background: the largest region, ties to the smaller label
    uint32_t best = 0;
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i) {
        const int b = t + i * kRegionThreads;
        if (b < nb) {
            const uint32_t c = parent[b];
            if (c) best = max(best, (c << 16) | (0xFFFFu - (uint32_t)b));
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) best = max(best, (uint32_t)__shfl_xor((int)best, o));
    if ((t & 63) == 0 && best) atomicMax(&misc[0], best);
    __syncthreads();
    const uint32_t bgkey = misc[0];
    const int bg = bgkey ? (int)(0xFFFFu - (bgkey & 0xFFFFu)) : -1;

    // lowest block row (+1) per label
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i) {
        const int b = t + i * kRegionThreads;
        if (b < nb) parent[b] = 0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i) {
        const int b = t + i * kRegionThreads;
        if (b < nb && !(st[i] >> 24)) atomicMax(&parent[lab[i]], (uint32_t)(b / gw + 1));
    }
    __syncthreads();

    // region depth: background and edge blocks follow the row ramp, other
    // regions sit at the ramp of their lowest row (ground contact)
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i) {
        const int b = t + i * kRegionThreads;
        if (b >= nb) continue;
        const int by = b / gw;
        int d;
        if ((st[i] >> 24) || (int)lab[i] == bg) d = ramp(by, gh);
        else d = ramp((int)parent[lab[i]] - 1, gh);
        f.binfo[b] = make_uint2(st[i], (uint32_t)d);
        f.labels[b] = (int32_t)lab[i];
    }
}

// ---------------------------------------------------------------------------
// k_render: one workgroup per band of rows, all lanes on one row at a time.
// Lane t owns the SEG = 4*Q contiguous pixels [t*SEG, t*SEG + SEG) of every
// row.  LDS holds a ring of 2r+1 rows of luma and raw depth (with a 4-byte
// pad on both sides), one z-buffer row per view, the depth -> offset table
// and the range-weight table.
constexpr int kPad = 4;

template <int R, bool ALIGNED, int Q>
__global__ void __launch_bounds__(1024) k_render(FrameDesc f, int rows_per_band, int bands) {
    extern __shared__ uint32_t lds[];
    constexpr int S = 2 * R + 1;
    constexpr int SEG = 4 * Q;
    const int W = f.w, H = f.h;
    const int t = threadIdx.x, NT = blockDim.x;
    const int lane = t & 63, wave = t >> 6, NW = NT >> 6;

    // XCD-aware band order: consecutive workgroups go to different XCDs, so
    // give each XCD a contiguous run of bands (shared halo rows stay in its L2)
    const int per = gridDim.x >> 3;
    const int band = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (band >= bands) return;
    const int y0 = band * rows_per_band;
    const int y1 = min(y0 + rows_per_band, H);

    const int WP = (W + 2 * kPad + 3) & ~3;
    const int W4 = (W + 3) & ~3;
    uint8_t* ringY = reinterpret_cast<uint8_t*>(lds);
    uint8_t* ringD = ringY + S * WP;
    uint32_t* keyL = reinterpret_cast<uint32_t*>(ringD + S * WP);
    uint32_t* keyR = keyL + W4;
    uint32_t* lut = keyR + W4;
    uint32_t* wr = lut + 256;
    int* agg = reinterpret_cast<int*>(wr + 256);

    // depth -> (left offset, right offset); Fig. 3 rule with rounding reading:
    // P = round(B*m/255), m = D (D > T, crossed) or 255 - D (uncrossed); the
    // left view takes ceil(P/2), the right view floor(P/2), opposite signs.
    for (int d = t; d < 256; d += NT) {
        const bool crossed = d > f.T;
        const int m = crossed ? d : 255 - d;
        const int P = (f.B * m + 127) / 255;
        const int a = (P + 1) >> 1, b = P >> 1;
        const int oL = crossed ? a : -a;
        const int oR = crossed ? -b : b;
        lut[d] = ((uint32_t)oL & 0xFFFFu) | ((uint32_t)oR << 16);
        wr[d] = d < 43 ? c_range_w[d] : 0u;
    }
    for (int i = t; i < W4; i += NT) { keyL[i] = 0; keyR[i] = 0; }

    const int xs = t * SEG;

    // luma + raw depth of image row yy into its ring slot
    auto fill_row = [&](int yy) {
        uint8_t* rY = ringY + (yy % S) * WP + kPad;
        uint8_t* rD = ringD + (yy % S) * WP + kPad;
        const bool dump = f.out_d0 && yy >= y0 && yy < y1;
#pragma unroll
        for (int qi = 0; qi < Q; ++qi) {
            const int x0 = xs + 4 * qi;
            if (x0 >= W) break;
            const int n = min(4, W - x0);
            const uint8_t* p = f.frame + ((size_t)yy * W + x0) * 3;
            int r[4], g[4], b[4], Y[4], D[4];
            load_quad<ALIGNED>(p, n, r, g, b);
#pragma unroll
            for (int j = 0; j < 4; ++j) Y[j] = luma(r[j], g[j], b[j]);
            if (f.depth_in) {
                const uint8_t* dp = f.depth_in + (size_t)yy * W + x0;
#pragma unroll
                for (int j = 0; j < 4; ++j) D[j] = j < n ? dp[j] : 0;
            } else {
                // pixel depth: region depth of the own block, or for an edge
                // block that of the non-edge 3x3 neighbour block whose mean
                // colour is nearest (first strict minimum in raster order)
                const int bx = x0 / f.K, by = yy / f.K;
                const uint2 own = f.binfo[by * f.gw + bx];
                if (!(own.x >> 24)) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) D[j] = (int)own.y;
                } else {
                    int best[4] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX};
                    const int fallback = ramp(by, f.gh);
#pragma unroll
                    for (int j = 0; j < 4; ++j) D[j] = fallback;
                    for (int dy = -1; dy <= 1; ++dy) {
                        const int cy = by + dy;
                        if (cy < 0 || cy >= f.gh) continue;
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int cx = bx + dx;
                            if (cx < 0 || cx >= f.gw) continue;
                            const uint2 c = f.binfo[cy * f.gw + cx];
                            if (c.x >> 24) continue;
                            const int mr = c.x & 255, mg = (c.x >> 8) & 255, mb = (c.x >> 16) & 255;
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                const int dd = iabs(r[j] - mr) + iabs(g[j] - mg) + iabs(b[j] - mb);
                                if (dd < best[j]) { best[j] = dd; D[j] = (int)c.y; }
                            }
                        }
                    }
                }
            }
            if constexpr (ALIGNED) {
                *reinterpret_cast<uint32_t*>(rY + x0) = Y[0] | (Y[1] << 8) | (Y[2] << 16) | (Y[3] << 24);
                *reinterpret_cast<uint32_t*>(rD + x0) = D[0] | (D[1] << 8) | (D[2] << 16) | (D[3] << 24);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (j < n) { rY[x0 + j] = (uint8_t)Y[j]; rD[x0 + j] = (uint8_t)D[j]; }
            }
            if (dump) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (j < n) f.out_d0[(size_t)yy * W + x0 + j] = (uint8_t)D[j];
            }
        }
    };

    for (int yy = y0 - R; yy < y0 + R; ++yy)
        if (yy >= 0 && yy < H) fill_row(yy);

    for (int y = y0; y < y1; ++y) {
        if (y + R < H) fill_row(y + R);
        __syncthreads();

        // ---- cross-bilateral filter and forward warp of both views
        {
            const uint8_t* cY = ringY + (y % S) * WP + kPad;
#pragma unroll
            for (int i = 0; i < SEG; ++i) {
                const int x = xs + i;
                if (x >= W) break;
                const int yp = cY[x];
                uint32_t acc = 0, wsum = 0;
#pragma unroll
                for (int dy = -R; dy <= R; ++dy) {
                    const int yy = y + dy;
                    if (yy < 0 || yy >= H) continue;
                    const uint8_t* rY = ringY + (yy % S) * WP + kPad;
                    const uint8_t* rD = ringD + (yy % S) * WP + kPad;
#pragma unroll
                    for (int dx = -R; dx <= R; ++dx) {
                        const int xx = x + dx;
                        if (xx < 0 || xx >= W) continue;
                        const uint32_t w = spatial_w(dx * dx + dy * dy) * wr[iabs((int)rY[xx] - yp)];
                        acc += w * rD[xx];
                        wsum += w;
                    }
                }
                const uint32_t df = (acc + (wsum >> 1)) / wsum;
                if (f.out_df) f.out_df[(size_t)y * W + x] = (uint8_t)df;
                const uint32_t lv = lut[df];
                const int oL = (int)(int16_t)(lv & 0xFFFFu);
                const int oR = (int)(int16_t)(lv >> 16);
                const uint32_t key = (1u << 24) | (df << 16) | (uint32_t)x;
                const int xl = x + oL, xr = x + oR;
                if ((unsigned)xl < (unsigned)W) atomicMax(&keyL[xl], key);
                if ((unsigned)xr < (unsigned)W) atomicMax(&keyR[xr], key);
            }
        }
        __syncthreads();

        // ---- hole fill: nearest valid pixel on each side by scans
        {
            uint32_t kl[SEG], kr[SEG];
            int lastL = -1, lastR = -1, firstL = W, firstR = W;
#pragma unroll
            for (int i = 0; i < SEG; ++i) {
                const int x = xs + i;
                kl[i] = x < W ? keyL[x] : 0u;
                kr[i] = x < W ? keyR[x] : 0u;
                if (kl[i]) lastL = x;
                if (kr[i]) lastR = x;
            }
#pragma unroll
            for (int i = SEG - 1; i >= 0; --i) {
                if (kl[i]) firstL = xs + i;
                if (kr[i]) firstR = xs + i;
            }
            // inclusive wave scans: prefix max of the last valid x, suffix
            // min of the first valid x
            int pL = lastL, pR = lastR, sL = firstL, sR = firstR;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int a = __shfl_up(pL, o), b = __shfl_up(pR, o);
                const int c = __shfl_down(sL, o), d = __shfl_down(sR, o);
                if (lane >= o) { pL = max(pL, a); pR = max(pR, b); }
                if (lane + o < 64) { sL = min(sL, c); sR = min(sR, d); }
            }
            if (lane == 63) { agg[wave] = pL; agg[NW + wave] = pR; }
            if (lane == 0) { agg[2 * NW + wave] = sL; agg[3 * NW + wave] = sR; }
            __syncthreads();
            int eL = __shfl_up(pL, 1), eR = __shfl_up(pR, 1);
            int fL = __shfl_down(sL, 1), fR = __shfl_down(sR, 1);
            if (lane == 0) { eL = -1; eR = -1; }
            if (lane == 63) { fL = W; fR = W; }
            for (int v = 0; v < wave; ++v) { eL = max(eL, agg[v]); eR = max(eR, agg[NW + v]); }
            for (int v = wave + 1; v < NW; ++v) { fL = min(fL, agg[2 * NW + v]); fR = min(fR, agg[3 * NW + v]); }

            int nearL[SEG], nearR[SEG];  // nearest valid x on the left
#pragma unroll
            for (int i = 0; i < SEG; ++i) {
                nearL[i] = eL; nearR[i] = eR;
                if (kl[i]) eL = xs + i;
                if (kr[i]) eR = xs + i;
            }
            int srcL[SEG], srcR[SEG];
#pragma unroll
            for (int i = SEG - 1; i >= 0; --i) {
                const int x = xs + i;
                // left view: equal depths take the left neighbour
                if (kl[i]) {
                    srcL[i] = kl[i] & 0xFFFF;
                } else {
                    const int a = nearL[i], b = fL;
                    if (a >= 0 && b < W) {
                        const uint32_t ka = keyL[a], kb = keyL[b];
                        srcL[i] = (((kb >> 16) & 255) < ((ka >> 16) & 255) ? kb : ka) & 0xFFFF;
                    } else if (a >= 0) {
                        srcL[i] = keyL[a] & 0xFFFF;
                    } else if (b < W) {
                        srcL[i] = keyL[b] & 0xFFFF;
                    } else {
                        srcL[i] = x;
                    }
                }
                // right view: equal depths take the right neighbour
                if (kr[i]) {
                    srcR[i] = kr[i] & 0xFFFF;
                } else {
                    const int a = nearR[i], b = fR;
                    if (a >= 0 && b < W) {
                        const uint32_t ka = keyR[a], kb = keyR[b];
                        srcR[i] = (((ka >> 16) & 255) < ((kb >> 16) & 255) ? ka : kb) & 0xFFFF;
                    } else if (a >= 0) {
                        srcR[i] = keyR[a] & 0xFFFF;
                    } else if (b < W) {
                        srcR[i] = keyR[b] & 0xFFFF;
                    } else {
                        srcR[i] = x;
                    }
                }
                if (kl[i]) fL = x;
                if (kr[i]) fR = x;
            }

            // ---- gather colours, anaglyph, RGB24 stores
            const uint8_t* row = f.frame + (size_t)y * W * 3;
#pragma unroll
            for (int qi = 0; qi < Q; ++qi) {
                const int x0 = xs + 4 * qi;
                if (x0 >= W) break;
                const int n = min(4, W - x0);
                int lr[4], lg[4], lb[4], rr[4], rg[4], rb[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (j < n) {
                        const uint8_t* pl = row + 3 * srcL[4 * qi + j];
                        const uint8_t* pr = row + 3 * srcR[4 * qi + j];
                        lr[j] = pl[0]; lg[j] = pl[1]; lb[j] = pl[2];
                        rr[j] = pr[0]; rg[j] = pr[1]; rb[j] = pr[2];
                    } else {
                        lr[j] = lg[j] = lb[j] = rr[j] = rg[j] = rb[j] = 0;
                    }
                }
                const size_t off = ((size_t)y * W + x0) * 3;
                if (f.out_l) store_quad<ALIGNED>(f.out_l + off, n, lr, lg, lb);
                if (f.out_r) store_quad<ALIGNED>(f.out_r + off, n, rr, rg, rb);
                if (f.out_a) store_quad<ALIGNED>(f.out_a + off, n, lr, rg, rb);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < SEG; ++i) {
            const int x = xs + i;
            if (x < W) { keyL[x] = 0; keyR[x] = 0; }
        }
    }
}

// ---------------------------------------------------------------------------
// host-side launch helpers

size_t render_lds_bytes(int w, int r, int threads, int /*quads*/) {
    const int S = 2 * r + 1;
    const size_t WP = (size_t)((w + 2 * kPad + 3) & ~3);
    const size_t W4 = (size_t)((w + 3) & ~3);
    return 2 * S * WP + 2 * W4 * 4 + 256 * 4 * 2 + 4 * (threads / 64) * 4;
}

static constexpr size_t kMaxLds = 160 * 1024;

bool render_shape(int w, int h, int r, int rows_per_band, RenderShape* out) {
    const int quads_row = (w + 3) / 4;
    int q = 1;
    while (q < 4 && quads_row > 1024 * q) q *= 2;
    if (quads_row > 1024 * q) return false;
    int threads = (quads_row + q - 1) / q;
    threads = ((threads + 63) / 64) * 64;
    const size_t lds = render_lds_bytes(w, r, threads, q);
    if (lds > kMaxLds) return false;
    int per_cu = (int)(kMaxLds / lds);
    per_cu = min(per_cu, 2048 / threads);
    per_cu = max(per_cu, 1);
    if (rows_per_band <= 0) {
        const int target = 256 * per_cu;
        rows_per_band = max((h + target - 1) / target, 4);
    }
    rows_per_band = min(rows_per_band, h);
    out->threads = threads;
    out->quads = q;
    out->rows_per_band = rows_per_band;
    out->bands = (h + rows_per_band - 1) / rows_per_band;
    out->grid = ((out->bands + 7) / 8) * 8;
    out->lds_bytes = lds;
    return true;
}

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

static size_t regions_lds_bytes(int nb) { return (size_t)(nb + (nb + 15) / 16 + 4) * 4; }

hipError_t launch_regions(const FrameDesc& f, hipStream_t s) {
    const int nb = f.gw * f.gh;
    hipLaunchKernelGGL(k_regions, dim3(1), dim3(kRegionThreads), regions_lds_bytes(nb), s, f);
    return hipGetLastError();
}

template <int R, bool A, int Q>
static hipError_t rd_launch(const FrameDesc& f, const RenderShape& rs, hipStream_t s) {
    hipLaunchKernelGGL((k_render<R, A, Q>), dim3(rs.grid), dim3(rs.threads), rs.lds_bytes, s, f,
                       rs.rows_per_band, rs.bands);
    return hipGetLastError();
}

template <int R, bool A>
static hipError_t rd_q(const FrameDesc& f, const RenderShape& rs, hipStream_t s) {
    switch (rs.quads) {
        case 1: return rd_launch<R, A, 1>(f, rs, s);
        case 2: return rd_launch<R, A, 2>(f, rs, s);
        case 4: return rd_launch<R, A, 4>(f, rs, s);
        default: return hipErrorInvalidValue;
    }
}

template <int R>
static hipError_t rd_a(const FrameDesc& f, const RenderShape& rs, hipStream_t s) {
    return f.aligned ? rd_q<R, true>(f, rs, s) : rd_q<R, false>(f, rs, s);
}

hipError_t launch_render(const FrameDesc& f, const RenderShape& rs, hipStream_t s) {
    switch (f.r) {
        case 0: return rd_a<0>(f, rs, s);
        case 1: return rd_a<1>(f, rs, s);
        case 2: return rd_a<2>(f, rs, s);
        case 3: return rd_a<3>(f, rs, s);
        default: return hipErrorInvalidValue;
    }
}

template <int R, bool A, int Q>
static hipError_t allow_lds() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_render<R, A, Q>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
}

template <int R, bool A>
static hipError_t allow_lds_q() {
    hipError_t e;
    if ((e = allow_lds<R, A, 1>()) != hipSuccess) return e;
    if ((e = allow_lds<R, A, 2>()) != hipSuccess) return e;
    return allow_lds<R, A, 4>();
}

template <int R>
static hipError_t allow_lds_a() {
    hipError_t e = allow_lds_q<R, true>();
    return e != hipSuccess ? e : allow_lds_q<R, false>();
}

hipError_t prepare_kernels(int /*device*/) {
    hipError_t e;
    if ((e = allow_lds_a<0>()) != hipSuccess) return e;
    if ((e = allow_lds_a<1>()) != hipSuccess) return e;
    if ((e = allow_lds_a<2>()) != hipSuccess) return e;
    if ((e = allow_lds_a<3>()) != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_regions),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
}

}  // namespace pstereo
