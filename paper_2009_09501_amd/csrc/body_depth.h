// Device bodies of the depth-map stages: block statistics and region grouping
// (used by the per-frame kernels and by the persistent batch kernel).
//
// The depth map follows the paper's conversion scheme (Section 3, Fig. 1:
// the depth map is the first of the six components; Section 4: it is the
// "iterative" stage) built from block colour and edge cues (Section 2 and
// Table 1: edge / region-boundary information, block processing).  The exact
// cues, thresholds and region-depth rule are the library's readings.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.h"

namespace pstereo {

// ---------------------------------------------------------------------------
// block statistics: per K x K block, rounded mean colour and edge flag.
//
// Tiles of 256 px x 4 RW rows on 256 lanes (four waves): wave w covers the RW
// rows [RW w, RW w + RW) of the tile (RW = 8 for blocks up to 16 px, 16 for
// larger ones, so that a block lies in one tile) and lane l the quad of
// pixels 4l .. 4l+3 in each of them, so every load instruction of a wave
// reads 768 contiguous bytes of one row; a lane issues all RW + 1 of its rows
// (its RW and the one below, for the vertical luma steps) before using any.
// Sums and luma come from byte dot products in registers; the horizontal step
// into the next quad takes that quad's first luma from the next lane (the
// tile's last lane loads the next tile's first pixel); the lanes of one block
// combine by lane shuffles, and blocks taller than a wave's rows add the
// waves' shares in LDS.
constexpr int kBsTileW = 256;  // px: 64 quads, one per lane of a wave

// Rows per wave of a block-statistics tile by default (the tile is four
// waves tall).
__host__ __device__ constexpr int bs_default_rw(int K) { return K <= 16 ? 8 : 16; }

// A 256 x 4 RWT px tile for blocks of K px (4 RWT >= K: a block never spans
// two tiles).
template <int K, int RWT = bs_default_rw(K)>
struct BsTile {
    static_assert(4 * RWT >= K && (RWT == 4 || RWT == 8 || RWT == 16), "block-statistics tile rows");
    static constexpr int RW = RWT;                                         // rows per wave
    static constexpr int TH = 4 * RW;                                      // tile rows
    static constexpr int QB = K / 4;                                       // lanes per block
    static constexpr int NBR = K >= RW ? 1 : RW / K;                       // block rows per wave
    static constexpr int kBlocks = (kBsTileW / K) * (TH / K);              // blocks per tile (K >= 4)
    static constexpr bool kCross = K > RW;                                 // blocks span waves
    static constexpr int kLdsWords = kCross ? 4 * kBlocks : 1;             // r, g, b, edge per block
};

// Tile rows of the block statistics for block size K (2 px blocks: 64).
__host__ __device__ constexpr int bs_tile_rows(int K) { return K <= 2 ? 64 : K <= 16 ? 32 : 64; }
// The same with a tuned height (0 = the default; else 16, 32 or 64, raised
// to K so that a block never spans two tiles; 2 px blocks keep 64).
__host__ __device__ constexpr int bs_tile_rows_tuned(int K, int rows) {
    return K <= 2 || rows == 0 ? bs_tile_rows(K) : (rows > K ? rows : K);
}

// Rounded mean sum / cnt of a block of cnt pixels, (sum + cnt / 2) / cnt: a
// shift for a whole K x K block (cnt = K * K, a power of two), the division
// only for blocks cut by the frame's right or bottom edge.
template <int K>
__device__ __forceinline__ uint32_t block_mean(uint32_t sum, uint32_t cnt) {
    constexpr uint32_t kFull = (uint32_t)(K * K);
    constexpr int kShift = __builtin_ctz(kFull);
    if (cnt == kFull) return (sum + kFull / 2) >> kShift;
    return (sum + cnt / 2) / cnt;
}

// The n (1..4) pixels of a quad starting at p as three dwords of RGB24 bytes,
// zero past the n-th pixel.  ALIGNED: a whole quad at a 4-byte aligned address.
template <bool ALIGNED>
__device__ __forceinline__ uint3 load_quad_words(const uint8_t* p, int n) {
    if constexpr (ALIGNED) {
        return *reinterpret_cast<const uint3*>(p);
    } else {
        uint32_t w[3] = {0u, 0u, 0u};
#pragma unroll
        for (int i = 0; i < 12; ++i)
            if (i < 3 * n) w[i >> 2] |= (uint32_t)p[i] << (8 * (i & 3));
        return make_uint3(w[0], w[1], w[2]);
    }
}

// Luma of the four pixels of a quad held in three dwords.
__device__ __forceinline__ void bs_quad_luma(uint3 q, uint32_t (&Y)[4]) {
    constexpr uint32_t wlo = 77u | (150u << 8) | (29u << 16);
    Y[0] = __builtin_amdgcn_udot4(q.x, wlo, 128u, false) >> 8;
    Y[1] = __builtin_amdgcn_udot4(__builtin_amdgcn_alignbyte(q.y, q.x, 3), wlo, 128u, false) >> 8;
    Y[2] = __builtin_amdgcn_udot4(__builtin_amdgcn_alignbyte(q.z, q.y, 2), wlo, 128u, false) >> 8;
    Y[3] = __builtin_amdgcn_udot4(q.z, wlo << 8, 128u, false) >> 8;
}

// One 256 x 4 RWT tile (tile_x, tile_y) on 256 lanes t = 0..255.  lds:
// BsTile<K, RWT>::kLdsWords words.  Inactive lane groups (active == false) do no
// memory work but pass the same barriers (blocks spanning waves only).
template <int K, bool ALIGNED, int RWT = bs_default_rw(K)>
__device__ __forceinline__ void bs_tile(const FrameDesc& f, int tile_x, int tile_y, int t, uint32_t* lds,
                                        bool active) {
    using T = BsTile<K, RWT>;
    constexpr int QB = T::QB, NBR = T::NBR, RW = T::RW;
    constexpr uint32_t wlo = 77u | (150u << 8) | (29u << 16);
    const int wave = t >> 6, lane = t & 63;
    const int W = f.w, H = active ? f.h : 0;
    const int x0 = tile_x * kBsTileW + 4 * lane;
    const int y0 = tile_y * T::TH + RW * wave;
    const int n = min(4, W - x0);  // pixels of the lane's quad inside the image (<= 0: none)
    const uint32_t g = (uint32_t)f.g;
    if (T::kCross)
        for (int i = t; i < T::kLdsWords; i += 256) lds[i] = 0;

    // every row's loads in flight before any is used
    const uint8_t* p0 = f.frame + ((size_t)y0 * W + x0) * 3;
    const size_t stride = (size_t)W * 3;
    uint3 v[RW + 1];
    uint32_t nx[RW];  // the tile's last lane: the next tile's first pixel per row
#pragma unroll
    for (int k = 0; k <= RW; ++k) {
        v[k] = make_uint3(0u, 0u, 0u);
        if (y0 + k < H && n > 0) v[k] = load_quad_words<ALIGNED>(p0 + k * stride, n);
    }
    const bool edge_lane = lane == 63 && x0 + 4 < W;
#pragma unroll
    for (int k = 0; k < RW; ++k) {
        nx[k] = 0u;
        if (edge_lane && y0 + k < H) {
            const uint8_t* q = p0 + k * stride + 12;
            nx[k] = ALIGNED ? *reinterpret_cast<const uint32_t*>(q)
                            : (uint32_t)q[0] | ((uint32_t)q[1] << 8) | ((uint32_t)q[2] << 16);
        }
    }

    // a step from pixel j to the right exists when j + 1 is in the image;
    // a pixel exists when j < n
    uint32_t sr[NBR], sg[NBR], sb[NBR], em[NBR];
#pragma unroll
    for (int i = 0; i < NBR; ++i) sr[i] = sg[i] = sb[i] = em[i] = 0u;
    // FULL: the wave's rows and the row below all lie inside the image (the
    // common case), so no row needs a bounds test
    auto rows = [&](auto full) {
        constexpr bool FULL = decltype(full)::value;
        uint32_t Yc[4];
        bs_quad_luma(v[0], Yc);
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const int br = (k * NBR) / RW;  // block row of row k inside the wave
            const int y = y0 + k;
            uint32_t Yb[4];
            bs_quad_luma(v[k + 1], Yb);  // the row below (zero past the image)
            const uint32_t yn_lane = (uint32_t)__shfl_down((int)Yc[0], 1);  // pixel x0 + 4 from the next lane
            if (FULL || y < H) {
                sr[br] = __builtin_amdgcn_udot4(v[k].x, 0x01000001u, sr[br], false);
                sr[br] = __builtin_amdgcn_udot4(v[k].y, 0x00010000u, sr[br], false);
                sr[br] = __builtin_amdgcn_udot4(v[k].z, 0x00000100u, sr[br], false);
                sg[br] = __builtin_amdgcn_udot4(v[k].x, 0x00000100u, sg[br], false);
                sg[br] = __builtin_amdgcn_udot4(v[k].y, 0x01000001u, sg[br], false);
                sg[br] = __builtin_amdgcn_udot4(v[k].z, 0x00010000u, sg[br], false);
                sb[br] = __builtin_amdgcn_udot4(v[k].x, 0x00010000u, sb[br], false);
                sb[br] = __builtin_amdgcn_udot4(v[k].y, 0x00000100u, sb[br], false);
                sb[br] = __builtin_amdgcn_udot4(v[k].z, 0x01000001u, sb[br], false);
                const uint32_t Yn = lane == 63 ? __builtin_amdgcn_udot4(nx[k], wlo, 128u, false) >> 8 : yn_lane;
                const uint32_t Yr[4] = {Yc[1], Yc[2], Yc[3], Yn};
                uint32_t dh[4], dv[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const bool h_ok = ALIGNED ? (j < 3 || x0 + 4 < W) : (j < n && x0 + j + 1 < W);
                    const bool v_ok = (ALIGNED || j < n) && (FULL || y + 1 < H);
                    dh[j] = h_ok ? __builtin_amdgcn_sad_u16(Yr[j], Yc[j], 0u) : 0u;
                    dv[j] = v_ok ? __builtin_amdgcn_sad_u16(Yb[j], Yc[j], 0u) : 0u;
                }
                em[br] = max(max(max(em[br], dh[0]), max(dh[1], dh[2])),
                             max(max(dh[3], dv[0]), max(max(dv[1], dv[2]), dv[3])));
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) Yc[j] = Yb[j];
        }
    };
    if (y0 + RW < H) rows(std::true_type{});
    else rows(std::false_type{});

    const int bx = x0 / K;  // the lane's block column (x0 >= 0)
    if (!T::kCross) {
        // K <= 16: a block lies in one wave, QB lanes wide; two 16-bit sums
        // per register (QB * K * 4 * 255 < 2^16)
#pragma unroll
        for (int br = 0; br < NBR; ++br) {
            uint32_t rg = sr[br] | (sg[br] << 16), be = sb[br] | ((em[br] > g ? 1u : 0u) << 16);
#pragma unroll
            for (int o = 1; o < QB; o <<= 1) {
                rg += (uint32_t)__shfl_xor((int)rg, o);
                be += (uint32_t)__shfl_xor((int)be, o);
            }
            const int by = (y0 + br * K) / K;
            if (active && lane % QB == 0 && bx < f.gw && by < f.gh && n > 0) {
                const uint32_t cnt = (uint32_t)((min(bx * K + K, W) - bx * K) * (min(by * K + K, H) - by * K));
                f.stats[by * f.gw + bx] = block_mean<K>(rg & 0xFFFFu, cnt) | (block_mean<K>(rg >> 16, cnt) << 8) |
                                          (block_mean<K>(be & 0xFFFFu, cnt) << 16) | ((be >> 16) ? 1u << 24 : 0u);
            }
        }
    } else {
        // blocks taller than RW: the wave's RW rows of its blocks, then across
        // waves (32-bit sums)
        uint32_t r = sr[0], gg = sg[0], b = sb[0], e = em[0] > g ? 1u : 0u;
#pragma unroll
        for (int o = 1; o < QB; o <<= 1) {
            r += (uint32_t)__shfl_xor((int)r, o);
            gg += (uint32_t)__shfl_xor((int)gg, o);
            b += (uint32_t)__shfl_xor((int)b, o);
            e |= (uint32_t)__shfl_xor((int)e, o);
        }
        __syncthreads();  // the LDS sums are zero
        constexpr int BC = kBsTileW / K;  // block columns per tile
        const int blk = (lane / QB) + BC * ((wave * RW) / K);
        if (lane % QB == 0) {
            atomicAdd(&lds[4 * blk + 0], r);
            atomicAdd(&lds[4 * blk + 1], gg);
            atomicAdd(&lds[4 * blk + 2], b);
            if (e) atomicOr(&lds[4 * blk + 3], 1u);
        }
        __syncthreads();
        if (t < T::kBlocks) {
            const int cbx = tile_x * BC + t % BC, cby = tile_y * (T::TH / K) + t / BC;
            if (active && cbx < f.gw && cby < f.gh) {
                const uint32_t cnt =
                    (uint32_t)((min(cbx * K + K, W) - cbx * K) * (min(cby * K + K, H) - cby * K));
                f.stats[cby * f.gw + cbx] = block_mean<K>(lds[4 * t + 0], cnt) |
                                            (block_mean<K>(lds[4 * t + 1], cnt) << 8) |
                                            (block_mean<K>(lds[4 * t + 2], cnt) << 16) | (lds[4 * t + 3] << 24);
            }
        }
    }
}

// Block statistics for blocks of 2 x 2 px (frames of at most 2^17 pixels,
// so this path is never the bulk of the work): 256 x 64 px tiles on 256
// lanes; lane t takes blocks t, t + 256, ... of the tile's 128 x 32 blocks,
// reading pixels bytewise and the luma steps to the right and below
// directly.  No barriers.
__device__ __forceinline__ void bs_tile_k2(const FrameDesc& f, int tile_x, int tile_y, int t, bool active) {
    if (!active) return;
    const int W = f.w, H = f.h;
    constexpr int BC = kBsTileW / 2, BR = 64 / 2;
    for (int i = t; i < BC * BR; i += 256) {
        const int bx = tile_x * BC + i % BC, by = tile_y * BR + i / BC;
        if (bx >= f.gw || by >= f.gh) continue;
        uint32_t sr = 0, sg = 0, sb = 0, cnt = 0, edge = 0;
        for (int dy = 0; dy < 2; ++dy) {
            for (int dx = 0; dx < 2; ++dx) {
                const int x = 2 * bx + dx, y = 2 * by + dy;
                if (x >= W || y >= H) continue;
                const uint8_t* p = f.frame + ((size_t)y * W + x) * 3;
                sr += p[0];
                sg += p[1];
                sb += p[2];
                ++cnt;
                const int Y = luma(p[0], p[1], p[2]);
                if (x + 1 < W && iabs(luma(p[3], p[4], p[5]) - Y) > f.g) edge = 1;
                if (y + 1 < H) {
                    const uint8_t* q = p + (size_t)W * 3;
                    if (iabs(luma(q[0], q[1], q[2]) - Y) > f.g) edge = 1;
                }
            }
        }
        f.stats[by * f.gw + bx] = ((sr + cnt / 2) / cnt) | (((sg + cnt / 2) / cnt) << 8) |
                                  (((sb + cnt / 2) / cnt) << 16) | (edge << 24);
    }
}

// ---------------------------------------------------------------------------
// region grouping, one workgroup of 1024 lanes per frame.
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

// Exact floor(n / d) for n, d < 2^16 from m = ceil(2^32 / d) (d >= 2): the
// product overshoots n / d by less than n / 2^32 < 1 / d, which never carries
// past the next integer.
__device__ __forceinline__ uint32_t div_u16(uint32_t n, uint32_t m, uint32_t d) {
    return d == 1 ? n : __umulhi(n, m);
}

// Region grouping of one frame on a whole 1024-lane workgroup; lds: the
// regions_lds_bytes(gw * gh) bytes of dynamic LDS.
//
// Lane t owns the 32 contiguous blocks [32t, 32t + 32).  Row segments (runs
// of right-linked blocks) are formed by a prefix-max scan, rows are joined by
// union-find in LDS only where the pair of segments changes along a row, and
// the label of a component (its smallest block index, always a segment start)
// is found at the root.  The label's own word then collects the lowest block
// row + 1 (low half, atomicMax) and the block count (high half, atomicAdd,
// after the rows); the lane owning the label block turns that into the
// region's depth.  Edge blocks are components of their own.
__device__ __forceinline__ void regions_body(const FrameDesc& f, uint32_t* lds) {
    const int gw = f.gw, gh = f.gh, nb = gw * gh;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    constexpr int NW = kRegionThreads / 64;
    uint32_t* parent = lds;                           // pidx(nb) words
    uint32_t* lrb = parent + pidx((uint32_t)nb) + 1;  // right-link bits, word j = blocks 32j..32j+31
    uint32_t* ldb = lrb + kRegionThreads;             // down-link bits
    uint32_t* eb = ldb + kRegionThreads;              // edge bits
    uint32_t* scan = eb + kRegionThreads;             // NW words
    uint32_t* misc = scan + NW;                       // [0]: background key
    uint32_t* binfo_w = reinterpret_cast<uint32_t*>(f.binfo);

    // 1. block statistics into LDS (strided, coalesced loads, all in flight),
    // and the statistics half of the block table
    {
        uint32_t sv[kRegionPer];
#pragma unroll
        for (int i = 0; i < kRegionPer; ++i) {
            const int b = i * kRegionThreads + t;
            sv[i] = b < nb ? f.stats[b] : 0u;
        }
#pragma unroll
        for (int i = 0; i < kRegionPer; ++i) {
            const int b = i * kRegionThreads + t;
            if (b < nb) {
                parent[pidx(b)] = sv[i];
                binfo_w[2 * b] = sv[i];
            }
        }
    }
    if (t == 0) misc[0] = 0;
    __syncthreads();

    // 2. edge / right-link / down-link bits of the owned blocks, branch-free
    // from LDS (lane t's words sit 33 apart: distinct banks across a wave).
    // Blocks past the grid read as edges.
    const int b0 = t * kRegionPer;
    const int nown = max(0, min(kRegionPer, nb - b0));
    const uint32_t own_mask = nown >= 32 ? 0xFFFFFFFFu : ((1u << nown) - 1u);
    uint32_t* own = parent + 33 * t;  // own[i] = parent[pidx(b0 + i)] for i < 32
    int B0 = b0;
    const uint32_t gwm = gw > 1 ? (uint32_t)((0x100000000ull + (uint32_t)gw - 1) / (uint32_t)gw) : 0u;
    const uint32_t row0 = div_u16((uint32_t)min(b0, nb - 1 > 0 ? nb - 1 : 0), gwm, (uint32_t)gw);
    uint32_t emask = 0, lr = 0, ld = 0;
    {
        constexpr uint32_t kPast = 0xFF000000u;
        // bit i: block b0 + i ends its row (then it has no right neighbour);
        // a run of 32 blocks crosses at most one row end when gw >= 32
        uint32_t rowend = 0;
        if (gw >= kRegionPer) {
            const int wrap = (int)((row0 + 1) * (uint32_t)gw) - b0;  // next row's first block, from b0
            if (wrap >= 1 && wrap <= kRegionPer) rowend = 1u << (wrap - 1);
        } else {
            for (int i = 0; i < kRegionPer; ++i)
                if ((b0 + i + 1) % gw == 0) rowend |= 1u << i;
        }
        // two halves of 16 blocks: 33 loads in flight per half
#pragma unroll
        for (int h = 0; h < kRegionPer; h += 16) {
            // unconditional loads from clamped (in-range) indices, then a
            // select: no branch per load
            uint32_t sv[17], dv[16];
            const int last = nb - 1;
#pragma unroll
            for (int i = 0; i <= 16; ++i) {
                const int b = b0 + h + i;
                const uint32_t v = parent[pidx((uint32_t)min(b, last))];
                sv[i] = b <= last ? v : kPast;
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int b = b0 + h + i + gw;
                const uint32_t v = parent[pidx((uint32_t)min(b, last))];
                dv[i] = b <= last ? v : kPast;
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const uint32_t sb = sv[i];
                const bool e = (sb >> 24) != 0;
                const bool row_end = (rowend >> (h + i)) & 1u;
                const bool rok = !row_end && !(sv[i + 1] >> 24) &&
                                 (int)__builtin_amdgcn_sad_u8(sb, sv[i + 1], 0u) <= f.tau;
                const bool dok = !(dv[i] >> 24) && (int)__builtin_amdgcn_sad_u8(sb, dv[i], 0u) <= f.tau;
                emask |= (uint32_t)e << (h + i);
                lr |= (uint32_t)(!e && rok) << (h + i);
                ld |= (uint32_t)(!e && dok) << (h + i);
            }
        }
    }
    emask = (uint32_t)opaque((int)(emask | ~own_mask));  // kept as one mask, not 32 flags
    lr &= own_mask;
    ld &= own_mask;
    lrb[t] = lr;
    ldb[t] = ld;
    eb[t] = emask;
    __syncthreads();

    B0 = opaque(b0);
    // 3. segments: start(b) = b is not right-linked from b - 1 (a row's first
    // block never is: the last block of a row has no right link)
    const uint32_t prev_lr = t > 0 ? lrb[t - 1] : 0u;
    const uint32_t linked_from_left = (lr << 1) | (prev_lr >> 31);
    const uint32_t starts = ~linked_from_left & own_mask;
    const int last_start = starts ? B0 + 31 - __clz(starts) : -1;
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
    const int seg_in = carry;   // segment start of block b0 when b0 is not a start
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i) {
        if ((starts >> i) & 1u) carry = B0 + i;
        if (i < nown) own[i] = (uint32_t)carry;
    }
    __syncthreads();

    B0 = opaque(b0);
    // 4. unions across rows, only where the pair of segments changes along
    // the row: skip b when b - 1 is in the same segment, also links down, and
    // the blocks below b - 1 and b are right-linked too (then b and the block
    // below it are already joined through b - 1).  Block b0 - 1 belongs to
    // the previous lane; its bits are read from the shared bitmaps.
    {
        const int c0 = B0 + gw;  // first block below the owned run
        uint32_t below_lr = 0;
        if (ld) {
            const int w = c0 >> 5, sh = c0 & 31;
            const uint32_t lo = lrb[w];
            const uint32_t hi = (w + 1 < kRegionThreads) ? lrb[w + 1] : 0u;
            below_lr = sh ? (lo >> sh) | (hi << (32 - sh)) : lo;  // bit i = right link of block c0 + i
        }
        uint32_t todo = ld & ~((ld & lr & below_lr) << 1);
        if ((todo & 1u) && t > 0 && ((ldb[t - 1] & prev_lr) >> 31)) {
            const int c = B0 - 1 + gw;  // below block b0 - 1 (exists: b0 - 1 links down)
            if ((lrb[c >> 5] >> (c & 31)) & 1u) todo &= ~1u;
        }
        while (todo) {
            const int i = __ffs(todo) - 1;
            todo &= todo - 1;
            uf_unite_s(parent, (uint32_t)(B0 + i), (uint32_t)(B0 + i + gw));
        }
    }
    __syncthreads();

    B0 = opaque(b0);
    // 5. labels of the segment starts: root, then the smallest start index of
    // the tree collected at the root as 0x10000 | min, then published in the
    // start's own word for the blocks of later lanes in the same segment
    uint32_t lab[kRegionPer];  // root, then label of each segment start; then label of each owned block
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i) lab[i] = ((starts >> i) & 1u) ? uf_find_s(parent, opaque(b0) + i) : 0u;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i)
        if (((starts >> i) & 1u) && lab[i] == (uint32_t)(B0 + i)) own[i] = 0xFFFFFFFFu;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i)
        if ((starts >> i) & 1u) atomicMin(&parent[pidx(lab[i])], 0x10000u | (uint32_t)(B0 + i));
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i)
        if ((starts >> i) & 1u) lab[i] = parent[pidx(lab[i])] & 0xFFFFu;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i)
        if ((starts >> i) & 1u) own[i] = lab[i];
    __syncthreads();
    {
        uint32_t cur = (nown && !(starts & 1u)) ? parent[pidx(seg_in)] : 0u;
#pragma unroll
        for (int i = 0; i < kRegionPer; ++i) {
            if ((starts >> i) & 1u) cur = lab[i];
            lab[i] = cur;
        }
    }
    // piece ends: last owned block of a run of equal labels
    uint32_t pend = 0;
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i)
        if (i + 1 < kRegionPer && lab[i + 1] != lab[i]) pend |= 1u << i;
    pend = (pend | (1u << (nown > 0 ? nown - 1 : 0))) & own_mask;
    // label blocks owned here (the component's smallest block)
    uint32_t lown = 0;
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i)
        if (lab[i] == (uint32_t)(B0 + i)) lown |= 1u << i;
    lown &= own_mask;
    __syncthreads();

    B0 = opaque(b0);
    // 6. per non-edge label: lowest row + 1, then the block count
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i)
        if ((lown >> i) & 1u) own[i] = 0;
    __syncthreads();
    const uint32_t nonedge_end = pend & ~emask;
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i)
        if ((nonedge_end >> i) & 1u)
            atomicMax(&parent[pidx(lab[i])], div_u16((uint32_t)(B0 + i), gwm, (uint32_t)gw) + 1u);
    __syncthreads();
    {
        // a piece is one edge block or all non-edge; its length is the
        // distance to the previous piece end
        int prev = -1;
#pragma unroll
        for (int i = 0; i < kRegionPer; ++i) {
            if ((pend >> i) & 1u) {
                if (!((emask >> i) & 1u)) atomicAdd(&parent[pidx(lab[i])], (uint32_t)(i - prev) << 16);
                prev = i;
            }
        }
    }
    __syncthreads();

    B0 = opaque(b0);
    // 7. background = the largest non-edge region, ties to the smaller label
    // (largest key (count << 16) | (0xFFFF - label)); each non-edge label's
    // word becomes its region depth: the ramp at its lowest row
    {
        uint32_t best = 0;
        const uint32_t lne = lown & ~emask;
#pragma unroll
        for (int i = 0; i < kRegionPer; ++i) {
            if ((lne >> i) & 1u) {
                const uint32_t w = own[i];
                best = max(best, (w & 0xFFFF0000u) | (0xFFFFu - (uint32_t)(B0 + i)));
                own[i] = (uint32_t)ramp((int)(w & 0xFFFFu) - 1, gh);
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) best = max(best, (uint32_t)__shfl_xor((int)best, o));
        if (lane == 0 && best) atomicMax(&misc[0], best);
    }
    __syncthreads();
    const uint32_t bgkey = misc[0];
    const uint32_t bg = bgkey ? 0xFFFFu - (bgkey & 0xFFFFu) : 0xFFFFFFFFu;

    B0 = opaque(b0);
    // 8. block depth: edge and background blocks follow the row ramp, any
    // other block takes its region's depth; packed (label << 8 | depth)
    {
        auto pack = [&](int i, int rr) {
            const bool own_ramp = ((emask >> i) & 1u) || lab[i] == bg;
            const int d = own_ramp ? rr : (int)parent[pidx(lab[i])];
            lab[i] = (lab[i] << 8) | (uint32_t)d;
        };
        if (gw >= kRegionPer) {
            // at most two rows: the ramps of both, picked per block
            const int r0 = ramp((int)row0, gh), r1 = ramp((int)row0 + 1, gh);
            const int wrap = (int)((row0 + 1) * (uint32_t)gw) - b0;
#pragma unroll
            for (int i = 0; i < kRegionPer; ++i)
                if (i < nown) pack(i, i < wrap ? r0 : r1);
        } else {
#pragma unroll
            for (int i = 0; i < kRegionPer; ++i)
                if (i < nown) pack(i, ramp((int)div_u16((uint32_t)(B0 + i), gwm, (uint32_t)gw), gh));
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRegionPer; ++i)
        if (i < nown) own[i] = lab[i];
    __syncthreads();
#pragma unroll 8
    for (int i = 0; i < kRegionPer; ++i) {
        const int b = i * kRegionThreads + t;
        if (b < nb) {
            const uint32_t v = parent[pidx(b)];
            binfo_w[2 * b + 1] = v & 255u;
            f.labels[b] = (int32_t)(v >> 8);
        }
    }
}

__host__ __device__ constexpr size_t regions_lds_bytes_c(int nb) {
    return (size_t)(nb + nb / 32 + 1 + 3 * kRegionThreads + kRegionThreads / 64 + 4) * 4;
}

// ---------------------------------------------------------------------------
// Strip-parallel region grouping.  The same components and labels as
// regions_body, computed in two launches (plus a per-block pass on request):
//   strips: one workgroup per strip of rstrip block rows (at most
//     kStripBlocks blocks, two per lane) finds the strip-local components by
//     union-find in LDS over horizontal runs of linked blocks (a root is
//     hooked under the smaller root, so every root is its component's
//     smallest block), enters every non-edge component into a slot table --
//     {label, block count} and its lowest block row + 1 -- writes each
//     block's {statistics, slot}, and lists the join candidates across the
//     boundary above it;
//   merge: one workgroup joins slots across strip boundaries (union-find over
//     slots, again rooted at the smallest label), sums counts and takes the
//     lowest row per merged component, picks the background and writes each
//     slot's final label and depth.  With more than kRegionSlots slots it
//     runs regions_body instead, for the whole frame;
//   final (only for the per-block dump): one lane per block turns its slot
//     into the final label and depth.  The depth filter resolves the depths
//     it needs from the slot table itself.

constexpr int kStripLanes = 1024;
constexpr int kStripBlocks = 2048;

__device__ __forceinline__ uint32_t ufl_find(uint32_t* par, uint32_t x) {
    while (true) {
        const uint32_t p = lds_load(&par[x]);
        if (p == x) return x;
        const uint32_t gp = lds_load(&par[p]);
        if (gp != p) lds_store(&par[x], gp);
        x = gp;
    }
}

// Join the sets of a and b, hooking the root with the larger key under the
// other (key: the index itself, or key[] when given).
__device__ __forceinline__ void ufl_unite(uint32_t* par, uint32_t a, uint32_t b, const uint32_t* key) {
    while (true) {
        a = ufl_find(par, a);
        b = ufl_find(par, b);
        if (a == b) return;
        const uint32_t ka = key ? key[a] : a, kb = key ? key[b] : b;
        if (ka < kb) { const uint32_t t = a; a = b; b = t; }
        if (atomicCAS(&par[a], a, b) == a) return;
    }
}

__device__ __forceinline__ bool linked(uint32_t s, uint32_t n, int tau) {
    return !((s | n) >> 24) && (int)__builtin_amdgcn_sad_u8(s, n, 0u) <= tau;
}

// Lanes with `pred` take consecutive numbers 1, 2, ... from the LDS counter
// *ctr (one atomic per wave); 0 for the others.
__device__ __forceinline__ uint32_t wave_claim(uint32_t* ctr, bool pred) {
    const unsigned long long m = __ballot(pred);
    if (!m) return 0u;
    const int lead = __ffsll((long long)m) - 1;
    uint32_t b = 0;
    if ((int)(threadIdx.x & 63) == lead) b = atomicAdd(ctr, (uint32_t)__popcll(m));
    b = __builtin_amdgcn_readlane(b, lead);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    return pred ? b + below + 1u : 0u;
}

__host__ __device__ constexpr size_t rg_strip_lds_words() { return 3 * kStripBlocks + 3 * kStripBlocks + 4; }

__device__ __forceinline__ void rg_strip_body(const FrameDesc& f, int strip, uint32_t* lds) {
    const int gw = f.gw, gh = f.gh, SR = f.rstrip;
    const int t = threadIdx.x;
    const int r0 = strip * SR;
    const int rows = min(SR, gh - r0);
    const int n = rows * gw, base = r0 * gw;
    const int nload = (r0 + rows < gh ? rows + 1 : rows) * gw;
    uint32_t* st = lds;                      // statistics of the strip and the row below
    uint32_t* sa = st + 2 * kStripBlocks;    // statistics of the row above the strip
    uint32_t* par = sa + kStripBlocks;       // union-find
    uint32_t* cnt = par + kStripBlocks;      // per root: non-edge blocks
    uint32_t* row = cnt + kStripBlocks;      // per root: lowest local row + 1
    uint32_t* misc = row + kStripBlocks;     // [0]: slots of this strip, [1]: its first slot,
                                             // [2]: its join candidates, [3]: their first entry
    uint32_t* starts = cnt;                  // run-start bits, 32 blocks per word (before the counts)
    const uint32_t gwm = gw > 1 ? (uint32_t)((0x100000000ull + (uint32_t)gw - 1) / (uint32_t)gw) : 0u;

    for (int j = t; j < nload; j += kStripLanes) st[j] = f.stats[base + j];
    if (r0 > 0)
        for (int j = t; j < gw; j += kStripLanes) sa[j] = f.stats[base - gw + j];
    for (int j = t; j < n; j += kStripLanes) par[j] = j;
    if (t == 0) {
        misc[0] = 0;
        misc[2] = 0;
    }
    __syncthreads();

    // horizontal runs: block j starts a run unless it is right-linked from
    // j - 1 in the same row; the start bits of a wave's 64 consecutive blocks
    // come from one ballot
    int xk[2];
    bool dk[2];  // down link inside the strip
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int j = t + k * kStripLanes;
        const bool in = j < n;
        const int x = in ? j - (int)div_u16((uint32_t)j, gwm, (uint32_t)gw) * gw : 0;
        xk[k] = x;
        const uint32_t sj = in ? st[j] : 0u;
        dk[k] = in && j + gw < n && linked(sj, st[j + gw], f.tau);
        const bool start = in && (x == 0 || !linked(st[j - 1], sj, f.tau));
        const unsigned long long m = __ballot(start);
        if ((t & 63) == 0 && j < n) {
            starts[j >> 5] = (uint32_t)m;
            starts[(j >> 5) + 1] = (uint32_t)(m >> 32);
        }
    }
    __syncthreads();
    // the start of block i's run: the last start bit at or before i (every
    // row's first block is one).  Each wave keeps, in its own slice of the
    // row array (unused until the counts), the last start at or before the
    // end of every 32-block word (a max-scan over the words, n <= 2048), so a
    // lookup reads at most two words
    uint32_t* lastw = row + 64 * (t >> 6);
    {
        const int w = t & 63;
        const uint32_t word = w < ((n + 31) >> 5) ? starts[w] : 0u;
        int v = word ? w * 32 + 31 - __clz(word) : -1;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(v, o);
            if (w >= o) v = max(v, u);
        }
        lastw[w] = (uint32_t)v;
    }
    auto run_of = [&](int i) -> uint32_t {
        const int w = i >> 5;
        const uint32_t m = starts[w] & ((((uint32_t)1u << (i & 31)) << 1) - 1u);
        return m ? (uint32_t)(w * 32 + 31 - __clz(m)) : lastw[w - 1];
    };

    // unions between runs along the down links inside the strip, one per
    // place where the pair of runs above and below changes
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int j = t + k * kStripLanes;
        if (!dk[k]) continue;
        if (xk[k] > 0 && linked(st[j - 1], st[j], f.tau) && linked(st[j - 1 + gw], st[j + gw], f.tau) &&
            linked(st[j - 1], st[j - 1 + gw], f.tau))
            continue;
        ufl_unite(par, run_of(j), run_of(j + gw), nullptr);
    }
    __syncthreads();

    // roots (= smallest block of each component, its first run's start);
    // per root the non-edge count and lowest row, one atomic per wave when
    // the wave's non-edge blocks share a root
    uint32_t root[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int j = t + k * kStripLanes;
        root[k] = j < n ? ufl_find(par, run_of(j)) : 0u;
    }
    __syncthreads();  // the run bits are read; the counts take their place
    for (int j = t; j < n; j += kStripLanes) {
        cnt[j] = 0;
        row[j] = 0;
    }
    __syncthreads();
    // per root the non-edge count and lowest row: one pair of atomics per
    // distinct root in a wave (its blocks are consecutive, so the highest
    // lane holds the lowest row); slots for the non-edge roots and entries
    // for the join candidates across the boundary above the strip -- the
    // down links from the row above into the first row, except where block
    // x - 1 links the same pair of components (right links in both rows and
    // a down link) -- numbered one atomic per wave
    uint32_t slot[2], cand[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int j = t + k * kStripLanes;
        const bool ne = j < n && !(st[j] >> 24);
        const uint32_t lrow = j < n ? div_u16((uint32_t)j, gwm, (uint32_t)gw) + 1u : 0u;
        for (unsigned long long todo = __ballot(ne); todo;) {
            const int lead = __ffsll((long long)todo) - 1;
            const uint32_t r = __builtin_amdgcn_readlane(root[k], lead);
            const unsigned long long m = __ballot(ne && root[k] == r);
            const uint32_t mr = __builtin_amdgcn_readlane(lrow, 63 - __clzll(m));
            if ((t & 63) == lead) {
                atomicAdd(&cnt[r], (uint32_t)__popcll(m));
                atomicMax(&row[r], mr);
            }
            todo &= ~m;
        }
        slot[k] = wave_claim(&misc[0], ne && root[k] == (uint32_t)j);
        bool c = r0 > 0 && j < gw && linked(sa[j], st[j], f.tau);
        if (c && j > 0 && linked(sa[j - 1], st[j - 1], f.tau) && linked(sa[j - 1], sa[j], f.tau) &&
            linked(st[j - 1], st[j], f.tau))
            c = false;
        cand[k] = wave_claim(&misc[2], c);
    }
    __syncthreads();
    if (t == 0) {
        misc[1] = atomicAdd(&f.rctl[0], misc[0]);
        if (r0 > 0) misc[3] = atomicAdd(&f.rctl[2], misc[2]);
    }
    __syncthreads();
    const uint32_t first = misc[1];
    // each root's slot replaces its union-find entry (the finds are done)
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int j = t + k * kStripLanes;
        if (!slot[k]) continue;
        const uint32_t sidx = first + slot[k] - 1u;
        par[j] = sidx;
        if (sidx < (uint32_t)kRegionSlots) {
            f.rent[sidx] = make_uint2((uint32_t)(base + j), cnt[j]);
            f.rrow[sidx] = (uint32_t)r0 + row[j];
        }
    }
    __syncthreads();
    // per block: statistics and the slot of its component (0 for edge blocks)
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int j = t + k * kStripLanes;
        if (j >= n) continue;
        const uint32_t s = st[j];
        f.binfo[base + j] = make_uint2(s, (s >> 24) ? 0u : par[root[k]]);
    }

    if (r0 > 0) {
        const uint32_t bfirst = misc[3];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int x = t + k * kStripLanes;
            if (!cand[k]) continue;
            const uint32_t idx = bfirst + cand[k] - 1u;
            if (idx < (uint32_t)kBoundSlots) f.rbnd[idx] = make_uint2((uint32_t)(base - gw + x), par[root[k]]);
        }
    }
}

__host__ __device__ constexpr size_t rg_merge_lds_words() { return 4 * (size_t)kRegionSlots + 4; }

__device__ __forceinline__ void rg_merge_body(const FrameDesc& f, uint32_t* lds) {
    const int t = threadIdx.x, lane = t & 63;
    const uint32_t nslot = f.rctl[0];
    if (nslot > (uint32_t)kRegionSlots) {
        // too many strip-local components: group the whole frame here
        regions_body(f, lds);
        __syncthreads();
        if (t == 0) {
            f.rctl[0] = 0;
            f.rctl[1] = 1;
            f.rctl[2] = 0;
        }
        return;
    }
    const int ns = (int)nslot;
    const int gw = f.gw, gh = f.gh, SR = f.rstrip;
    uint32_t* par = lds;
    uint32_t* lab = par + kRegionSlots;
    uint32_t* cnt = lab + kRegionSlots;
    uint32_t* row = cnt + kRegionSlots;
    uint32_t* misc = row + kRegionSlots;  // [0]: background key
    // the strips' join candidates (each a slot below and the block above,
    // whose slot is a dependent load) are fetched while the slots load
    const uint32_t ncand = f.rctl[2];
    constexpr int CU = kBoundSlots / kStripLanes;
    const bool listed = ncand <= (uint32_t)kBoundSlots;
    uint32_t ca[CU], cb[CU];
    if (listed) {
        uint2 e[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u)
            if (t + u * kStripLanes < (int)ncand) e[u] = f.rbnd[t + u * kStripLanes];
#pragma unroll
        for (int u = 0; u < CU; ++u)
            if (t + u * kStripLanes < (int)ncand) {
                ca[u] = f.binfo[e[u].x].y;
                cb[u] = e[u].y;
            }
    }
    for (int s = t; s < ns; s += kStripLanes) {
        const uint2 e = f.rent[s];
        par[s] = s;
        lab[s] = e.x;
        cnt[s] = e.y;
        row[s] = f.rrow[s];
    }
    if (t == 0) misc[0] = 0;
    __syncthreads();

    // joins across strip boundaries: the down link from the last row of a
    // strip to the first row of the next, skipped where the left neighbour
    // links the same pair of strip-local components
    const int nbnd = (gh + SR - 1) / SR - 1;
    const int total = nbnd * gw;
    const uint32_t gwm = gw > 1 ? (uint32_t)((0x100000000ull + (uint32_t)gw - 1) / (uint32_t)gw) : 0u;
    if (listed) {
        // the strips' compacted join candidates
#pragma unroll
        for (int u = 0; u < CU; ++u)
            if (t + u * kStripLanes < (int)ncand) ufl_unite(par, ca[u], cb[u], lab);
    } else
    // every boundary position, four per lane at a time, every global load of
    // the four issued before any is used
    for (int q0 = t; q0 < total; q0 += 4 * kStripLanes) {
        // {statistics, slot} of the two blocks and of their left neighbours
        uint2 eb[4], ec[4], eb1[4], ec1[4];
        int xs[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = q0 + u * kStripLanes;
            const int qq = q < total ? q : 0;
            const int kb = (int)div_u16((uint32_t)qq, gwm, (uint32_t)gw);
            const int x = qq - kb * gw;
            const int b = ((kb + 1) * SR - 1) * gw + x, c = b + gw;
            const int bl = x > 0 ? b - 1 : b, cl = x > 0 ? c - 1 : c;
            xs[u] = q < total ? x : -1;
            eb[u] = f.binfo[b];
            ec[u] = f.binfo[c];
            eb1[u] = f.binfo[bl];
            ec1[u] = f.binfo[cl];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            bool join = xs[u] >= 0 && linked(eb[u].x, ec[u].x, f.tau);
            if (join && xs[u] > 0 && linked(eb1[u].x, ec1[u].x, f.tau) && eb1[u].y == eb[u].y && ec1[u].y == ec[u].y)
                join = false;
            if (join) ufl_unite(par, eb[u].y, ec[u].y, lab);
        }
    }
    __syncthreads();

    // merged component totals at the roots (the root holds the smallest label)
    for (int s = t; s < ns; s += kStripLanes) {
        const uint32_t r = ufl_find(par, s);
        if (r != (uint32_t)s) {
            atomicAdd(&cnt[r], cnt[s]);
            atomicMax(&row[r], row[s]);
        }
    }
    __syncthreads();
    uint32_t best = 0;
    for (int s = t; s < ns; s += kStripLanes)
        if (par[s] == (uint32_t)s) best = max(best, (cnt[s] << 16) | (0xFFFFu - lab[s]));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) best = max(best, (uint32_t)__shfl_xor((int)best, o));
    if (lane == 0 && best) atomicMax(&misc[0], best);
    __syncthreads();
    const uint32_t bgkey = misc[0];
    const uint32_t bg = bgkey ? 0xFFFFu - (bgkey & 0xFFFFu) : 0xFFFFFFFFu;
    for (int s = t; s < ns; s += kStripLanes) {
        const uint32_t r = ufl_find(par, s);
        const uint32_t L = lab[r];
        const uint32_t d = (uint32_t)ramp((int)row[r] - 1, gh);
        f.rfin[s] = (L << 9) | ((L == bg ? 1u : 0u) << 8) | d;
    }
    __syncthreads();
    if (t == 0) {
        f.rctl[0] = 0;
        f.rctl[1] = 0;
        f.rctl[2] = 0;
    }
}

// One block per lane: final label and depth from the block's slot.
__device__ __forceinline__ void rg_final_block(const FrameDesc& f, int b) {
    const int gw = f.gw, gh = f.gh;
    if (b >= gw * gh || f.rctl[1]) return;
    uint32_t* binfo_w = reinterpret_cast<uint32_t*>(f.binfo);
    const uint32_t s = binfo_w[2 * b];
    const int by = b / gw;
    uint32_t label = (uint32_t)b;
    int d;
    if (s >> 24) {
        d = ramp(by, gh);
    } else {
        const uint32_t v = f.rfin[binfo_w[2 * b + 1]];
        label = v >> 9;
        d = ((v >> 8) & 1u) ? ramp(by, gh) : (int)(v & 255u);
    }
    binfo_w[2 * b + 1] = (uint32_t)d;
    f.labels[b] = (int32_t)label;
}

}  // namespace pstereo
