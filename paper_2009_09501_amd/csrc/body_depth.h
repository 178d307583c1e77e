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

#include "device_common.h"

namespace pstereo {

// ---------------------------------------------------------------------------
// block statistics: per K x K block, rounded mean colour and edge flag.
//
// Tiles of 64 x 64 px, 256 lanes: lane = one quad (4 px) in each of four
// rows 16 apart, so K | 64 keeps every block inside one tile.
// Horizontal luma steps use the next pixel's bytes; vertical steps go through
// an LDS tile of packed luma that also holds the first row below the tile.
// The lanes of one block reduce by cross-lane xor within the wave, then one
// LDS atomic per wave and block.
template <int K>
struct BsTile {
    static constexpr int TH = 64;               // tile rows
    static constexpr int RPT = 4;               // consecutive rows per lane
    static constexpr int BC = 64 / K;           // block columns per tile
    static constexpr int BR = TH / K;           // block rows per tile
    static constexpr int QB = K / 4;            // quads per block row
    static constexpr int LB = K / RPT;          // lane rows per block
    static constexpr bool kInWave = LB <= 4;    // a block's lanes lie in one wave (K <= 16)
    // luma of each lane row's first row; block sums of blocks spanning waves
    static constexpr int kLdsWords = 16 * 16 + (kInWave ? 0 : BC * BR * 4);
};

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

// One 64 x 64 tile (tile_x, tile_y) on 256 lanes t = 0..255 (a multiple of
// four whole waves): lane t takes quad t % 16 of the four consecutive rows
// from 4 (t / 16), all four rows' loads in flight together, and sums them in
// registers; a block's lanes then combine by lane shuffles (blocks spanning
// waves through LDS atomics as well).  lds: BsTile<K>::kLdsWords words.
// Inactive lane groups (active == false) do no memory work but pass the same
// barriers.
template <int K, bool ALIGNED>
__device__ __forceinline__ void bs_tile(const FrameDesc& f, int tile_x, int tile_y, int t, uint32_t* lds,
                                        bool active) {
    using T = BsTile<K>;
    constexpr int RPT = T::RPT, QB = T::QB, LB = T::LB;
    uint32_t* yfirst = lds;     // [lane row][quad]
    uint32_t* acc = lds + 256;  // blocks spanning waves: r, g, b, edge
    const int W = f.w, H = active ? f.h : 0;
    const int qx = t & 15, lr = t >> 4;
    const int tx0 = tile_x * 64, ty0 = tile_y * T::TH;
    const int x0 = tx0 + 4 * qx, y0 = ty0 + RPT * lr;
    const int n = ALIGNED ? 4 : min(4, W - x0);  // aligned frames hold whole quads
    const uint32_t g = (uint32_t)f.g;
    if (!T::kInWave)
        for (int i = t; i < T::BC * T::BR * 4; i += 256) acc[i] = 0;

    // edge: the block has a luma step above g; emax: the largest step seen
    // by the aligned path (compared with g once at the end)
    uint32_t sr = 0, sg = 0, sb = 0, edge = 0, emax = 0;
    uint32_t yq[RPT];     // packed luma bytes of the lane's quad, one word per row
    uint32_t ybelow = 0;  // the row below the tile (last lane row only)
    if (ALIGNED) {
        uint3 v[RPT + 1];
        uint32_t nx[RPT];
        // the lane's quad in its first row; the next rows one uniform row
        // stride apart
        const uint8_t* p0 = f.frame + ((size_t)y0 * W + x0) * 3;
        const size_t stride = (size_t)W * 3;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int y = y0 + k;
            if (y < H && x0 < W) {
                const uint8_t* p = p0 + k * stride;
                v[k] = *reinterpret_cast<const uint3*>(p);
                if (x0 + 4 < W) nx[k] = *reinterpret_cast<const uint32_t*>(p + 12);
            }
        }
        if (lr == 15 && ty0 + T::TH < H && x0 < W)
            v[RPT] = *reinterpret_cast<const uint3*>(f.frame + ((size_t)(ty0 + T::TH) * W + x0) * 3);
        constexpr uint32_t wlo = 77u | (150u << 8) | (29u << 16);
        auto quad_luma = [&](uint3 q, uint32_t (&Y)[4]) {
            Y[0] = __builtin_amdgcn_udot4(q.x, wlo, 128u, false) >> 8;
            Y[1] = __builtin_amdgcn_udot4(__builtin_amdgcn_alignbyte(q.y, q.x, 3), wlo, 128u, false) >> 8;
            Y[2] = __builtin_amdgcn_udot4(__builtin_amdgcn_alignbyte(q.z, q.y, 2), wlo, 128u, false) >> 8;
            Y[3] = __builtin_amdgcn_udot4(q.z, wlo << 8, 128u, false) >> 8;
        };
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const bool in = y0 + k < H && x0 < W;
            yq[k] = 0;
            if (!in) continue;
            // four pixels = three dwords; sums and luma by byte dot products
            sr = __builtin_amdgcn_udot4(v[k].x, 0x01000001u, sr, false);
            sr = __builtin_amdgcn_udot4(v[k].y, 0x00010000u, sr, false);
            sr = __builtin_amdgcn_udot4(v[k].z, 0x00000100u, sr, false);
            sg = __builtin_amdgcn_udot4(v[k].x, 0x00000100u, sg, false);
            sg = __builtin_amdgcn_udot4(v[k].y, 0x01000001u, sg, false);
            sg = __builtin_amdgcn_udot4(v[k].z, 0x00010000u, sg, false);
            sb = __builtin_amdgcn_udot4(v[k].x, 0x00010000u, sb, false);
            sb = __builtin_amdgcn_udot4(v[k].y, 0x00000100u, sb, false);
            sb = __builtin_amdgcn_udot4(v[k].z, 0x01000001u, sb, false);
            uint32_t Y[4];
            quad_luma(v[k], Y);
            const uint32_t Yn = x0 + 4 < W ? __builtin_amdgcn_udot4(nx[k], wlo, 128u, false) >> 8 : Y[3];  // no step past the last column
            const uint32_t hmax = max(max(__builtin_amdgcn_sad_u16(Y[1], Y[0], 0u), __builtin_amdgcn_sad_u16(Y[2], Y[1], 0u)),
                                      max(__builtin_amdgcn_sad_u16(Y[3], Y[2], 0u), __builtin_amdgcn_sad_u16(Yn, Y[3], 0u)));
            emax = max(emax, hmax);
            yq[k] = Y[0] | (Y[1] << 8) | (Y[2] << 16) | (Y[3] << 24);
        }
        if (lr == 15 && ty0 + T::TH < H && x0 < W) {
            uint32_t Y[4];
            quad_luma(v[RPT], Y);
            ybelow = Y[0] | (Y[1] << 8) | (Y[2] << 16) | (Y[3] << 24);
        }
    } else {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int y = y0 + k;
            yq[k] = 0;
            if (y < H && x0 < W) {
                const uint8_t* p = f.frame + ((size_t)y * W + x0) * 3;
                int r[4], gg[4], b[4], Y[4];
                load_quad<false>(p, n, r, gg, b);
                int ynext = 0;
                if (x0 + 4 < W) ynext = luma(p[12], p[13], p[14]);
#pragma unroll
                for (int j = 0; j < 4; ++j) Y[j] = luma(r[j], gg[j], b[j]);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (j < n) {
                        sr += r[j]; sg += gg[j]; sb += b[j];
                        yq[k] |= (uint32_t)Y[j] << (8 * j);
                        if (x0 + j + 1 < W && iabs((j < 3 ? Y[j + 1] : ynext) - Y[j]) > f.g) edge = 1;
                    }
                }
            }
        }
        if (lr == 15 && ty0 + T::TH < H && x0 < W) {
            int r[4], gg[4], b[4];
            load_quad<false>(f.frame + ((size_t)(ty0 + T::TH) * W + x0) * 3, n, r, gg, b);
#pragma unroll
            for (int j = 0; j < 4; ++j) if (j < n) ybelow |= (uint32_t)luma(r[j], gg[j], b[j]) << (8 * j);
        }
    }
    yfirst[lr * 16 + qx] = yq[0];
    __syncthreads();
    // vertical steps: rows inside the lane's four, then the next lane row's
    // first row (the row below the tile for the last lane row)
    const uint32_t below_last = lr < 15 ? yfirst[(lr + 1) * 16 + qx] : ybelow;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int y = y0 + k;
        if (y + 1 < H && x0 < W) {
            const uint32_t below = k + 1 < RPT ? yq[k + 1] : below_last;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (j < n) emax = max(emax, __builtin_amdgcn_sad_u16((below >> (8 * j)) & 255u, (yq[k] >> (8 * j)) & 255u, 0u));
        }
    }
    if (emax > g) edge = 1;
    const int bxl = qx / QB, byl = lr / LB;  // the lane's block in the tile
    if (T::kInWave) {
        // two 16-bit sums per register: a block holds K * K / 16 <= 16 lanes
        // of at most 16 pixels, 16 x 16 x 255 < 2^16
        uint32_t rg = sr | (sg << 16), be = sb | (edge << 16);
#pragma unroll
        for (int o = 1; o < QB; o <<= 1) {
            rg += __shfl_xor(rg, o);
            be += __shfl_xor(be, o);
        }
#pragma unroll
        for (int o = 1; o < LB; o <<= 1) {
            rg += __shfl_xor(rg, 16 * o);
            be += __shfl_xor(be, 16 * o);
        }
        const int bx = tile_x * T::BC + bxl, by = tile_y * T::BR + byl;
        if (active && qx % QB == 0 && lr % LB == 0 && bx < f.gw && by < f.gh) {
            const uint32_t cnt = (uint32_t)((min(bx * K + K, W) - bx * K) * (min(by * K + K, H) - by * K));
            const uint32_t mr = block_mean<K>((rg & 0xFFFFu), cnt);
            const uint32_t mg = block_mean<K>((rg >> 16), cnt);
            const uint32_t mb = block_mean<K>((be & 0xFFFFu), cnt);
            f.stats[by * f.gw + bx] = mr | (mg << 8) | (mb << 16) | ((be >> 16) ? 1u << 24 : 0u);
        }
    } else {
        // the wave's share of each block (four lane rows), then across waves
#pragma unroll
        for (int o = 1; o < QB; o <<= 1) {
            sr += __shfl_xor(sr, o);
            sg += __shfl_xor(sg, o);
            sb += __shfl_xor(sb, o);
            edge |= __shfl_xor(edge, o);
        }
#pragma unroll
        for (int o = 16; o < 64; o <<= 1) {
            sr += __shfl_xor(sr, o);
            sg += __shfl_xor(sg, o);
            sb += __shfl_xor(sb, o);
            edge |= __shfl_xor(edge, o);
        }
        if (qx % QB == 0 && (lr & 3) == 0) {
            const int blk = bxl + T::BC * byl;
            atomicAdd(&acc[4 * blk + 0], sr);
            atomicAdd(&acc[4 * blk + 1], sg);
            atomicAdd(&acc[4 * blk + 2], sb);
            if (edge) atomicOr(&acc[4 * blk + 3], 1u);
        }
        __syncthreads();
        for (int i = t; i < T::BC * T::BR; i += 256) {
            const int bx = tile_x * T::BC + i % T::BC, by = tile_y * T::BR + i / T::BC;
            if (active && bx < f.gw && by < f.gh) {
                const uint32_t cnt = (uint32_t)((min(bx * K + K, W) - bx * K) * (min(by * K + K, H) - by * K));
                const uint32_t mr = block_mean<K>(acc[4 * i + 0], cnt);
                const uint32_t mg = block_mean<K>(acc[4 * i + 1], cnt);
                const uint32_t mb = block_mean<K>(acc[4 * i + 2], cnt);
                f.stats[by * f.gw + bx] = mr | (mg << 8) | (mb << 16) | (acc[4 * i + 3] << 24);
            }
        }
    }
}

// Block statistics for blocks of 2 x 2 px (frames of at most 2^17 pixels,
// so this path is never the bulk of the work): the same 64 x 64 px tiles on
// 256 lanes; lane t takes block column t % 32 of the tile's 32 x 32 blocks in
// block rows t / 32 + 8 k, k = 0..3, reading pixels bytewise and the luma
// steps to the right and below directly.  No barriers.
__device__ __forceinline__ void bs_tile_k2(const FrameDesc& f, int tile_x, int tile_y, int t, bool active) {
    if (!active) return;
    const int W = f.w, H = f.h;
    const int bx = tile_x * 32 + (t & 31);
    if (bx >= f.gw) return;
    for (int k = 0; k < 4; ++k) {
        const int by = tile_y * 32 + (t >> 5) + 8 * k;
        if (by >= f.gh) break;
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
