// Device bodies of the stereo rendering: filtered depth, then both views
// (used by the per-frame kernels and by the persistent batch kernel).
//
//   k_cbf   pixel depth (from the block tables) and its cross-bilateral
//           filter guided by luma (Section 3: filtered depth map; Section 4:
//           GPU cross-bilateral filtering), on 64 x 16 pixel tiles with a
//           halo in LDS.  Windows whose depths are all equal take the exact
//           shortcut; the other quads are compacted into a workgroup list so
//           that only they pay for the weighted sum.  Output: filtered depth,
//           one byte per pixel, in a scratch buffer.
//   k_warp  one image row per workgroup: left / right frame reconstruction
//           (Section 4, Fig. 3 code: depth -> shift, threshold T, half the
//           stereo base per view) as a forward warp whose z-buffer is an LDS
//           atomic max on (depth << 24 | RGB) -- the nearer source wins and
//           its colour travels in the key; then inpainting of the holes
//           (Section 3: post-processed frames) from the nearer valid pixel
//           of the row, found with wave ballots; then anaglyph composition
//           (Fig. 3 code: red from the left view, green and blue from the
//           right) and RGB24 stores.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>

#include "device_common.h"

namespace pstereo {

// Distinct squared distances dx^2 + dy^2 inside a (2r+1)^2 window, r <= 3.
__host__ __device__ constexpr int k_value(int i) {
    return i == 0 ? 0 : i == 1 ? 1 : i == 2 ? 2 : i == 3 ? 4 : i == 4 ? 5 : i == 5 ? 8
         : i == 6 ? 9 : i == 7 ? 10 : i == 8 ? 13 : 18;
}
__host__ __device__ constexpr int k_index(int k) {
    return k == 0 ? 0 : k == 1 ? 1 : k == 2 ? 2 : k == 4 ? 3 : k == 5 ? 4 : k == 8 ? 5
         : k == 9 ? 6 : k == 10 ? 7 : k == 13 ? 8 : 9;
}
__host__ __device__ constexpr int k_count(int r) { return r == 0 ? 1 : r == 1 ? 3 : r == 2 ? 6 : 10; }

// Product weights ws(k) * wr(|d|) of the cross-bilateral filter for every
// distinct squared distance k (k_index order) and signed luma difference
// d = -255..255.  In LDS row k holds 512 u16 entries, entry d + 255 (the last
// one unused), two to a word; the table for radius r is the prefix of
// k_count(r) rows.  Indexed by the signed difference, a tap's entry sits at
// byte offset 2 Yq + (510 - 2 Yp) of its row (doubled luma), one add per tap.
__host__ __device__ constexpr uint32_t cbf_w(int k, int j) {
    return j < 511 ? spatial_w(k_value(k)) * range_w(j < 255 ? 255 - j : j - 255) : 0u;
}
// The range weight is 0 from |d| = kRangeTaps on, so only words kCbfW0 ..
// kCbfW0 + kCbfWords - 1 of a row are non-zero; global memory holds just
// those, in kCbfCopies copies that successive workgroups take in turn (every
// workgroup reads the table, and one copy would sit in few L2 channels).
constexpr int kRangeTaps = 43;
constexpr int kCbfW0 = (255 - (kRangeTaps - 1)) / 2;             // 106
constexpr int kCbfWords = (255 + (kRangeTaps - 1)) / 2 + 1 - kCbfW0;  // 43
constexpr int kCbfCopies = 32;
static_assert(range_w(kRangeTaps) == 0 && range_w(kRangeTaps - 1) != 0, "range weight support");
struct CbfWeightTable {
    uint32_t w[kCbfCopies][10 * kCbfWords];
};
__host__ __device__ constexpr CbfWeightTable make_cbf_weights() {
    CbfWeightTable t{};
    for (int k = 0; k < 10; ++k)
        for (int i = 0; i < kCbfWords; ++i) {
            const int j = 2 * (kCbfW0 + i);
            t.w[0][k * kCbfWords + i] = cbf_w(k, j) | cbf_w(k, j + 1) << 16;
        }
    for (int c = 1; c < kCbfCopies; ++c)
        for (int i = 0; i < 10 * kCbfWords; ++i) t.w[c][i] = t.w[0][i];
    return t;
}
__device__ const CbfWeightTable kCbfWeights = make_cbf_weights();

// Depth -> (left offset, right offset) of the Fig. 3 rule with the rounding
// reading: P = round(B*m/255), m = D when D > T (crossed) else 255 - D
// (uncrossed); the left view moves by ceil(P/2), the right view by floor(P/2),
// in opposite directions.  Packed as (oL & 0xFFFF) | (oR << 16).
__device__ __forceinline__ uint32_t shift_entry(int d, int B, int T) {
    const bool crossed = d > T;
    const int m = crossed ? d : 255 - d;
    const int P = (B * m + 127) / 255;
    const int a = (P + 1) >> 1, b = P >> 1;
    const int oL = crossed ? a : -a;
    const int oR = crossed ? -b : b;
    return ((uint32_t)oL & 0xFFFFu) | ((uint32_t)oR << 16);
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Packed-integer helpers (single gfx950 instructions).
__device__ __forceinline__ uint32_t dot2_u16(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, a), __builtin_bit_cast(u16x2, b), c, false);
}
__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) { return __builtin_amdgcn_perm(hi, lo, sel); }
__device__ __forceinline__ uint32_t alignbyte(uint32_t hi, uint32_t lo, uint32_t s) { return __builtin_amdgcn_alignbyte(hi, lo, s); }

// The four RGB24 pixels of a quad held in three dwords, as four R | G << 8 |
// B << 16 words (top byte zero).
__device__ __forceinline__ void quad_colours(uint3 v, uint32_t (&c)[4]) {
    c[0] = v.x & 0xFFFFFFu;
    c[1] = alignbyte(v.y, v.x, 3) & 0xFFFFFFu;
    c[2] = alignbyte(v.z, v.y, 2) & 0xFFFFFFu;
    c[3] = v.z >> 8;
}

// Luma of the four pixels of an aligned quad, doubled, as u16 pairs
// (2Y0 | 2Y1 << 16, 2Y2 | 2Y3 << 16).  Luma = byte 1 of 77R + 150G + 29B + 128.
__device__ __forceinline__ void quad_luma2(uint3 v, uint32_t& y01, uint32_t& y23) {
    constexpr uint32_t wlo = 77u | (150u << 8) | (29u << 16);  // R, G, B in bytes 0..2
    constexpr uint32_t whi = wlo << 8;                         // R, G, B in bytes 1..3
    const uint32_t r0 = __builtin_amdgcn_udot4(v.x, wlo, 128u, false);
    const uint32_t r1 = __builtin_amdgcn_udot4(alignbyte(v.y, v.x, 3), wlo, 128u, false);
    const uint32_t r2 = __builtin_amdgcn_udot4(alignbyte(v.z, v.y, 2), wlo, 128u, false);
    const uint32_t r3 = __builtin_amdgcn_udot4(v.z, whi, 128u, false);
    y01 = perm(r1, r0, 0x0c050c01u) << 1;
    y23 = perm(r3, r2, 0x0c050c01u) << 1;
}

// Region depth of a block in row by after the strip-parallel grouping, from
// its {statistics, component slot}: edge blocks and the background follow
// the row ramp, other blocks take their merged component's depth.
__device__ __forceinline__ uint32_t block_depth_from_slots(const FrameDesc& f, int by, uint2 e) {
    if (e.x >> 24) return (uint32_t)ramp(by, f.gh);
    const uint32_t v = f.rfin[e.y];
    return ((v >> 8) & 1u) ? (uint32_t)ramp(by, f.gh) : (v & 255u);
}

// The search key of a block in the filter's staged table (second word of its
// entry): its region depth when it is a non-edge block, else kNoCandidate,
// which stays above every candidate's key (distance << 16 | index << 8 |
// depth, distance <= 765) with any index or distance added and does not
// overflow.
constexpr uint32_t kNoCandidate = 0xFC000000u;

// Raw depth of the four pixels of a quad: the region depth of their block, or
// for an edge block that of the non-edge 3x3 neighbour block whose mean colour
// is nearest (L1), first strict minimum in raster order; with no candidate
// the ramp of the block row.  col[j] = R | G << 8 | B << 16 of pixel j; the
// L1 distance to a block mean (stats word, edge byte zero for candidates) is
// one v_sad_u8.  The blocks come from a table staged in LDS: tab holds the
// blocks [bx_lo, bx_lo + bw) x [by_lo, ...), {statistics, search key}, and
// covers every in-grid block the lookup can touch; K = 1 << ks.
__device__ __forceinline__ void quad_depth_tab(const FrameDesc& f, int x0, int yy, int ks, const uint2* tab,
                                               int bx_lo, int by_lo, int bw, const uint32_t (&col)[4],
                                               uint32_t (&D)[4]) {
    const int bx = x0 >> ks, by = yy >> ks;
    const uint2 own = tab[(by - by_lo) * bw + (bx - bx_lo)];
    if (!(own.x >> 24)) {
#pragma unroll
        for (int j = 0; j < 4; ++j) D[j] = own.y;
        return;
    }
    // branch-free: per pixel the minimum of (distance << 16) + (k << 8 |
    // depth) over the candidates k in raster order (distance <= 765), so
    // that ties go to the first -- one v_sad_hi_u8 per candidate; a
    // non-candidate's key starts at kNoCandidate
    uint32_t best[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const uint2 c = tab[(by - by_lo + k / 3 - 1) * bw + (bx - bx_lo + k % 3 - 1)];
        const uint32_t tag = c.y | ((uint32_t)k << 8);
#pragma unroll
        for (int j = 0; j < 4; ++j) best[j] = min(best[j], __builtin_amdgcn_sad_hi_u8(col[j], c.x, tag));
    }
    // the ramp of the block row only where a pixel found no candidate (rare)
    bool none = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) none |= best[j] >= kNoCandidate;
    uint32_t fallback = 0;
    if (none) fallback = (uint32_t)ramp(by, f.gh);
#pragma unroll
    for (int j = 0; j < 4; ++j) D[j] = best[j] >= kNoCandidate ? fallback : (best[j] & 255u);
}

// Raw depth of the four pixels of a quad for blocks of 2 px (the quad spans
// two block columns): the same rule as quad_depth_tab, per pixel, from the
// block table in global memory (frames of 2 px blocks hold at most 2^17
// pixels, so this path is never the bulk of the work).  strips: block depths
// are resolved through the merge's slot table.
__device__ __forceinline__ uint2 block_entry_global(const FrameDesc& f, int bx, int by, bool strips) {
    if (bx < 0 || bx >= f.gw || by < 0 || by >= f.gh) return make_uint2(1u << 24, 0u);
    uint2 e = f.binfo[by * f.gw + bx];
    if (strips) e.y = block_depth_from_slots(f, by, e);
    return e;
}

__device__ __forceinline__ void quad_depth_k2(const FrameDesc& f, int x0, int yy, bool strips,
                                              const uint32_t (&col)[4], uint32_t (&D)[4]) {
    const int by = yy >> 1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int bx = (x0 + j) >> 1;
        const uint2 own = block_entry_global(f, bx, by, strips);
        if (!(own.x >> 24)) {
            D[j] = own.y;
            continue;
        }
        // first strict minimum of the L1 colour distance over the non-edge
        // blocks of the 3 x 3 neighbourhood, in raster order
        int best = -1;
        uint32_t bestd = 0, bestdep = 0;
        for (int k = 0; k < 9; ++k) {
            const uint2 c = block_entry_global(f, bx + k % 3 - 1, by + k / 3 - 1, strips);
            if (c.x >> 24) continue;
            const uint32_t d = __builtin_amdgcn_sad_u8(col[j], c.x, 0u);
            if (best < 0 || d < bestd) {
                best = k;
                bestd = d;
                bestdep = c.y;
            }
        }
        D[j] = best >= 0 ? bestdep : (uint32_t)ramp(by, f.gh);
    }
}

// ---------------------------------------------------------------------------
// k_cbf: 64 x 32 pixel tiles, 256 lanes; lane = one quad in each of two tile
// rows (ty and ty + 16).  LDS holds, for the tile and a 4 px / R row halo,
// doubled luma and raw depth as u16 pairs (two dwords per quad).  A window of
// quad x0 reads the six dwords of columns x0-4 .. x0+7 per row.
constexpr int kTileQ = 16;                   // quads per tile row
constexpr int kTileW = 4 * kTileQ;           // 64 px
constexpr int kTileH = 32;                   // rows
constexpr int kTileQuads = kTileQ + 2;       // quads per LDS row: one extra each side
constexpr int kRowWords = 2 * kTileQuads;    // 36 dwords per LDS row and plane

// Window of a pixel pair at an even LDS column c0: the words from the one
// holding column c0 - R through the one holding c0 + 1 + R.
template <int R>
struct CbfPairWin {
    static constexpr int kW0 = (R + 1) >> 1;  // words before c0's word
    static constexpr int kWords = (2 * kW0 + 1 + R) / 2 + 1;
};

// Filtered depth of the two pixels x0, x0 + 1 of one row.  yw / dw: the
// window words of each of the 2R + 1 rows, luma doubled and raw depth as u16
// pairs; pixel j sits at window column 2 kW0 + j, so every tap's word and half
// are compile-time constants.  Taps go in pairs (c, c + 1) of one word (c
// even; a pair's tap outside dx = -R..R has weight 0 and reads nothing), so
// the weighted depth sum and the weight sum each take one dot2 per pair on the
// word as stored.  CLIP: some window column lies outside the image and gets
// weight 0.
template <int R, bool CLIP>
__device__ __forceinline__ void cbf_pair(const uint32_t (&yw)[2 * R + 1][CbfPairWin<R>::kWords],
                                         const uint32_t (&dw)[2 * R + 1][CbfPairWin<R>::kWords], uint32_t rows_ok,
                                         int x0, int W, const uint16_t* wtab, uint32_t (&df)[2]) {
    constexpr int PW = CbfPairWin<R>::kWords;
    const uint8_t* wt = reinterpret_cast<const uint8_t*>(wtab);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int pc = 2 * CbfPairWin<R>::kW0 + j;
        // byte offset of a tap's weight in its table row: 2 Yq + (510 - 2 Yp)
        const uint32_t base = 510u - ((yw[R][pc >> 1] >> (16 * (pc & 1))) & 0xFFFFu);
        uint32_t acc = 0, wsum = 0;
#pragma unroll
        for (int dy = -R; dy <= R; ++dy) {
            if (!((rows_ok >> (dy + R)) & 1u)) continue;
            const uint32_t(&yr)[PW] = yw[dy + R];
            const uint32_t(&dr)[PW] = dw[dy + R];
#pragma unroll
            for (int dx = -R - ((pc - R) & 1); dx <= R; dx += 2) {
                const int c = pc + dx;  // even
                uint32_t w0 = 0, w1 = 0;
                if (dx >= -R) {
                    const uint32_t y0 = yr[c >> 1] & 0xFFFFu;
                    w0 = *reinterpret_cast<const uint16_t*>(wt + k_index(dx * dx + dy * dy) * 1024 + (y0 + base));
                    if (CLIP && (unsigned)(x0 + j + dx) >= (unsigned)W) w0 = 0;
                }
                if (dx + 1 <= R) {
                    const uint32_t y1 = yr[c >> 1] >> 16;
                    w1 = *reinterpret_cast<const uint16_t*>(wt + k_index((dx + 1) * (dx + 1) + dy * dy) * 1024 + (y1 + base));
                    if (CLIP && (unsigned)(x0 + j + dx + 1) >= (unsigned)W) w1 = 0;
                }
                const uint32_t wp = w0 | (w1 << 16);
                acc = dot2_u16(wp, dr[c >> 1], acc);
                wsum = dot2_u16(wp, 0x00010001u, wsum);
            }
        }
        df[j] = div_small_quotient(acc + (wsum >> 1), wsum);
    }
}

template <int R>
struct CbfTile {
    static constexpr int TR = kTileH + 2 * R;  // LDS rows incl. halo
    static constexpr int NK = k_count(R);
    // tY, tD: TR * kRowWords words each; wtab: NK * 512 u16; work: 512 u16; nwork
    // block table of the tile, its halo and one ring of neighbours: at most
    // 21 x 13 blocks (K = 4, R = 3), uint2 each
    static constexpr int kBlkEntries = 288;
    static constexpr int kBlkOff = (2 * TR * kRowWords + NK * 256 + 256 + 1 + 1) & ~1;  // 8-byte aligned
    static constexpr int kLdsWords = kBlkOff + 2 * kBlkEntries;
};

// A lane's frame loads for one tile: three raw dwords per quad of the tile
// and its halo (aligned frames; unaligned ones load bytes in the prologue).
template <int R>
struct CbfIn {
    static constexpr int NQ = (CbfTile<R>::TR * kTileQuads + 255) / 256;
    uint3 vq[NQ];
};

// Issue the loads of tile (tile_x, tile_y) for lane t; quads outside the
// image (or all, when H = 0) load nothing and are not read later.
template <int R, bool ALIGNED>
__device__ __forceinline__ void cbf_load(const FrameDesc& f, int tile_x, int tile_y, int t, int H, CbfIn<R>& in) {
    if (!ALIGNED) return;
    const int W = f.w, tx0 = tile_x * kTileW, ty0 = tile_y * kTileH;
#pragma unroll
    for (int k = 0; k < CbfIn<R>::NQ; ++k) {
        const int i = t + 256 * k;
        const int tr = i / kTileQuads, tq = i - tr * kTileQuads;
        const int yy = ty0 - R + tr, x0 = tx0 - 4 + 4 * tq;
        if (i < CbfTile<R>::TR * kTileQuads && yy >= 0 && yy < H && x0 >= 0 && x0 < W)
            in.vq[k] = *reinterpret_cast<const uint3*>(f.frame + ((size_t)yy * W + x0) * 3);
    }
}

// One 64 x 32 tile (tile_x, tile_y) on 256 lanes t = 0..255 (four whole
// waves).  lds: CbfTile<R>::kLdsWords words.  Inactive lane groups do no
// memory work but pass the same three barriers.  K2: blocks of 2 px (raw
// depth looked up per pixel in global memory, no block table in LDS).
template <int R, bool ALIGNED, bool K2 = false>
__device__ __forceinline__ void cbf_tile(const FrameDesc& f, int tile_x, int tile_y, int t, uint32_t* lds,
                                         bool active) {
    constexpr int S = 2 * R + 1;
    constexpr int TR = CbfTile<R>::TR;
    constexpr int NK = CbfTile<R>::NK;
    uint32_t* tY = lds;
    uint32_t* tD = tY + TR * kRowWords;
    uint16_t* wtab = reinterpret_cast<uint16_t*>(tD + TR * kRowWords);
    uint16_t* work = wtab + NK * 512;
    int* nwork_p = reinterpret_cast<int*>(work + 512);
    int& nwork = *nwork_p;
    uint2* btab = reinterpret_cast<uint2*>(lds + CbfTile<R>::kBlkOff);

    const int W = f.w, H = active ? f.h : 0;
    const int tx0 = tile_x * kTileW, ty0 = tile_y * kTileH;

    // the frame loads of all of a lane's quads of the tile and its halo go
    // out first, to arrive while the block table is staged
    constexpr int NQ = CbfIn<R>::NQ;
    CbfIn<R> in;
    cbf_load<R, ALIGNED>(f, tile_x, tile_y, t, H, in);

    // the non-zero words of the weight table likewise: lane t holds word t
    // of every row
    uint32_t wq[NK];
    {
        const uint32_t* src = kCbfWeights.w[(blockIdx.x + blockIdx.y) % kCbfCopies];
        const bool nz = (unsigned)(t - kCbfW0) < (unsigned)kCbfWords;
#pragma unroll
        for (int k = 0; k < NK; ++k) wq[k] = nz ? src[k * kCbfWords + t - kCbfW0] : 0u;
    }

    // the tile's block table (halo and one ring of neighbours, clipped to the
    // grid) into LDS, so the raw depth needs no global lookups
    // (clipped to the grid plus one ring outside it, whose entries are
    // marked as edge blocks)
    const int ks = __builtin_ctz((unsigned)f.K);
    const int bx_lo = max(-1, ((tx0 - 4) >> ks) - 1), bx_hi = min(f.gw, ((tx0 + 4 * kTileQuads - 5) >> ks) + 1);
    const int by_lo = max(-1, ((ty0 - R) >> ks) - 1), by_hi = min(f.gh, ((ty0 + kTileH - 1 + R) >> ks) + 1);
    const int bw = bx_hi - bx_lo + 1;
    if (!K2 && !f.depth_in && H > 0) {
        const int nbt = bw * (by_hi - by_lo + 1);
        // after the strip-parallel grouping (unless its merge grouped the
        // whole frame itself) a block's region depth is resolved here from
        // its component slot and the merge's slot table
        const bool strips = f.rstrip > 0 && f.rctl[1] == 0;
        for (int i = t; i < nbt; i += 256) {
            const int r = i / bw;
            const int by = by_lo + r, bx = bx_lo + (i - r * bw);
            uint2 e = make_uint2(1u << 24, kNoCandidate);
            if (by >= 0 && by < f.gh && bx >= 0 && bx < f.gw) {
                e = f.binfo[by * f.gw + bx];
                if (strips) e.y = block_depth_from_slots(f, by, e);
                if (e.x >> 24) e.y = kNoCandidate;  // an edge block is never a candidate
            }
            btab[i] = e;
        }
    }
#pragma unroll
    for (int k = 0; k < NK; ++k) reinterpret_cast<uint32_t*>(wtab)[k * 256 + t] = wq[k];
    if (t == 0) nwork = 0;
    __syncthreads();

    // doubled luma + raw depth of the tile and its halo (columns tx0-4 ..
    // tx0+67)
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        const int i = t + 256 * k;
        if (i >= TR * kTileQuads) break;
        const int tr = i / kTileQuads, tq = i - tr * kTileQuads;
        const int yy = ty0 - R + tr;
        const int x0 = tx0 - 4 + 4 * tq;
        uint32_t y01 = 0, y23 = 0, d01 = 0, d23 = 0;
        if (yy >= 0 && yy < H && x0 >= 0 && x0 < W) {
            const int n = min(4, W - x0);
            const uint8_t* p = f.frame + ((size_t)yy * W + x0) * 3;
            uint32_t col[4], D[4];
            if (ALIGNED) {
                const uint3 v = in.vq[k];
                quad_luma2(v, y01, y23);
                quad_colours(v, col);
            } else {
                uint32_t Y[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (j < n) {
                        Y[j] = 2u * (uint32_t)luma(p[3 * j], p[3 * j + 1], p[3 * j + 2]);
                        col[j] = p[3 * j] | ((uint32_t)p[3 * j + 1] << 8) | ((uint32_t)p[3 * j + 2] << 16);
                    } else {
                        Y[j] = 0;
                        col[j] = 0;
                    }
                }
                y01 = Y[0] | (Y[1] << 16);
                y23 = Y[2] | (Y[3] << 16);
            }
            if (f.depth_in) {
                const uint8_t* dp = f.depth_in + (size_t)yy * W + x0;
#pragma unroll
                for (int j = 0; j < 4; ++j) D[j] = j < n ? dp[j] : 0u;
            } else if (K2) {
                quad_depth_k2(f, x0, yy, f.rstrip > 0 && f.rctl[1] == 0, col, D);
            } else {
                quad_depth_tab(f, x0, yy, ks, btab, bx_lo, by_lo, bw, col, D);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) if (j >= n) D[j] = 0;
            d01 = D[0] | (D[1] << 16);
            d23 = D[2] | (D[3] << 16);
            if (f.out_d0 && tr >= R && tr < R + kTileH && tq >= 1 && tq <= kTileQ) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (j < n) f.out_d0[(size_t)yy * W + x0 + j] = (uint8_t)D[j];
            }
        }
        tY[tr * kRowWords + 2 * tq] = y01;
        tY[tr * kRowWords + 2 * tq + 1] = y23;
        tD[tr * kRowWords + 2 * tq] = d01;
        tD[tr * kRowWords + 2 * tq + 1] = d23;
    }
    __syncthreads();

    auto store_df = [&](int x0_, int y_, const uint32_t (&df)[4]) {
        const int n = min(4, W - x0_);
        const size_t o = (size_t)y_ * W + x0_;
        if (ALIGNED) {
            *reinterpret_cast<uint32_t*>(f.df + o) = df[0] | (df[1] << 8) | (df[2] << 16) | (df[3] << 24);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) if (j < n) f.df[o + j] = (uint8_t)df[j];
        }
        if (f.out_df) {
#pragma unroll
            for (int j = 0; j < 4; ++j) if (j < n) f.out_df[o + j] = (uint8_t)df[j];
        }
    };

    const int qx = t & (kTileQ - 1);
    const int lane = t & 63;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int ty = (t >> 4) + 16 * half;
        const int x0 = tx0 + 4 * qx, y = ty0 + ty;
        bool needs = false;
        if (x0 < W && y < H) {
            // exact shortcut: all in-window depths (columns x0-R .. x0+3+R,
            // rows inside the image) equal -> the normalised weighted sum is
            // that depth.  With blocks of 8 px or more the window's pixels
            // inside the image lie in at most 2 x 2 blocks: when those are
            // non-edge blocks of one region depth the window is uniform
            // (four table reads); else the depths are compared pixel by pixel
            // (a window over non-edge blocks of different depths holds pixels
            // of each -- every block under it holds a window pixel -- so it
            // is not uniform and goes to the filter without the pixel test:
            // the block-row steps of the background ramp are most of these)
            uint32_t c = 0, bad = 1, sure = 0;
            if (!K2 && !f.depth_in && ks >= 3) {
                const int bxa = max(x0 - R, 0) >> ks, bxb = min(x0 + 3 + R, W - 1) >> ks;
                const int bya = max(y - R, 0) >> ks, byb = min(y + R, H - 1) >> ks;
                const uint2 e00 = btab[(bya - by_lo) * bw + (bxa - bx_lo)], e01 = btab[(bya - by_lo) * bw + (bxb - bx_lo)];
                const uint2 e10 = btab[(byb - by_lo) * bw + (bxa - bx_lo)], e11 = btab[(byb - by_lo) * bw + (bxb - bx_lo)];
                c = e00.y;
                const uint32_t edge = (e00.x | e01.x | e10.x | e11.x) >> 24;
                const uint32_t differ = (e01.y ^ c) | (e10.y ^ c) | (e11.y ^ c);
                bad = edge | differ;
                sure = !edge && differ;
            }
            if (bad && !sure) {
                c = tD[(ty + R) * kRowWords + 2 * qx + 2] & 0xFFFFu;
                bad = 0;
                const uint32_t splat = c | (c << 16);
#pragma unroll
                for (int i = 0; i < S; ++i) {
                    const int yy = y + i - R;
                    if (yy < 0 || yy >= H) continue;
                    const int base = (ty + i) * kRowWords + 2 * qx;
#pragma unroll
                    for (int k = (4 - R) >> 1; k <= (7 + R) >> 1; ++k) {
                        const uint32_t mask = ((2 * k >= 4 - R) ? 0xFFFFu : 0u) | ((2 * k + 1 <= 7 + R) ? 0xFFFF0000u : 0u);
                        bad |= (tD[base + k] ^ splat) & mask;
                    }
                }
            }
            if (!bad) {
                const uint32_t df[4] = {c, c, c, c};
                store_df(x0, y, df);
            } else {
                needs = true;
            }
        }
        // compact the quads that need the full filter
        const unsigned long long m = __ballot(needs);
        if (m) {
            int base = 0;
            if (lane == 0) base = atomicAdd(&nwork, __popcll(m));
            base = __shfl(base, 0);
            if (needs) work[base + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)(t + 256 * half);
        }
    }
    __syncthreads();
    // the full filter: two lanes per listed quad, two pixels each (half the
    // serial length of one lane per quad); the even lane of a pair takes its
    // partner's two results by a lane shuffle and stores all four
    constexpr int PW = CbfPairWin<R>::kWords;
    const int nw2 = 2 * nwork;
    for (int i0 = 0; i0 < nw2; i0 += 256) {
        const int i = i0 + t;
        const bool on = i < nw2;
        const int q = on ? work[i >> 1] : 0;
        const int hf = i & 1;
        const int qx_ = q & (kTileQ - 1), ty_ = (q & 255) / kTileQ + 16 * (q >> 8);
        const int x0_ = tx0 + 4 * qx_, y_ = ty0 + ty_;
        uint32_t df2[2] = {0u, 0u};
        if (on) {
            // the pair's first pixel is LDS column 4 qx + 4 + 2 hf
            const int wb = 2 * qx_ + 2 + hf - CbfPairWin<R>::kW0;
            uint32_t yw[S][PW], dw[S][PW], rows_ok = 0;
#pragma unroll
            for (int r = 0; r < S; ++r) {
                const int yy = y_ + r - R;
                if (yy >= 0 && yy < H) rows_ok |= 1u << r;
                const int base = (ty_ + r) * kRowWords + wb;
#pragma unroll
                for (int k = 0; k < PW; ++k) { yw[r][k] = tY[base + k]; dw[r][k] = tD[base + k]; }
            }
            const int xp = x0_ + 2 * hf;
            if (xp - R >= 0 && xp + 1 + R < W) cbf_pair<R, false>(yw, dw, rows_ok, xp, W, wtab, df2);
            else cbf_pair<R, true>(yw, dw, rows_ok, xp, W, wtab, df2);
        }
        const uint32_t other = (uint32_t)__shfl_xor((int)(df2[0] | (df2[1] << 8)), 1);
        if (on && !hf) {
            const uint32_t df[4] = {df2[0], df2[1], other & 255u, other >> 8};
            store_df(x0_, y_, df);
        }
    }
}

// ---------------------------------------------------------------------------
// k_warp: one image row per workgroup.  Lane t owns the quads t, t + NT,
// t + 2 NT, ... (Q of them), so the lanes of a wave always touch consecutive
// quads: coalesced global traffic.  Quad iteration qi of wave w covers the
// 256-pixel chunk c = qi * NW + w, and chunks follow each other along the
// row, which is what the hole search walks.  The z-buffer index of pixel x is
// swizzled to x + x / 32 so that the four pixels of the lanes' quads spread
// over all LDS banks.
__device__ __forceinline__ int kidx(int x) { return x + (x >> 5); }

// 1 if k != 0, else 0, as one v_min_u32 (the optimiser would turn min(k, 1)
// back into a compare and a select through VCC).
__device__ __forceinline__ uint32_t nonzero_bit(uint32_t k) {
    uint32_t r;
    asm("v_min_u32 %0, %1, 1" : "=v"(r) : "v"(k));
    return r;
}

// kidx(x) held as one value, so that the word address is formed from it in
// one shift-add instead of the two shifted terms the optimiser distributes
// it into.
__device__ __forceinline__ int kidx_held(int x) {
    int k = kidx(x);
    asm("" : "+v"(k));
    return k;
}

// Per-byte mean of two packed colours, rounded half up, with no carries
// between bytes: (a | b) - ((a ^ b) >> 1) per byte.
__device__ __forceinline__ uint32_t avg_bytes(uint32_t a, uint32_t b) {
    return (a | b) - (((a ^ b) >> 1) & 0x7F7F7F7Fu);
}

// Two packed R | G << 8 | B << 16 pixels to 6 bytes at an even address.
__device__ __forceinline__ void store_px2_u16(uint8_t* p, uint32_t c0, uint32_t c1) {
    uint16_t* q = reinterpret_cast<uint16_t*>(p);
    q[0] = (uint16_t)c0;
    q[1] = (uint16_t)(((c0 >> 16) & 0xFFu) | ((c1 & 0xFFu) << 8));
    q[2] = (uint16_t)(c1 >> 8);
}

__device__ __forceinline__ void store_px_bytes(uint8_t* p, uint32_t c) {
    p[0] = (uint8_t)c;
    p[1] = (uint8_t)(c >> 8);
    p[2] = (uint8_t)(c >> 16);
}

// The outputs of four pixels x0..x0+3 of row y from their left / right view
// colours (R | G << 8 | B << 16): left and right views, the anaglyph (red
// from the left view, green and blue from the right), and the half
// side-by-side frame when requested (half column p = mean of view columns 2p,
// 2p + 1 rounded up per byte; left view in the first floor(W/2) columns,
// right view after them).  ALIGNED: W % 4 == 0 and 4-byte aligned buffers,
// four pixels = three dwords.
template <bool ALIGNED>
__device__ __forceinline__ void store_quad_views(const FrameDesc& f, int y, int x0, const uint32_t* cl,
                                                 const uint32_t* cr) {
    const int W = f.w;
    const int n = min(4, W - x0);
    const size_t off = ((size_t)y * W + x0) * 3;
    // unaligned rows: byte stores of the quad's pixels inside the row
    auto store4 = [&](uint8_t* out, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
        if (!out) return;
        const uint32_t c[4] = {c0, c1, c2, c3};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (j < n) {
                out[off + 3 * j] = (uint8_t)c[j];
                out[off + 3 * j + 1] = (uint8_t)(c[j] >> 8);
                out[off + 3 * j + 2] = (uint8_t)(c[j] >> 16);
            }
        }
    };
    if (ALIGNED) {
        // both views packed once; in the three dwords of a quad the red bytes
        // sit at fixed places, so the anaglyph is one bit-field insert per
        // dword
        const uint3 lp = make_uint3(perm(cl[1], cl[0], 0x04020100u), perm(cl[2], cl[1], 0x05040201u),
                                    perm(cl[3], cl[2], 0x06050402u));
        const uint3 rp = make_uint3(perm(cr[1], cr[0], 0x04020100u), perm(cr[2], cr[1], 0x05040201u),
                                    perm(cr[3], cr[2], 0x06050402u));
        if (f.out_l) *reinterpret_cast<uint3*>(f.out_l + off) = lp;
        if (f.out_r) *reinterpret_cast<uint3*>(f.out_r + off) = rp;
        if (f.out_a) {
            constexpr uint32_t m0 = 0xFF0000FFu, m1 = 0x00FF0000u, m2 = 0x0000FF00u;
            *reinterpret_cast<uint3*>(f.out_a + off) =
                make_uint3((lp.x & m0) | (rp.x & ~m0), (lp.y & m1) | (rp.y & ~m1), (lp.z & m2) | (rp.z & ~m2));
        }
    } else {
        store4(f.out_l, cl[0], cl[1], cl[2], cl[3]);
        store4(f.out_r, cr[0], cr[1], cr[2], cr[3]);
        store4(f.out_a, (cl[0] & 0xFFu) | (cr[0] & 0xFFFF00u), (cl[1] & 0xFFu) | (cr[1] & 0xFFFF00u),
               (cl[2] & 0xFFu) | (cr[2] & 0xFFFF00u), (cl[3] & 0xFFu) | (cr[3] & 0xFFFF00u));
    }
    if (f.out_h) {
        const int hw = W >> 1;
        const uint32_t l0 = avg_bytes(cl[0], cl[1]), l1 = avg_bytes(cl[2], cl[3]);
        const uint32_t r0 = avg_bytes(cr[0], cr[1]), r1 = avg_bytes(cr[2], cr[3]);
        const int p0 = x0 >> 1;
        uint8_t* row = f.out_h + (size_t)y * W * 3;
        if (ALIGNED) {
            // W % 4 == 0: both pairs exist, and both halves start at even
            // byte offsets
            store_px2_u16(row + (size_t)p0 * 3, l0, l1);
            store_px2_u16(row + (size_t)(hw + p0) * 3, r0, r1);
        } else {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int xa = x0 + 2 * k;
                if (xa >= W) break;
                const int pc = p0 + k;
                const bool pair = xa + 1 < W;
                const uint32_t lm = pair ? (k ? l1 : l0) : cl[2 * k];
                const uint32_t rm = pair ? (k ? r1 : r0) : cr[2 * k];
                if (pc < hw) store_px_bytes(row + (size_t)pc * 3, lm);
                store_px_bytes(row + (size_t)(hw + pc) * 3, rm);
            }
        }
    }
}

// LDS of the warp of one row: both z-buffers (kidx-padded), the shift
// table, the zero-key tag, the row's filtered depth, and per chunk (Q x 64
// lanes' quads) the keys at its valid extremes.
__host__ __device__ constexpr size_t warp_lds_bytes(int w, int threads, int q) {
    return (size_t)(2 * (((w + 3) & ~3) + ((w + 3) & ~3) / 32 + 1) * 4 + 256 * 4 + ((w + 3) & ~3) +
                    8 * q * (threads / 64) * 4 + 4);
}

// A lane's share of one image row: the frame bytes of its Q quads (three
// raw dwords per quad when aligned, else four decoded R | G << 8 | B << 16
// colours) and their filtered depths.
template <bool ALIGNED, int Q>
struct WarpRowIn {
    static constexpr int kPerQuad = ALIGNED ? 3 : 4;
    uint32_t c[kPerQuad * Q];
    uint32_t dq[Q];
};

template <bool ALIGNED, int Q>
__device__ __forceinline__ void warp_load(const FrameDesc& f, int y, int t, int NT, WarpRowIn<ALIGNED, Q>& in) {
    constexpr int P = WarpRowIn<ALIGNED, Q>::kPerQuad;
    const int W = f.w;
    const uint8_t* drow = f.df + (size_t)y * W;
    // the lane's first quad of the row; its next quads a uniform 12 NT bytes
    // apart
    const uint8_t* q0 = f.frame + ((size_t)y * W + 4 * t) * 3;
#pragma unroll
    for (int qi = 0; qi < Q; ++qi) {
        const int x0 = 4 * (qi * NT + t);
#pragma unroll
        for (int j = 0; j < P; ++j) in.c[P * qi + j] = 0;
        in.dq[qi] = 0;
        if (x0 >= W) continue;
        if (ALIGNED) {
            const uint3 v = *reinterpret_cast<const uint3*>(q0 + (size_t)qi * 12 * NT);
            in.c[P * qi] = v.x;
            in.c[P * qi + 1] = v.y;
            in.c[P * qi + 2] = v.z;
            in.dq[qi] = *reinterpret_cast<const uint32_t*>(drow + x0);
        } else {
            const int n = min(4, W - x0);
            const uint8_t* p = f.frame + ((size_t)y * W + x0) * 3;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                in.c[P * qi + j] = j < n ? (p[3 * j] | ((uint32_t)p[3 * j + 1] << 8) | ((uint32_t)p[3 * j + 2] << 16)) : 0u;
                if (j < n) in.dq[qi] |= (uint32_t)drow[x0 + j] << (8 * j);
            }
        }
    }
}

// The warp's standing LDS state for rows of width W: the shift table, and
// both z-buffers zero.  Each row's validity pass zeroes the words of x < W;
// the padding words past the row, where out-of-row targets land, are never
// read at this width, so the state holds from row to row of one frame (rows
// of another width need a fresh preparation).  A barrier must follow before
// the first row.
__device__ __forceinline__ void warp_prepare(const FrameDesc& f, int W, int t, int NT, uint32_t* lds) {
    const int KW = kidx((W + 3) & ~3) + 1;
    uint32_t* lut = lds + 2 * KW;
    for (int d = t; d < 256; d += NT) lut[d] = shift_entry(d, f.B, f.T);
    for (int i = t; i < 2 * KW; i += NT) lds[i] = 0;
    if (t == 0) lut[256] = 0;  // the zero-key tag
}

// Key of the last (LAST) or first valid pixel of a quad: mask m (bit j =
// pixel j valid) over keys k[0..3]; 0 when none.
template <bool LAST>
__device__ __forceinline__ uint32_t quad_extreme_key(uint32_t m, const uint32_t* k) {
    uint32_t r = 0;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
        const int j = LAST ? jj : 3 - jj;
        if ((m >> j) & 1u) r = k[j];
    }
    return r;
}

// The key of the last (LAST) or first valid pixel of a wave's chunk, read
// back from the view's z-buffer: any = ballot of the lanes whose quad holds a
// valid pixel, m = the lane's quad mask, c0 = the chunk's first pixel; 0 when
// the chunk has none.  Uniform: one lane's mask, one broadcast LDS read.
template <bool LAST>
__device__ __forceinline__ uint32_t chunk_extreme_key(unsigned long long any, uint32_t m, const uint32_t* key,
                                                      int c0) {
    if (!any) return 0u;
    const int src = LAST ? 63 - __clzll(any) : __ffsll((long long)any) - 1;
    const uint32_t ms = __builtin_amdgcn_readlane(m, src);
    const int j = LAST ? 31 - __clz(ms) : __ffs(ms) - 1;
    return key[kidx(c0 + 4 * src + j)];
}

// Hole fill of one view's quad: pixel j with valid bit clear takes the
// nearer valid pixel on either side of the row, the smaller depth winning
// and ties going left (LEFT_TIES, the left view) or right; with a valid
// pixel on one side only that one; with none, the source pixel (need bit j).
// k: the quad's keys; ex / ef: key of the nearest valid pixel before / after
// the quad, hx / hf: whether it exists.  Returns the four colours.
template <bool LEFT_TIES>
__device__ __forceinline__ void fill_quad(uint32_t m, uint32_t own, const uint32_t* k, uint32_t ex, bool hx,
                                          uint32_t ef, bool hf, uint32_t* c, uint32_t& need) {
    uint32_t lk[4], rk[4], lh = 0, rh = 0;
    uint32_t run = ex;
    bool has = hx;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        lk[j] = run;
        if (has) lh |= 1u << j;
        if ((m >> j) & 1u) { run = k[j]; has = true; }
    }
    run = ef;
    has = hf;
#pragma unroll
    for (int j = 3; j >= 0; --j) {
        rk[j] = run;
        if (has) rh |= 1u << j;
        if ((m >> j) & 1u) { run = k[j]; has = true; }
    }
    // branch-free per pixel: an invalid pixel's key is 0, which is also its
    // colour when neither side has a valid pixel
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const bool valid = (m >> j) & 1u;
        const bool a = (lh >> j) & 1u, b = (rh >> j) & 1u;
        const uint32_t ka = lk[j], kb = rk[j];
        const bool nearer_b = LEFT_TIES ? (kb >> 24) < (ka >> 24) : (kb >> 24) <= (ka >> 24);
        const uint32_t fill = b && (!a || nearer_b) ? kb : (a ? ka : 0u);
        const uint32_t v = valid ? k[j] : fill;
        if (!valid && !a && !b && ((own >> j) & 1u)) need |= 1u << j;
        c[j] = v & 0xFFFFFFu;
    }
}

// One view's colours of a lane's quad after the hole fill (fill_quad), for
// the views whose wave has a hole; the nearest valid keys outside the quad
// come from the wave's lanes (shuffles, run on all lanes) or from the other
// chunks' published extremes (entry words pw (last) and pw + 1 (first),
// flag bit pbit).
template <bool LEFT_TIES>
__device__ __forceinline__ void fill_view(uint32_t qv, uint32_t oq, const uint32_t* k, unsigned long long any,
                                          unsigned long long below, unsigned long long above, int lane,
                                          const uint32_t* pub, int ch, int NC, int pw, uint32_t pbit, uint32_t* c,
                                          uint32_t& need) {
    if (!__ballot((oq & ~qv) != 0)) {
#pragma unroll
        for (int j = 0; j < 4; ++j) c[j] = k[j] & 0xFFFFFFu;
        return;
    }
    const unsigned long long lb = any & below, la = any & above;
    uint32_t ex = (uint32_t)__shfl((int)quad_extreme_key<true>(qv, k), lb ? 63 - __clzll(lb) : lane);
    uint32_t ef = (uint32_t)__shfl((int)quad_extreme_key<false>(qv, k), la ? __ffsll(la) - 1 : lane);
    bool hx = lb != 0, hf = la != 0;
    if (oq & ~qv) {
        for (int o = ch - 1; o >= 0 && !hx; --o)
            if (pub[8 * o + 4] & pbit) {
                ex = pub[8 * o + pw];
                hx = true;
            }
        for (int o = ch + 1; o < NC && !hf; ++o)
            if (pub[8 * o + 4] & pbit) {
                ef = pub[8 * o + pw + 1];
                hf = true;
            }
    }
    fill_quad<LEFT_TIES>(qv, oq, k, ex, hx, ef, hf, c, need);
}

// Image row y on NT lanes t = 0..NT-1 (whole waves) from the lane's loaded
// share `in`; when next_y >= 0 the share of row next_y is loaded into `next`
// while this row is resolved.  lds: warp_lds_bytes(w, NT, Q) bytes in the
// state warp_prepare leaves, which the row restores.  Two barriers; inactive
// lane groups do no memory work but pass them too.
template <bool ALIGNED, int Q>
__device__ __forceinline__ void warp_row_body(const FrameDesc& f, int y, int t, int NT, uint32_t* lds, bool active,
                                              const WarpRowIn<ALIGNED, Q>& in, int next_y,
                                              WarpRowIn<ALIGNED, Q>& next) {
    const int W = active ? f.w : 0;
    // wave: the same for all lanes of a wave (whole waves), held uniform
    const int lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6), NW = NT >> 6;
    const int NC = Q * NW;  // chunks per row
    const int W4 = (W + 3) & ~3;
    const int KW = kidx(W4) + 1;
    uint32_t* keyL = lds;
    uint32_t* keyR = keyL + KW;
    const uint32_t* lut = keyR + KW;                                  // 256 entries
    uint32_t* ztag = keyR + KW + 256;                                 // y + 1 if a source of row y has key 0
    uint8_t* drow_l = reinterpret_cast<uint8_t*>(ztag + 1);           // the row's filtered depth, W4 bytes
    uint32_t* pub = reinterpret_cast<uint32_t*>(drow_l + W4);         // per chunk: 8 words

    // ---- forward warp of the row's pixels into both views; the key carries
    // the depth above the colour, so the atomic max keeps the nearer source
    // and its colour
    // a target outside the row lands on a padding word (x in [W, W4]: the
    // word of x = W4 is a spare one past the row), which nothing reads, so
    // the atomics need no branch
    bool zero_key = false;
#pragma unroll
    for (int qi = 0; qi < Q; ++qi) {
        const int x0 = 4 * (qi * NT + t);
        if (x0 >= W) continue;
        const int n = ALIGNED ? 4 : min(4, W - x0);
        uint32_t c[4];
        if (ALIGNED) {
            quad_colours(make_uint3(in.c[3 * qi], in.c[3 * qi + 1], in.c[3 * qi + 2]), c);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) c[j] = in.c[4 * qi + j];
        }
        const uint32_t dq = in.dq[qi];
        *reinterpret_cast<uint32_t*>(drow_l + x0) = dq;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!ALIGNED && j >= n) continue;
            const int x = x0 + j;
            const uint32_t d = (dq >> (8 * j)) & 255u;
            const uint32_t lv = lut[d];
            const int xl = (int)min((unsigned)(x + (int)(int16_t)(lv & 0xFFFFu)), (unsigned)W4);
            const int xr = (int)min((unsigned)(x + (int)(int16_t)(lv >> 16)), (unsigned)W4);
            const uint32_t key = (d << 24) | c[j];
            zero_key |= key == 0;
            atomicMax(&keyL[kidx_held(xl)], key);
            atomicMax(&keyR[kidx_held(xr)], key);
        }
    }
    if (__ballot(zero_key) && (t & 63) == 0) *ztag = (uint32_t)y + 1u;
    __syncthreads();

    // the next row's share is loaded while this row is resolved
    if (next_y >= 0) warp_load<ALIGNED, Q>(f, next_y, t, NT, next);

    // ---- validity, and the z-buffers back to zero: a landed source has a
    // non-zero key, except a black source of depth 0, whose key is 0; such a
    // source is the only one that can land on a zero key, so in a row that
    // has one (the tag) zero keys check the depth at their depth-0 source
    // position directly
    uint32_t kl[4 * Q], kr[4 * Q];
    uint32_t vL = 0, vR = 0, own = 0;  // bit 4 qi + j
#pragma unroll
    for (int qi = 0; qi < Q; ++qi) {
        const int x0 = 4 * (qi * NT + t);
        // aligned rows hold whole quads only
        const bool quad_in = x0 < W;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int x = x0 + j;
            const int i = 4 * qi + j;
            kl[i] = 0;
            kr[i] = 0;
            if (ALIGNED ? quad_in : x < W) {
                kl[i] = keyL[kidx(x)];
                kr[i] = keyR[kidx(x)];
                own |= 1u << i;
            }
        }
    }
    // the valid bits once every read is out
#pragma unroll
    for (int i = 0; i < 4 * Q; ++i) {
        vL |= nonzero_bit(kl[i]) << i;
        vR |= nonzero_bit(kr[i]) << i;
    }
    // the lane's z-buffer words back to zero (after the chunk's extreme keys
    // are read back below: the words of a chunk are this wave's alone, and
    // its LDS accesses complete in order)
    auto clear_own = [&]() {
#pragma unroll
        for (int qi = 0; qi < Q; ++qi) {
            const int x0 = 4 * (qi * NT + t);
            const bool quad_in = x0 < W;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (ALIGNED ? quad_in : x0 + j < W) {
                    keyL[kidx(x0 + j)] = 0;
                    keyR[kidx(x0 + j)] = 0;
                }
            }
        }
    };
    if (*ztag == (uint32_t)y + 1u && __ballot((own & ~(vL & vR)) != 0)) {
        const uint32_t lv0 = lut[0];
        const int o0[2] = {(int)(int16_t)(lv0 & 0xFFFFu), (int)(int16_t)(lv0 >> 16)};
        const uint32_t* d32 = reinterpret_cast<const uint32_t*>(drow_l);
        const int nd = W4 >> 2;
#pragma unroll
        for (int qi = 0; qi < Q; ++qi) {
            const int x0 = 4 * (qi * NT + t);
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                uint32_t& vm = v ? vR : vL;
                const uint32_t z = (own & ~vm) >> (4 * qi) & 15u;
                if (!z) continue;
                // the four sources x0 + j - o0 are consecutive bytes
                const int b = x0 - o0[v];
                const int i0 = b >> 2;
                const uint32_t w0 = d32[min(max(i0, 0), nd - 1)], w1 = d32[min(max(i0 + 1, 0), nd - 1)];
                const uint32_t bytes = alignbyte(w1, w0, (uint32_t)(b & 3));
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (((z >> j) & 1u) && (unsigned)(b + j) < (unsigned)W && !((bytes >> (8 * j)) & 255u))
                        vm |= 1u << (4 * qi + j);
            }
        }
    }
    if (f.ipc) {
        // block-iterative inpainting follows: leave the warped colours and the
        // holes, no row fill
        const size_t plane = (size_t)f.w * f.h;
#pragma unroll
        for (int qi = 0; qi < Q; ++qi) {
            const int x0 = 4 * (qi * NT + t);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = 4 * qi + j;
                if (!((own >> i) & 1u)) continue;
                const size_t o = (size_t)y * W + x0 + j;
                f.ipc[o] = kl[i] & 0xFFFFFFu;
                f.ipt[o] = ((vL >> i) & 1u) ? 0 : 0xFFFF;
                f.ipc[plane + o] = kr[i] & 0xFFFFFFu;
                f.ipt[plane + o] = ((vR >> i) & 1u) ? 0 : 0xFFFF;
            }
        }
        clear_own();
        __syncthreads();  // the z-buffers and the row depth are free again
        return;
    }
    // per chunk: ballot of the quads holding a valid pixel; the keys at the
    // chunk's extremes go to LDS for the other chunks
    unsigned long long anyL[Q], anyR[Q];
#pragma unroll
    for (int qi = 0; qi < Q; ++qi) {
        const uint32_t ql = (vL >> (4 * qi)) & 15u, qr = (vR >> (4 * qi)) & 15u;
        anyL[qi] = __ballot(ql != 0);
        anyR[qi] = __ballot(qr != 0);
        const int c0 = 4 * (qi * NT + 64 * wave);  // the chunk's first pixel
        const uint32_t a = chunk_extreme_key<true>(anyL[qi], ql, keyL, c0);
        const uint32_t b = chunk_extreme_key<false>(anyL[qi], ql, keyL, c0);
        const uint32_t c = chunk_extreme_key<true>(anyR[qi], qr, keyR, c0);
        const uint32_t d = chunk_extreme_key<false>(anyR[qi], qr, keyR, c0);
        if (lane == 0) {
            uint32_t* p = pub + 8 * (qi * NW + wave);
            p[0] = a;
            p[1] = b;
            p[2] = c;
            p[3] = d;
            p[4] = (anyL[qi] ? 1u : 0u) | (anyR[qi] ? 2u : 0u);
        }
    }
    clear_own();
    __syncthreads();

    // ---- hole filling from the nearest valid keys: inside the quad, in the
    // chunk through the ballots (shuffles run on all lanes of the wave), else
    // in the other chunks; then the anaglyph and the stores
    const unsigned long long below = (1ull << lane) - 1ull;
    const unsigned long long above = ~((2ull << lane) - 1ull);
#pragma unroll
    for (int qi = 0; qi < Q; ++qi) {
        const int x0 = 4 * (qi * NT + t);
        const uint32_t ql = (vL >> (4 * qi)) & 15u, qr = (vR >> (4 * qi)) & 15u;
        const uint32_t oq = (own >> (4 * qi)) & 15u;
        uint32_t cl[4], cr[4], needL = 0, needR = 0;
        const int ch = qi * NW + wave;
        fill_view<true>(ql, oq, &kl[4 * qi], anyL[qi], below, above, lane, pub, ch, NC, 0, 1u, cl, needL);
        fill_view<false>(qr, oq, &kr[4 * qi], anyR[qi], below, above, lane, pub, ch, NC, 2, 2u, cr, needR);
        if (needL | needR) {
            // a view row without any valid pixel keeps the source pixels
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (!(((needL | needR) >> j) & 1u)) continue;
                const uint8_t* p = f.frame + ((size_t)y * W + x0 + j) * 3;
                const uint32_t src = p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16);
                if ((needL >> j) & 1u) cl[j] = src;
                if ((needR >> j) & 1u) cr[j] = src;
            }
        }
        if (x0 < W) store_quad_views<ALIGNED>(f, y, x0, cl, cr);
    }
}

// LDS bytes of the gather row: the shift table and the row's source colours.
__host__ __device__ constexpr size_t gather_lds_bytes(int w) {
    return (size_t)(256 + ((w + 3) & ~3) + (((w + 3) & ~3) >> 5) + 1) * 4;  // 256 + kidx(W4) + 1 words
}

// Image row y by the Fig. 3 gather (Section 4): each destination pixel reads
// the filtered depth at its own position and copies the source pixel its
// view's offset points back to (its own source pixel when that lies outside
// the row); no occlusion test, no holes.  The source row's colours are staged
// in LDS (padded every 32 words) so the gathers are LDS reads.
template <bool ALIGNED>
__device__ __forceinline__ void gather_row(const FrameDesc& f, int y, int t, int NT, uint32_t* lds) {
    const int W = f.w;
    uint32_t* lut = lds;           // 256 entries
    uint32_t* rowc = lut + 256;    // source colours, kidx-indexed
    for (int d = t; d < 256; d += NT) lut[d] = shift_entry(d, f.B, f.T);
    const uint8_t* src = f.frame + (size_t)y * W * 3;
    for (int x0 = 4 * t; x0 < W; x0 += 4 * NT) {
        uint32_t c[4];
        if (ALIGNED) {
            quad_colours(*reinterpret_cast<const uint3*>(src + (size_t)x0 * 3), c);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint8_t* p = src + (size_t)(x0 + j) * 3;
                c[j] = x0 + j < W ? (p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16)) : 0u;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) rowc[kidx(x0 + j)] = c[j];
    }
    __syncthreads();
    const uint8_t* drow = f.df + (size_t)y * W;
    for (int x0 = 4 * t; x0 < W; x0 += 4 * NT) {
        uint32_t dq = 0;
        if (ALIGNED) {
            dq = *reinterpret_cast<const uint32_t*>(drow + x0);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (x0 + j < W) dq |= (uint32_t)drow[x0 + j] << (8 * j);
        }
        uint32_t cl[4], cr[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int x = x0 + j;
            const uint32_t lv = lut[(dq >> (8 * j)) & 255u];
            int xl = x - (int)(int16_t)(lv & 0xFFFFu);
            int xr = x - (int)(int16_t)(lv >> 16);
            if ((unsigned)xl >= (unsigned)W) xl = x;
            if ((unsigned)xr >= (unsigned)W) xr = x;
            cl[j] = x < W ? rowc[kidx(xl)] : 0u;
            cr[j] = x < W ? rowc[kidx(xr)] : 0u;
        }
        store_quad_views<ALIGNED>(f, y, x0, cl, cr);
    }
}

// One Jacobi sweep of the block-iterative inpainting over pixel p = (x, y) of
// view v: a hole (tag 0xFFFF) with at least two undamaged 8-neighbours --
// tag below `sweep`, so pixels filled in this same sweep do not count --
// takes their per-channel mean rounded half up and the tag `sweep`.  Updates
// in place are safe: a pixel written in this sweep is never read as
// undamaged in it.  Returns 1 if p was filled.
__device__ __forceinline__ int inpaint_pixel(const FrameDesc& f, int v, int x, int y, int sweep) {
    const int W = f.w, H = f.h;
    const size_t plane = (size_t)W * H * v;
    const size_t o = plane + (size_t)y * W + x;
    if (f.ipt[o] != 0xFFFF) return 0;
    int cnt = 0;
    uint32_t s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            if (!dx && !dy) continue;
            const int xx = x + dx, yy = y + dy;
            if ((unsigned)xx >= (unsigned)W || (unsigned)yy >= (unsigned)H) continue;
            const size_t q = plane + (size_t)yy * W + xx;
            if ((int)f.ipt[q] >= sweep) continue;
            const uint32_t c = f.ipc[q];
            ++cnt;
            s0 += c & 255u;
            s1 += (c >> 8) & 255u;
            s2 += c >> 16;
        }
    }
    if (cnt < 2) return 0;
    const uint32_t h = (uint32_t)cnt >> 1;
    f.ipc[o] = ((s0 + h) / cnt) | (((s1 + h) / cnt) << 8) | (((s2 + h) / cnt) << 16);
    f.ipt[o] = (uint16_t)sweep;
    return 1;
}

// One image row (the single-row form used by the batch kernels), from and
// to any LDS contents.
template <bool ALIGNED, int Q>
__device__ __forceinline__ void warp_row(const FrameDesc& f, int y, int t, int NT, uint32_t* lds, bool active) {
    WarpRowIn<ALIGNED, Q> in, unused;
    if (active) {
        warp_load<ALIGNED, Q>(f, y, t, NT, in);
    } else {
#pragma unroll
        for (int i = 0; i < WarpRowIn<ALIGNED, Q>::kPerQuad * Q; ++i) in.c[i] = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) in.dq[i] = 0;
    }
    warp_prepare(f, active ? f.w : 0, t, NT, lds);
    __syncthreads();
    warp_row_body<ALIGNED, Q>(f, y, t, NT, lds, active, in, -1, unused);
}

// Rows y0, y0 + step, ... below y_end of the frame, the LDS state prepared
// once, each row's loads issued during the previous row (one or two quads per
// lane: a second row's share of four would not fit the registers).
template <bool ALIGNED, int Q>
__device__ __forceinline__ void warp_rows(const FrameDesc& f, int y0, int y_end, int step, int t, int NT,
                                          uint32_t* lds) {
    static_assert(Q < 4, "four quads per lane take one row at a time");
    if (y0 >= y_end) return;
    WarpRowIn<ALIGNED, Q> cur, nxt;
    warp_load<ALIGNED, Q>(f, y0, t, NT, cur);
    warp_prepare(f, f.w, t, NT, lds);
    __syncthreads();
    for (int y = y0; y < y_end; y += step) {
        const int ny = y + step < y_end ? y + step : -1;
        warp_row_body<ALIGNED, Q>(f, y, t, NT, lds, true, cur, ny, nxt);
        cur = nxt;
    }
}

}  // namespace pstereo
