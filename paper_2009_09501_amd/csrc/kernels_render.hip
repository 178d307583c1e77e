// gfx950 kernels of the stereo rendering: filtered depth, then both views.
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

__device__ __forceinline__ uint32_t byte_of(uint32_t w, int i) { return (w >> (8 * i)) & 255u; }

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

// Raw depth of the four pixels of a quad: the region depth of their block, or
// for an edge block that of the non-edge 3x3 neighbour block whose mean colour
// is nearest (L1), first strict minimum in raster order; with no candidate
// the ramp of the block row.  The nine neighbour loads are unconditional
// (clamped) so they are all in flight together.
__device__ __forceinline__ void quad_depth(const FrameDesc& f, int x0, int yy, const int (&r)[4],
                                           const int (&g)[4], const int (&b)[4], int (&D)[4]) {
    const int bx = x0 / f.K, by = yy / f.K;
    const uint2 own = f.binfo[by * f.gw + bx];
    if (!(own.x >> 24)) {
#pragma unroll
        for (int j = 0; j < 4; ++j) D[j] = (int)own.y;
        return;
    }
    uint2 c[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int cx = min(max(bx + k % 3 - 1, 0), f.gw - 1);
        const int cy = min(max(by + k / 3 - 1, 0), f.gh - 1);
        c[k] = f.binfo[cy * f.gw + cx];
    }
    int best[4] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX};
    const int fallback = ramp(by, f.gh);
#pragma unroll
    for (int j = 0; j < 4; ++j) D[j] = fallback;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int cx = bx + k % 3 - 1, cy = by + k / 3 - 1;
        if (cx < 0 || cx >= f.gw || cy < 0 || cy >= f.gh || (c[k].x >> 24)) continue;
        const int mr = c[k].x & 255, mg = (c[k].x >> 8) & 255, mb = (c[k].x >> 16) & 255;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int dd = iabs(r[j] - mr) + iabs(g[j] - mg) + iabs(b[j] - mb);
            if (dd < best[j]) { best[j] = dd; D[j] = (int)c[k].y; }
        }
    }
}

// Filtered depth of the four pixels x0..x0+3 of one row.  The window words
// hold bytes of columns x0-4 .. x0+7 for rows y-R .. y+R (rows outside the
// image are flagged off in rows_ok).  CLIP: some window column lies outside
// the image and is skipped.
template <int R, bool CLIP>
__device__ __forceinline__ void cbf_quad(const uint32_t (&yw)[2 * R + 1][3], const uint32_t (&dw)[2 * R + 1][3],
                                         uint32_t rows_ok, int x0, int W, const uint16_t* wtab, uint32_t (&df)[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int yp = (int)byte_of(yw[R][1], j);
        uint32_t acc = 0, wsum = 0;
#pragma unroll
        for (int dy = -R; dy <= R; ++dy) {
            if (!((rows_ok >> (dy + R)) & 1u)) continue;
#pragma unroll
            for (int dx = -R; dx <= R; ++dx) {
                if (CLIP) {
                    const int xx = x0 + j + dx;
                    if (xx < 0 || xx >= W) continue;
                }
                const int c = 4 + j + dx;
                const int yq = (int)byte_of(yw[dy + R][c >> 2], c & 3);
                const uint32_t dq = byte_of(dw[dy + R][c >> 2], c & 3);
                const uint32_t w = wtab[k_index(dx * dx + dy * dy) * 256 + iabs(yq - yp)];
                acc += w * dq;
                wsum += w;
            }
        }
        df[j] = div_small_quotient(acc + (wsum >> 1), wsum);
    }
}

// ---------------------------------------------------------------------------
// k_cbf: 64 x 16 pixel tiles, 256 lanes, lane = one quad of one tile row.
constexpr int kTileQ = 16;                   // quads per tile row
constexpr int kTileW = 4 * kTileQ;           // 64 px
constexpr int kTileH = 16;                   // rows
constexpr int kTileWords = kTileQ + 2;       // LDS dwords per tile row: 4 px halo each side

template <int R, bool ALIGNED>
__global__ void __launch_bounds__(256) k_cbf(FrameDesc f) {
    constexpr int S = 2 * R + 1;
    constexpr int TR = kTileH + 2 * R;       // tile rows incl. halo
    constexpr int NK = k_count(R);
    __shared__ uint32_t tY[TR * kTileWords];
    __shared__ uint32_t tD[TR * kTileWords];
    __shared__ uint16_t wtab[NK * 256];
    __shared__ uint16_t work[256];
    __shared__ int nwork;

    const int W = f.w, H = f.h;
    const int t = threadIdx.x;
    const int tx0 = blockIdx.x * kTileW, ty0 = blockIdx.y * kTileH;

    // product weights ws[k] * wr[d] per distinct squared distance k
    for (int i = t; i < NK * 256; i += 256) wtab[i] = (uint16_t)(spatial_w(k_value(i >> 8)) * range_w(i & 255));
    if (t == 0) nwork = 0;

    // luma + raw depth of the tile and its halo (columns tx0-4 .. tx0+67)
    for (int i = t; i < TR * kTileWords; i += 256) {
        const int tr = i / kTileWords, tq = i - tr * kTileWords;
        const int yy = ty0 - R + tr;
        const int x0 = tx0 - 4 + 4 * tq;
        uint32_t py = 0, pd = 0;
        if (yy >= 0 && yy < H && x0 >= 0 && x0 < W) {
            const int n = min(4, W - x0);
            int r[4], g[4], b[4], D[4];
            load_quad<ALIGNED>(f.frame + ((size_t)yy * W + x0) * 3, n, r, g, b);
            if (f.depth_in) {
                const uint8_t* dp = f.depth_in + (size_t)yy * W + x0;
#pragma unroll
                for (int j = 0; j < 4; ++j) D[j] = j < n ? dp[j] : 0;
            } else {
                quad_depth(f, x0, yy, r, g, b, D);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (j < n) {
                    py |= (uint32_t)luma(r[j], g[j], b[j]) << (8 * j);
                    pd |= (uint32_t)D[j] << (8 * j);
                }
            }
            if (f.out_d0 && tr >= R && tr < R + kTileH && tq >= 1 && tq <= kTileQ) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (j < n) f.out_d0[(size_t)yy * W + x0 + j] = (uint8_t)D[j];
            }
        }
        tY[i] = py;
        tD[i] = pd;
    }
    __syncthreads();

    const int qx = t & (kTileQ - 1), ty = t / kTileQ;
    const int x0 = tx0 + 4 * qx, y = ty0 + ty;
    const bool mine = x0 < W && y < H;

    auto window = [&](int qx_, int ty_, uint32_t (&yw)[S][3], uint32_t (&dw)[S][3], uint32_t& rows_ok) {
        const int y_ = ty0 + ty_;
        rows_ok = 0;
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const int yy = y_ + i - R;
            if (yy >= 0 && yy < H) rows_ok |= 1u << i;
            const int base = (ty_ + i) * kTileWords + qx_;
#pragma unroll
            for (int k = 0; k < 3; ++k) { yw[i][k] = tY[base + k]; dw[i][k] = tD[base + k]; }
        }
    };
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

    bool needs = false;
    if (mine) {
        uint32_t yw[S][3], dw[S][3], rows_ok;
        window(qx, ty, yw, dw, rows_ok);
        // exact shortcut: all depths of the window equal -> the normalised
        // weighted sum is that depth
        const uint32_t c = byte_of(dw[R][1], 0);
        const uint32_t splat = c * 0x01010101u;
        constexpr uint32_t himask = (R == 3) ? 0xFFFFFFu : (R == 2) ? 0xFFFFu : (R == 1) ? 0xFFu : 0u;
        constexpr int losh = (R == 0) ? 31 : 8 * (4 - R);
        bool uniform = true;
#pragma unroll
        for (int i = 0; i < S; ++i) {
            if (!((rows_ok >> i) & 1u)) continue;
            uniform = uniform && dw[i][1] == splat;
            if (R > 0)
                uniform = uniform && (dw[i][0] >> losh) == (splat >> losh) && (dw[i][2] & himask) == (splat & himask);
        }
        if (uniform) {
            const uint32_t df[4] = {c, c, c, c};
            store_df(x0, y, df);
        } else {
            needs = true;
        }
    }
    // compact the quads that need the full filter
    const unsigned long long m = __ballot(needs);
    if (m) {
        const int lane = t & 63;
        int base = 0;
        if (lane == 0) base = atomicAdd(&nwork, __popcll(m));
        base = __shfl(base, 0);
        if (needs) work[base + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)t;
    }
    __syncthreads();
    const int nw = nwork;
    for (int i = t; i < nw; i += 256) {
        const int q = work[i];
        const int qx_ = q & (kTileQ - 1), ty_ = q / kTileQ;
        const int x0_ = tx0 + 4 * qx_, y_ = ty0 + ty_;
        uint32_t yw[S][3], dw[S][3], rows_ok, df[4];
        window(qx_, ty_, yw, dw, rows_ok);
        if (x0_ - R >= 0 && x0_ + 3 + R < W) cbf_quad<R, false>(yw, dw, rows_ok, x0_, W, wtab, df);
        else cbf_quad<R, true>(yw, dw, rows_ok, x0_, W, wtab, df);
        store_df(x0_, y_, df);
    }
}

// ---------------------------------------------------------------------------
// k_warp: one image row per workgroup; lane t owns pixels [4Q t, 4Q t + 4Q).
template <bool ALIGNED, int Q>
__global__ void __launch_bounds__(1024) k_warp(FrameDesc f) {
    extern __shared__ uint32_t lds[];
    constexpr int SEG = 4 * Q;
    const int W = f.w;
    const int y = blockIdx.x;
    const int t = threadIdx.x, NT = blockDim.x;
    const int lane = t & 63, wave = t >> 6, NW = NT >> 6;
    const int W4 = (W + 3) & ~3;
    uint32_t* keyL = lds;
    uint32_t* keyR = keyL + W4;
    uint32_t* lut = keyR + W4;                       // 256 entries
    int* pub = reinterpret_cast<int*>(lut + 256);    // per wave: last L, first L, last R, first R

    for (int d = t; d < 256; d += NT) lut[d] = shift_entry(d, f.B, f.T);
    const int xs = t * SEG;
#pragma unroll
    for (int qi = 0; qi < Q; ++qi) {
        const int x0 = xs + 4 * qi;
        if (x0 < W) {
            *reinterpret_cast<uint4*>(keyL + x0) = make_uint4(0, 0, 0, 0);
            *reinterpret_cast<uint4*>(keyR + x0) = make_uint4(0, 0, 0, 0);
        }
    }
    __syncthreads();

    // ---- forward warp of the row's pixels into both views
    const uint8_t* drow = f.df + (size_t)y * W;
    uint32_t col[SEG];  // own source colours, R | G << 8 | B << 16
#pragma unroll
    for (int qi = 0; qi < Q; ++qi) {
        const int x0 = xs + 4 * qi;
        int r[4] = {0, 0, 0, 0}, g[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0};
        uint32_t dq = 0;
        int n = 0;
        if (x0 < W) {
            n = min(4, W - x0);
            load_quad<ALIGNED>(f.frame + ((size_t)y * W + x0) * 3, n, r, g, b);
            if (ALIGNED) {
                dq = *reinterpret_cast<const uint32_t*>(drow + x0);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) if (j < n) dq |= (uint32_t)drow[x0 + j] << (8 * j);
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            col[4 * qi + j] = (uint32_t)r[j] | ((uint32_t)g[j] << 8) | ((uint32_t)b[j] << 16);
            if (j >= n) continue;
            const int x = x0 + j;
            const uint32_t d = byte_of(dq, j);
            const uint32_t lv = lut[d];
            const int xl = x + (int)(int16_t)(lv & 0xFFFFu);
            const int xr = x + (int)(int16_t)(lv >> 16);
            const uint32_t key = (d << 24) | col[4 * qi + j];
            if ((unsigned)xl < (unsigned)W) atomicMax(&keyL[xl], key);
            if ((unsigned)xr < (unsigned)W) atomicMax(&keyR[xr], key);
        }
    }
    __syncthreads();

    // ---- validity: a landed source has a non-zero key, except a black source
    // of depth 0, whose key is 0; such a source is the only one that can land
    // on a zero key, so check it directly
    const uint32_t lv0 = lut[0];
    const int o0L = (int)(int16_t)(lv0 & 0xFFFFu), o0R = (int)(int16_t)(lv0 >> 16);
    uint32_t kl[SEG], kr[SEG];
    uint32_t vL = 0, vR = 0;  // valid bits of the own pixels
#pragma unroll
    for (int qi = 0; qi < Q; ++qi) {
        const int x0 = xs + 4 * qi;
        uint4 a = make_uint4(0, 0, 0, 0), b = make_uint4(0, 0, 0, 0);
        if (x0 < W) {
            a = *reinterpret_cast<const uint4*>(keyL + x0);
            b = *reinterpret_cast<const uint4*>(keyR + x0);
        }
        kl[4 * qi + 0] = a.x; kl[4 * qi + 1] = a.y; kl[4 * qi + 2] = a.z; kl[4 * qi + 3] = a.w;
        kr[4 * qi + 0] = b.x; kr[4 * qi + 1] = b.y; kr[4 * qi + 2] = b.z; kr[4 * qi + 3] = b.w;
    }
#pragma unroll
    for (int i = 0; i < SEG; ++i) {
        const int x = xs + i;
        if (x >= W) break;
        if (kl[i]) vL |= 1u << i;
        else {
            const int s0 = x - o0L;
            if ((unsigned)s0 < (unsigned)W && drow[s0] == 0) vL |= 1u << i;
        }
        if (kr[i]) vR |= 1u << i;
        else {
            const int s0 = x - o0R;
            if ((unsigned)s0 < (unsigned)W && drow[s0] == 0) vR |= 1u << i;
        }
    }
    const int lastL = vL ? xs + 31 - __clz(vL) : -1, firstL = vL ? xs + __ffs(vL) - 1 : W;
    const int lastR = vR ? xs + 31 - __clz(vR) : -1, firstR = vR ? xs + __ffs(vR) - 1 : W;
    const unsigned long long anyL = __ballot(vL != 0), anyR = __ballot(vR != 0);
    // per-wave extremes, published for the other waves (shuffles run on all lanes)
    const int wLastL = __shfl(lastL, anyL ? 63 - __clzll(anyL) : 0);
    const int wFirstL = __shfl(firstL, anyL ? __ffsll(anyL) - 1 : 0);
    const int wLastR = __shfl(lastR, anyR ? 63 - __clzll(anyR) : 0);
    const int wFirstR = __shfl(firstR, anyR ? __ffsll(anyR) - 1 : 0);
    if (lane == 0) {
        pub[4 * wave + 0] = anyL ? wLastL : -1;
        pub[4 * wave + 1] = anyL ? wFirstL : W;
        pub[4 * wave + 2] = anyR ? wLastR : -1;
        pub[4 * wave + 3] = anyR ? wFirstR : W;
    }
    // nearest valid pixel outside the own segment, inside the wave
    const unsigned long long below = (1ull << lane) - 1ull;
    const unsigned long long above = ~((2ull << lane) - 1ull);
    const unsigned long long mLb = anyL & below, mRb = anyR & below;
    const unsigned long long mLa = anyL & above, mRa = anyR & above;
    int exL = __shfl(lastL, mLb ? 63 - __clzll(mLb) : lane);
    int exR = __shfl(lastR, mRb ? 63 - __clzll(mRb) : lane);
    int efL = __shfl(firstL, mLa ? __ffsll(mLa) - 1 : lane);
    int efR = __shfl(firstR, mRa ? __ffsll(mRa) - 1 : lane);
    if (!mLb) exL = -1;
    if (!mRb) exR = -1;
    if (!mLa) efL = W;
    if (!mRa) efR = W;
    __syncthreads();
    // ... or in another wave
    for (int v = wave - 1; v >= 0 && (exL < 0 || exR < 0); --v) {
        if (exL < 0) exL = pub[4 * v + 0];
        if (exR < 0) exR = pub[4 * v + 2];
    }
    for (int v = wave + 1; v < NW && (efL >= W || efR >= W); ++v) {
        if (efL >= W) efL = pub[4 * v + 1];
        if (efR >= W) efR = pub[4 * v + 3];
    }

    // ---- inpainting: a hole copies the nearer valid pixel of the warped row
    // with the smaller depth (background); equal depths go left in the left
    // view, right in the right view; a row without valid pixels keeps the
    // source pixel
    uint32_t cl[SEG], cr[SEG];
#pragma unroll
    for (int i = 0; i < SEG; ++i) {
        cl[i] = kl[i] & 0xFFFFFFu;
        cr[i] = kr[i] & 0xFFFFFFu;
    }
    const uint32_t own = xs >= W ? 0u : (W - xs >= SEG ? ((1u << SEG) - 1u) : ((1u << (W - xs)) - 1u));
    if (own & ~(vL & vR)) {
#pragma unroll
        for (int i = 0; i < SEG; ++i) {
            const int x = xs + i;
            if (x >= W) break;
            const uint32_t lowmask = (1u << i) - 1u;
            const uint32_t highmask = ~((2u << i) - 1u);  // i < SEG <= 16
            if (!((vL >> i) & 1u)) {
                const uint32_t lo = vL & lowmask, hi = vL & highmask;
                const int a = lo ? xs + 31 - __clz(lo) : exL;
                const int b = hi ? xs + __ffs(hi) - 1 : efL;
                uint32_t k;
                if (a >= 0 && b < W) {
                    const uint32_t ka = keyL[a], kb = keyL[b];
                    k = (kb >> 24) < (ka >> 24) ? kb : ka;
                } else if (a >= 0) {
                    k = keyL[a];
                } else if (b < W) {
                    k = keyL[b];
                } else {
                    k = col[i];
                }
                cl[i] = k & 0xFFFFFFu;
            }
            if (!((vR >> i) & 1u)) {
                const uint32_t lo = vR & lowmask, hi = vR & highmask;
                const int a = lo ? xs + 31 - __clz(lo) : exR;
                const int b = hi ? xs + __ffs(hi) - 1 : efR;
                uint32_t k;
                if (a >= 0 && b < W) {
                    const uint32_t ka = keyR[a], kb = keyR[b];
                    k = (ka >> 24) < (kb >> 24) ? ka : kb;
                } else if (a >= 0) {
                    k = keyR[a];
                } else if (b < W) {
                    k = keyR[b];
                } else {
                    k = col[i];
                }
                cr[i] = k & 0xFFFFFFu;
            }
        }
    }

    // ---- anaglyph and stores
#pragma unroll
    for (int qi = 0; qi < Q; ++qi) {
        const int x0 = xs + 4 * qi;
        if (x0 >= W) break;
        const int n = min(4, W - x0);
        const size_t off = ((size_t)y * W + x0) * 3;
        int r[4], g[4], b[4];
        if (f.out_l) {
#pragma unroll
            for (int j = 0; j < 4; ++j) { r[j] = byte_of(cl[4 * qi + j], 0); g[j] = byte_of(cl[4 * qi + j], 1); b[j] = byte_of(cl[4 * qi + j], 2); }
            store_quad<ALIGNED>(f.out_l + off, n, r, g, b);
        }
        if (f.out_r) {
#pragma unroll
            for (int j = 0; j < 4; ++j) { r[j] = byte_of(cr[4 * qi + j], 0); g[j] = byte_of(cr[4 * qi + j], 1); b[j] = byte_of(cr[4 * qi + j], 2); }
            store_quad<ALIGNED>(f.out_r + off, n, r, g, b);
        }
        if (f.out_a) {
#pragma unroll
            for (int j = 0; j < 4; ++j) { r[j] = byte_of(cl[4 * qi + j], 0); g[j] = byte_of(cr[4 * qi + j], 1); b[j] = byte_of(cr[4 * qi + j], 2); }
            store_quad<ALIGNED>(f.out_a + off, n, r, g, b);
        }
    }
}

// ---------------------------------------------------------------------------
// host-side launch helpers

bool warp_shape(int w, WarpShape* out) {
    const int quads = (w + 3) / 4;
    int q = 1;
    while (q < 4 && (quads + q - 1) / q > 256) q *= 2;
    int threads = ((quads + q - 1) / q + 63) / 64 * 64;
    if (threads > 1024) return false;
    const size_t W4 = (size_t)((w + 3) & ~3);
    const size_t lds = 2 * W4 * 4 + 256 * 4 + 4 * (threads / 64) * 4;
    if (lds > kMaxLds) return false;
    out->threads = threads;
    out->quads = q;
    out->lds_bytes = lds;
    return true;
}

template <int R, bool A>
static hipError_t cbf_launch(const FrameDesc& f, hipStream_t s) {
    dim3 grid((f.w + kTileW - 1) / kTileW, (f.h + kTileH - 1) / kTileH);
    hipLaunchKernelGGL((k_cbf<R, A>), grid, dim3(256), 0, s, f);
    return hipGetLastError();
}

template <bool A>
static hipError_t cbf_r(const FrameDesc& f, hipStream_t s) {
    switch (f.r) {
        case 0: return cbf_launch<0, A>(f, s);
        case 1: return cbf_launch<1, A>(f, s);
        case 2: return cbf_launch<2, A>(f, s);
        case 3: return cbf_launch<3, A>(f, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_cbf(const FrameDesc& f, hipStream_t s) {
    return f.aligned ? cbf_r<true>(f, s) : cbf_r<false>(f, s);
}

template <bool A, int Q>
static hipError_t warp_launch(const FrameDesc& f, const WarpShape& ws, hipStream_t s) {
    hipLaunchKernelGGL((k_warp<A, Q>), dim3(f.h), dim3(ws.threads), ws.lds_bytes, s, f);
    return hipGetLastError();
}

template <bool A>
static hipError_t warp_q(const FrameDesc& f, const WarpShape& ws, hipStream_t s) {
    switch (ws.quads) {
        case 1: return warp_launch<A, 1>(f, ws, s);
        case 2: return warp_launch<A, 2>(f, ws, s);
        case 4: return warp_launch<A, 4>(f, ws, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_warp(const FrameDesc& f, const WarpShape& ws, hipStream_t s) {
    return f.aligned ? warp_q<true>(f, ws, s) : warp_q<false>(f, ws, s);
}

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
