/*
 * oracle.c -- plain, slow CPU oracle of the 2D -> 3D pseudo-stereo (DIBR)
 * pipeline of "3D Pseudo Stereo Visualization with GPGPU Support"
 * (Al-Oraiqat & Zori).
 *
 * TEST INFRASTRUCTURE.  This library exists to check the GPU library: only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg load it.  It
 * shares no source, header, table or helper with the GPU library.
 *
 * Every stage is a separate scalar loop nest, in the order of the paper's
 * conversion scheme (Section 3, Fig. 1; Section 4, the seven steps):
 *
 *   depth map (O1-O8)  ->  cross-bilateral filtered depth (O9)
 *   -> left / right frame reconstruction (O10-O11)
 *   -> left / right inpainting (O12)  ->  stereo formatting (O13).
 *
 * The paper fixes only the stage order, the depth -> shift rule with threshold
 * 150 and the anaglyph channel assignment (Section 4, Fig. 3 code).  The
 * depth-cue algorithm, the filter constants, the rounding and the hole rule
 * are not printed; each function below states the reading it implements.
 * All arithmetic is integer except the one-time construction of the
 * cross-bilateral weight tables from exp() in double precision.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_INVALID (-1)
#define ORC_E_NOMEM (-2)

#define ORC_MAX_BLOCKS 32768
#define ORC_MAX_RADIUS 3

/* ------------------------------------------------------------------ O1 */
/* Luma guide of the depth cues and of the cross-bilateral filter.  The paper
 * does not say how a colour becomes intensity; the reading is BT.601-style
 * weights in Q8 that sum to 256, rounded half up. */
static int orc_luma(int r, int g, int b) {
    return (77 * r + 150 * g + 29 * b + 128) >> 8;
}

void oracle_luma(const uint8_t *rgb, int64_t n_pixels, uint8_t *y_out) {
    for (int64_t i = 0; i < n_pixels; i++)
        y_out[i] = (uint8_t)orc_luma(rgb[3 * i], rgb[3 * i + 1], rgb[3 * i + 2]);
}

/* ------------------------------------------------------------------ O2 */
/* Block grid of the block-based depth generation (Section 3: block image
 * processing; Fig. 3 inpainting pseudocode: Frame_Blocks).  Auto rule: the
 * smallest K in {8,16,32,64} whose grid has at most 32768 blocks. */
int oracle_auto_block(int w, int h) {
    static const int cand[4] = {8, 16, 32, 64};
    for (int i = 0; i < 4; i++) {
        int64_t gw = (w + cand[i] - 1) / cand[i];
        int64_t gh = (h + cand[i] - 1) / cand[i];
        if (gw * gh <= ORC_MAX_BLOCKS) return cand[i];
    }
    return -1;
}

/* ------------------------------------------------------------------ O9 */
/* Cross-bilateral weights (Section 3: filtered depth map; Section 4: GPU
 * cross-bilateral filtering).  Constants are a reading: sigma_s = 1.5 px,
 * sigma_r = 12 luma levels, weights rounded half up to 0..255. */
static int orc_ws[2 * ORC_MAX_RADIUS * ORC_MAX_RADIUS + 1];
static int orc_wr[256];
static int orc_tables_ready = 0;

static void orc_build_tables(void) {
    if (orc_tables_ready) return;
    const double ss = 1.5, sr = 12.0;
    for (int k = 0; k <= 2 * ORC_MAX_RADIUS * ORC_MAX_RADIUS; k++)
        orc_ws[k] = (int)floor(255.0 * exp(-(double)k / (2.0 * ss * ss)) + 0.5);
    for (int d = 0; d < 256; d++)
        orc_wr[d] = (int)floor(255.0 * exp(-(double)(d * d) / (2.0 * sr * sr)) + 0.5);
    orc_tables_ready = 1;
}

void oracle_weight_tables(int32_t *ws_out, int32_t *wr_out) {
    orc_build_tables();
    for (int k = 0; k <= 2 * ORC_MAX_RADIUS * ORC_MAX_RADIUS; k++) ws_out[k] = orc_ws[k];
    for (int d = 0; d < 256; d++) wr_out[d] = orc_wr[d];
}

/* ----------------------------------------------------------------- O10 */
/* Depth -> horizontal shift (Section 4, Fig. 3 code): a filtered depth above
 * the threshold (150) is shifted one way in proportion to D/255, otherwise the
 * other way in proportion to 1 - D/255; the two views move symmetrically by
 * half the stereo base.  Reading: exact rational total parallax rounded half
 * up, P = round(B*m/255) with m = D (crossed, in front) or 255-D (uncrossed);
 * the left view takes ceil(P/2) and the right view floor(P/2), so the total is
 * exactly P and B is the maximum disparity.  T = -1 gives a linear mode in
 * which D = 0 has zero parallax. */
void oracle_disparity_lut(int B, int T, int32_t *P_out, int32_t *oL_out, int32_t *oR_out) {
    for (int D = 0; D < 256; D++) {
        int m, s;
        if (D > T) { m = D; s = +1; } else { m = 255 - D; s = -1; }
        int P = (B * m + 127) / 255;
        int a = (P + 1) / 2;
        int b = P / 2;
        P_out[D] = s * P;
        oL_out[D] = s * a;
        oR_out[D] = -s * b;
    }
}

/* ------------------------------------------------- row-range stages */
/* The row-independent stages below each take a half-open range of image rows
 * [y0, y1); the whole-frame entry runs them over all rows, either in one call or split
 * into row bands on several threads (the CPU baseline's row-parallel mode).
 * A band's result does not depend on how the rows are split. */

/* O1: luma of every pixel of rows y0..y1-1. */
static void orc_luma_rows(const uint8_t *frame, int w, int y0, int y1, uint8_t *Y) {
    for (int64_t i = (int64_t)y0 * w; i < (int64_t)y1 * w; i++)
        Y[i] = (uint8_t)orc_luma(frame[3 * i], frame[3 * i + 1], frame[3 * i + 2]);
}

#define RAMP(row) (gh > 1 ? (255 * (row) + (gh - 1) / 2) / (gh - 1) : 0)

/* O8: pixel depth.  Non-edge block: its region depth.  Edge block: the
 * region depth of the non-edge block among the 3x3 neighbours whose mean
 * colour is nearest (L1) to the pixel, first strict minimum in raster order;
 * with no candidate, the ramp of the block row. */
static void orc_depth_rows(const uint8_t *frame, int w, int K, int gw, int gh, const uint32_t *stats,
                           const uint8_t *dblk, int y0, int y1, uint8_t *D0) {
    for (int y = y0; y < y1; y++) {
        for (int x = 0; x < w; x++) {
            int64_t i = (int64_t)y * w + x;
            int bx = x / K, by = y / K, b = by * gw + bx;
            if (!(stats[b] >> 24)) { D0[i] = dblk[b]; continue; }
            int best = -1, bestd = 0;
            for (int dy = -1; dy <= 1; dy++) {
                for (int dx = -1; dx <= 1; dx++) {
                    int cx = bx + dx, cy = by + dy;
                    if (cx < 0 || cx >= gw || cy < 0 || cy >= gh) continue;
                    uint32_t sc = stats[cy * gw + cx];
                    if (sc >> 24) continue;
                    int d = 0;
                    for (int c = 0; c < 3; c++)
                        d += abs((int)frame[3 * i + c] - (int)((sc >> (8 * c)) & 255));
                    if (best < 0 || d < bestd) { best = cy * gw + cx; bestd = d; }
                }
            }
            D0[i] = best >= 0 ? dblk[best] : (uint8_t)RAMP(by);
        }
    }
}

/* O9: cross-bilateral filter of the depth map guided by luma: window
 * (2r+1)^2 clipped to the image, weight ws[dx^2+dy^2] * wr[|Y(q)-Y(p)|],
 * normalised sum rounded half up. */
static void orc_cbf_rows(const uint8_t *Y, const uint8_t *D0, int w, int h, int r, int y0, int y1,
                         uint8_t *Df) {
    for (int y = y0; y < y1; y++) {
        for (int x = 0; x < w; x++) {
            int64_t i = (int64_t)y * w + x;
            uint64_t acc = 0, wsum = 0;
            for (int dy = -r; dy <= r; dy++) {
                for (int dx = -r; dx <= r; dx++) {
                    int qx = x + dx, qy = y + dy;
                    if (qx < 0 || qx >= w || qy < 0 || qy >= h) continue;
                    int64_t q = (int64_t)qy * w + qx;
                    uint64_t wt = (uint64_t)orc_ws[dx * dx + dy * dy] * (uint64_t)orc_wr[abs((int)Y[q] - (int)Y[i])];
                    acc += wt * D0[q];
                    wsum += wt;
                }
            }
            Df[i] = (uint8_t)((acc + wsum / 2) / wsum);
        }
    }
}

/* O11 + O12 for one view over rows y0..y1-1; key and pick are w-entry
 * work rows of the caller. */
static void orc_view_rows(const uint8_t *frame, const uint8_t *Df, int w, int view, const int32_t *off,
                          int y0, int y1, uint32_t *key, int32_t *pick, uint8_t *V, int32_t *dw,
                          int32_t *ds) {
    for (int y = y0; y < y1; y++) {
        const int64_t row = (int64_t)y * w;
        /* O11: forward warp of every source pixel of the row to
         * x + offset(depth); at a collision the nearer source (larger
         * depth) wins, then the larger source x.  This is the left / right
         * frame reconstruction (Section 4, Fig. 3 code) written as a
         * z-buffered scatter instead of a gather at the destination's
         * depth. */
        for (int x = 0; x < w; x++) key[x] = 0;
        for (int x = 0; x < w; x++) {
            int d = Df[row + x];
            int xd = x + off[d];
            if (xd < 0 || xd >= w) continue;
            uint32_t k = (1u << 24) | ((uint32_t)d << 16) | (uint32_t)x;
            if (k > key[xd]) key[xd] = k;
        }
        /* O12: inpainting of holes (Section 3: post-processed frames;
         * Section 4: GPU inpainting).  A hole copies the nearer valid
         * pixel of the warped row on its left or right: the one with the
         * smaller depth (background); equal depths go left in the left
         * view and right in the right view; a row with no valid pixel
         * copies the source row, as the Fig. 3 code does for an
         * out-of-range shift.  Fill colours come from the warped row
         * before filling. */
        for (int xd = 0; xd < w; xd++) {
            if (key[xd]) { pick[xd] = (int32_t)(key[xd] & 0xFFFF); continue; }
            int xl = -1, xr = -1;
            for (int j = xd - 1; j >= 0; j--) if (key[j]) { xl = j; break; }
            for (int j = xd + 1; j < w; j++) if (key[j]) { xr = j; break; }
            int chosen;
            if (xl >= 0 && xr >= 0) {
                int dl = (key[xl] >> 16) & 255, dr = (key[xr] >> 16) & 255;
                if (dl < dr) chosen = xl;
                else if (dr < dl) chosen = xr;
                else chosen = view == 0 ? xl : xr;
                pick[xd] = (int32_t)(key[chosen] & 0xFFFF);
            } else if (xl >= 0) {
                pick[xd] = (int32_t)(key[xl] & 0xFFFF);
            } else if (xr >= 0) {
                pick[xd] = (int32_t)(key[xr] & 0xFFFF);
            } else {
                pick[xd] = xd;
            }
        }
        for (int xd = 0; xd < w; xd++) {
            int64_t src = row + pick[xd];
            for (int c = 0; c < 3; c++) V[3 * (row + xd) + c] = frame[3 * src + c];
            if (dw) dw[row + xd] = key[xd] ? (int32_t)(key[xd] & 0xFFFF) : -1;
            if (ds) ds[row + xd] = pick[xd];
        }
    }
}

/* O13: red-cyan anaglyph of rows y0..y1-1: red from the left view, green
 * and blue from the right view (Fig. 3 code: res from the left and right
 * reconstructions); the views copied out beside it. */
static void orc_compose_rows(const uint8_t *Lv, const uint8_t *Rv, int w, int y0, int y1, uint8_t *out_L,
                             uint8_t *out_R, uint8_t *out_A) {
    for (int64_t i = (int64_t)y0 * w; i < (int64_t)y1 * w; i++) {
        if (out_L) for (int c = 0; c < 3; c++) out_L[3 * i + c] = Lv[3 * i + c];
        if (out_R) for (int c = 0; c < 3; c++) out_R[3 * i + c] = Rv[3 * i + c];
        if (out_A) {
            out_A[3 * i + 0] = Lv[3 * i + 0];
            out_A[3 * i + 1] = Rv[3 * i + 1];
            out_A[3 * i + 2] = Rv[3 * i + 2];
        }
    }
}
#undef RAMP

/* One row-parallel stage: which stage, its arguments, and the band of rows of
 * one thread. */
typedef struct {
    int stage;  /* 1 luma, 8 pixel depth, 9 filter, 11 views + anaglyph */
    const uint8_t *frame;
    int w, h, K, gw, gh, r;
    const uint32_t *stats;
    const uint8_t *dblk;
    uint8_t *Y, *D0, *Df, *Lv, *Rv;
    const int32_t *offL, *offR;
    int32_t *dwL, *dwR, *dsL, *dsR;
    uint8_t *out_L, *out_R, *out_A;
    uint32_t *key;
    int32_t *pick;
    int y0, y1;
} orc_band;

static void *orc_band_run(void *arg) {
    orc_band *b = (orc_band *)arg;
    switch (b->stage) {
    case 1: orc_luma_rows(b->frame, b->w, b->y0, b->y1, b->Y); break;
    case 8: orc_depth_rows(b->frame, b->w, b->K, b->gw, b->gh, b->stats, b->dblk, b->y0, b->y1, b->D0); break;
    case 9: orc_cbf_rows(b->Y, b->D0, b->w, b->h, b->r, b->y0, b->y1, b->Df); break;
    case 11:
        orc_view_rows(b->frame, b->Df, b->w, 0, b->offL, b->y0, b->y1, b->key, b->pick, b->Lv, b->dwL, b->dsL);
        orc_view_rows(b->frame, b->Df, b->w, 1, b->offR, b->y0, b->y1, b->key, b->pick, b->Rv, b->dwR, b->dsR);
        orc_compose_rows(b->Lv, b->Rv, b->w, b->y0, b->y1, b->out_L, b->out_R, b->out_A);
        break;
    }
    return NULL;
}

/* Run one stage over all rows: in the calling thread (nthreads <= 1), or in
 * nthreads contiguous row bands, each on its own thread.  Returns 0, or
 * ORC_E_NOMEM if a thread or its work rows could not be created. */
static int orc_rows(orc_band proto, int nthreads) {
    if (nthreads > proto.h) nthreads = proto.h;
    if (nthreads <= 1) {
        proto.y0 = 0;
        proto.y1 = proto.h;
        orc_band_run(&proto);
        return ORC_OK;
    }
    orc_band *bands = calloc((size_t)nthreads, sizeof(orc_band));
    pthread_t *tid = calloc((size_t)nthreads, sizeof(pthread_t));
    int *started = calloc((size_t)nthreads, sizeof(int));
    int rc = (bands && tid && started) ? ORC_OK : ORC_E_NOMEM;
    for (int t = 0; rc == ORC_OK && t < nthreads; t++) {
        bands[t] = proto;
        bands[t].y0 = (int)((int64_t)proto.h * t / nthreads);
        bands[t].y1 = (int)((int64_t)proto.h * (t + 1) / nthreads);
        bands[t].key = NULL;
        bands[t].pick = NULL;
        if (proto.stage == 11) {
            bands[t].key = malloc(sizeof(uint32_t) * proto.w);
            bands[t].pick = malloc(sizeof(int32_t) * proto.w);
            if (!bands[t].key || !bands[t].pick) { rc = ORC_E_NOMEM; break; }
        }
        if (pthread_create(&tid[t], NULL, orc_band_run, &bands[t]) != 0) { rc = ORC_E_NOMEM; break; }
        started[t] = 1;
    }
    for (int t = 0; t < nthreads; t++)
        if (started && started[t]) pthread_join(tid[t], NULL);
    for (int t = 0; bands && t < nthreads; t++) { free(bands[t].key); free(bands[t].pick); }
    free(bands);
    free(tid);
    free(started);
    return rc;
}

/* -------------------------------------------------------------- driver */
static int orc_synthesize(const uint8_t *frame, int w, int h,
                          int B, int T, int K, int g, int tau, int r,
                          const uint8_t *depth_in,
                          uint8_t *out_L, uint8_t *out_R, uint8_t *out_A,
                          uint8_t *dump_Y, uint32_t *dump_stats, int32_t *dump_labels,
                          uint8_t *dump_dblk, uint8_t *dump_D0, uint8_t *dump_Df,
                          int32_t *dump_warpL, int32_t *dump_warpR,
                          int32_t *dump_srcL, int32_t *dump_srcR, int nthreads) {
    if (!frame || w < 1 || h < 1 || w > 65535 || h > 65535) return ORC_E_INVALID;
    if (B < 0 || B > 255 || T < -1 || T > 255 || r < 0 || r > ORC_MAX_RADIUS) return ORC_E_INVALID;
    if (g < 0 || g > 255 || tau < 0 || tau > 765) return ORC_E_INVALID;
    if (K == 0) K = oracle_auto_block(w, h);
    if (K < 1 || K > 64) return ORC_E_INVALID;
    const int gw = (w + K - 1) / K, gh = (h + K - 1) / K;
    const int nb = gw * gh;
    if (!depth_in && (int64_t)gw * gh > ORC_MAX_BLOCKS) return ORC_E_INVALID;
    orc_build_tables();

    const int64_t npx = (int64_t)w * h;
    uint8_t *Y = malloc(npx), *D0 = malloc(npx), *Df = malloc(npx);
    uint32_t *stats = malloc(sizeof(uint32_t) * nb);
    int32_t *lab = malloc(sizeof(int32_t) * nb);
    uint8_t *dblk = malloc(nb);
    uint8_t *linkR = malloc(nb), *linkD = malloc(nb);
    int32_t *cnt = malloc(sizeof(int32_t) * nb), *rmax = malloc(sizeof(int32_t) * nb);
    uint32_t *key = malloc(sizeof(uint32_t) * w);
    int32_t *pick = malloc(sizeof(int32_t) * w);
    uint8_t *Lv = malloc(3 * npx), *Rv = malloc(3 * npx);
    int ok = Y && D0 && Df && stats && lab && dblk && linkR && linkD && cnt && rmax && key && pick && Lv && Rv;
    int rc = ORC_OK;
    if (!ok) { rc = ORC_E_NOMEM; goto done; }

    orc_band band;
    memset(&band, 0, sizeof band);
    band.frame = frame;
    band.w = w;
    band.h = h;
    band.K = K;
    band.gw = gw;
    band.gh = gh;
    band.r = r;
    band.stats = stats;
    band.dblk = dblk;
    band.Y = Y;
    band.D0 = D0;
    band.Df = Df;
    band.Lv = Lv;
    band.Rv = Rv;

    /* O1: luma of every pixel. */
    band.stage = 1;
    if ((rc = orc_rows(band, nthreads)) != ORC_OK) goto done;

    /* ramp h(row): top of the frame far (0), bottom near (255); larger depth
     * value = nearer, as the Fig. 3 code sends D > 150 to the crossed shift. */
#define RAMP(row) (gh > 1 ? (255 * (row) + (gh - 1) / 2) / (gh - 1) : 0)

    if (depth_in) {
        /* depth supplied by the caller: it replaces the depth map (O2-O8) */
        memcpy(D0, depth_in, npx);
        for (int b = 0; b < nb; b++) { stats[b] = 0; lab[b] = b; dblk[b] = 0; }
    } else {
        /* O3: rounded block means of R, G, B.  O4: edge flag = some forward
         * luma difference (right or down, possibly into the next block) above
         * g.  These are the edge / region-boundary cues of the depth
         * generation (Section 2 on the edge-information system; Table 1:
         * region boundary information). */
        for (int by = 0; by < gh; by++) {
            for (int bx = 0; bx < gw; bx++) {
                int64_t s[3] = {0, 0, 0};
                int n = 0, e = 0;
                for (int y = by * K; y < (by + 1) * K && y < h; y++) {
                    for (int x = bx * K; x < (bx + 1) * K && x < w; x++) {
                        int64_t i = (int64_t)y * w + x;
                        for (int c = 0; c < 3; c++) s[c] += frame[3 * i + c];
                        n++;
                        if (x + 1 < w && abs((int)Y[i + 1] - (int)Y[i]) > g) e = 1;
                        if (y + 1 < h && abs((int)Y[i + w] - (int)Y[i]) > g) e = 1;
                    }
                }
                uint32_t mu[3];
                for (int c = 0; c < 3; c++) mu[c] = (uint32_t)((s[c] + n / 2) / n);
                stats[by * gw + bx] = mu[0] | (mu[1] << 8) | (mu[2] << 16) | ((uint32_t)e << 24);
            }
        }

        /* O5: right / down neighbours are linked when both are non-edge blocks
         * and their mean colours differ by at most tau in summed L1 distance. */
        for (int b = 0; b < nb; b++) {
            int bx = b % gw, by = b / gw;
            linkR[b] = 0;
            linkD[b] = 0;
            uint32_t sb = stats[b];
            if (sb >> 24) continue;
            if (bx + 1 < gw && !(stats[b + 1] >> 24)) {
                uint32_t sn = stats[b + 1];
                int d = 0;
                for (int c = 0; c < 3; c++)
                    d += abs((int)((sb >> (8 * c)) & 255) - (int)((sn >> (8 * c)) & 255));
                linkR[b] = d <= tau;
            }
            if (by + 1 < gh && !(stats[b + gw] >> 24)) {
                uint32_t sn = stats[b + gw];
                int d = 0;
                for (int c = 0; c < 3; c++)
                    d += abs((int)((sb >> (8 * c)) & 255) - (int)((sn >> (8 * c)) & 255));
                linkD[b] = d <= tau;
            }
        }

        /* O6: region label = minimum block index of the connected component of
         * the link graph, reached by iterating min-label propagation until
         * nothing changes (the "iterative" depth generation of Section 4). */
        for (int b = 0; b < nb; b++) lab[b] = b;
        for (int changed = 1; changed;) {
            changed = 0;
            for (int pass = 0; pass < 2; pass++) {
                for (int i = 0; i < nb; i++) {
                    int b = pass == 0 ? i : nb - 1 - i;
                    int bx = b % gw, by = b / gw;
                    int m = lab[b];
                    if (bx + 1 < gw && linkR[b] && lab[b + 1] < m) m = lab[b + 1];
                    if (bx > 0 && linkR[b - 1] && lab[b - 1] < m) m = lab[b - 1];
                    if (by + 1 < gh && linkD[b] && lab[b + gw] < m) m = lab[b + gw];
                    if (by > 0 && linkD[b - gw] && lab[b - gw] < m) m = lab[b - gw];
                    if (m < lab[b]) { lab[b] = m; changed = 1; }
                }
            }
        }

        /* O7: region depth.  Background = the largest non-edge region (ties:
         * smaller label); it follows the row ramp.  Any other non-edge region
         * sits at the ramp depth of its lowest block row (ground contact).
         * Edge blocks get the ramp of their own row; that value is only a
         * placeholder, O8 never reads it. */
        for (int b = 0; b < nb; b++) { cnt[b] = 0; rmax[b] = -1; }
        for (int b = 0; b < nb; b++) {
            if (stats[b] >> 24) continue;
            cnt[lab[b]]++;
            if (b / gw > rmax[lab[b]]) rmax[lab[b]] = b / gw;
        }
        int bg = -1;
        for (int l = 0; l < nb; l++)
            if (cnt[l] > 0 && (bg < 0 || cnt[l] > cnt[bg])) bg = l;
        for (int b = 0; b < nb; b++) {
            int by = b / gw;
            if ((stats[b] >> 24) || lab[b] == bg) dblk[b] = (uint8_t)RAMP(by);
            else dblk[b] = (uint8_t)RAMP(rmax[lab[b]]);
        }

        /* O8: pixel depth (orc_depth_rows). */
        band.stage = 8;
        if ((rc = orc_rows(band, nthreads)) != ORC_OK) goto done;
    }
#undef RAMP

    /* O9: cross-bilateral filter (orc_cbf_rows). */
    band.stage = 9;
    if ((rc = orc_rows(band, nthreads)) != ORC_OK) goto done;

    /* O10: depth -> per-view offsets. */
    int32_t lutP[256], lutL[256], lutR[256];
    oracle_disparity_lut(B, T, lutP, lutL, lutR);

    /* O11 + O12 per view, then O13, row by row (orc_view_rows,
     * orc_compose_rows). */
    band.stage = 11;
    band.offL = lutL;
    band.offR = lutR;
    band.dwL = dump_warpL;
    band.dwR = dump_warpR;
    band.dsL = dump_srcL;
    band.dsR = dump_srcR;
    band.out_L = out_L;
    band.out_R = out_R;
    band.out_A = out_A;
    band.key = key;
    band.pick = pick;
    if ((rc = orc_rows(band, nthreads)) != ORC_OK) goto done;

    if (dump_Y) memcpy(dump_Y, Y, npx);
    if (dump_D0) memcpy(dump_D0, D0, npx);
    if (dump_Df) memcpy(dump_Df, Df, npx);
    if (dump_stats) memcpy(dump_stats, stats, sizeof(uint32_t) * nb);
    if (dump_labels) memcpy(dump_labels, lab, sizeof(int32_t) * nb);
    if (dump_dblk) memcpy(dump_dblk, dblk, nb);

done:
    free(Y); free(D0); free(Df); free(stats); free(lab); free(dblk);
    free(linkR); free(linkD); free(cnt); free(rmax); free(key); free(pick);
    free(Lv); free(Rv);
    return rc;
}

int oracle_synthesize(const uint8_t *frame, int w, int h,
                      int B, int T, int K, int g, int tau, int r,
                      const uint8_t *depth_in,
                      uint8_t *out_L, uint8_t *out_R, uint8_t *out_A,
                      uint8_t *dump_Y, uint32_t *dump_stats, int32_t *dump_labels,
                      uint8_t *dump_dblk, uint8_t *dump_D0, uint8_t *dump_Df,
                      int32_t *dump_warpL, int32_t *dump_warpR,
                      int32_t *dump_srcL, int32_t *dump_srcR) {
    return orc_synthesize(frame, w, h, B, T, K, g, tau, r, depth_in, out_L, out_R, out_A, dump_Y, dump_stats,
                          dump_labels, dump_dblk, dump_D0, dump_Df, dump_warpL, dump_warpR, dump_srcL, dump_srcR, 1);
}

/* The same pipeline with its row-independent stages (O1, O8, O9, O11-O13)
 * split into nthreads row bands on as many threads; the block stages O2-O7
 * stay on the calling thread.  Outputs only (the CPU baseline's row-parallel
 * mode); they equal oracle_synthesize's for any nthreads. */
int oracle_synthesize_mt(const uint8_t *frame, int w, int h, int B, int T, int K, int g, int tau, int r,
                         uint8_t *out_L, uint8_t *out_R, uint8_t *out_A, int nthreads) {
    return orc_synthesize(frame, w, h, B, T, K, g, tau, r, NULL, out_L, out_R, out_A, NULL, NULL, NULL, NULL, NULL,
                          NULL, NULL, NULL, NULL, NULL, nthreads < 1 ? 1 : nthreads);
}

/* ---------------------------------------------------------- HSBS output */
/* Half side-by-side stereo frame, the second output format the paper's
 * timing compares against the anaglyph (Section 5).  The format is only named;
 * the reading: an image of the input's size whose left half holds the left
 * view squeezed to half width and whose right half holds the right view
 * squeezed likewise.  Column p of a half is the mean of columns 2p and 2p+1 of
 * its view, per channel, rounded half up.  The left half has floor(w/2)
 * columns and the right half the remaining ceil(w/2); for odd w the right
 * half's last column has only column w-1 of the right view and copies it. */
int oracle_hsbs(const uint8_t *L, const uint8_t *R, int w, int h, uint8_t *out) {
    if (!L || !R || !out || w < 1 || h < 1) return ORC_E_INVALID;
    const int hw = w / 2;
    for (int y = 0; y < h; ++y) {
        const uint8_t *lrow = L + (size_t)y * w * 3;
        const uint8_t *rrow = R + (size_t)y * w * 3;
        uint8_t *orow = out + (size_t)y * w * 3;
        for (int p = 0; p < hw; ++p) {
            for (int c = 0; c < 3; ++c) {
                const int a = lrow[(2 * p) * 3 + c], b = lrow[(2 * p + 1) * 3 + c];
                orow[p * 3 + c] = (uint8_t)((a + b + 1) / 2);
            }
        }
        for (int p = 0; hw + p < w; ++p) {
            for (int c = 0; c < 3; ++c) {
                int v;
                if (2 * p + 1 < w) {
                    const int a = rrow[(2 * p) * 3 + c], b = rrow[(2 * p + 1) * 3 + c];
                    v = (a + b + 1) / 2;
                } else {
                    v = rrow[(2 * p) * 3 + c];
                }
                orow[(hw + p) * 3 + c] = (uint8_t)v;
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------- Fig. 3 gather warp */
/* The reconstruction exactly as the Fig. 3 code organises it: every
 * destination pixel reads the filtered depth at its own position, takes the
 * per-view offset of that depth (the O10 table, the reading of the code's
 * shift expressions) and copies the source pixel it points back to; a source
 * position outside the row copies the destination's own source pixel, as the
 * code's else branches do.  There is no occlusion test and nothing is left to
 * fill.  The anaglyph takes red from the gathered left view and green and
 * blue from the gathered right view, as the code writes res.  Df is the
 * filtered depth map of the frame (u8 [h][w]). */
int oracle_gather(const uint8_t *frame, const uint8_t *Df, int w, int h, int B, int T,
                  uint8_t *out_L, uint8_t *out_R, uint8_t *out_A) {
    if (!frame || !Df || w < 1 || h < 1 || B < 0 || B > 255 || T < -1 || T > 255) return ORC_E_INVALID;
    int32_t lutP[256], lutL[256], lutR[256];
    oracle_disparity_lut(B, T, lutP, lutL, lutR);
    for (int y = 0; y < h; y++) {
        for (int x = 0; x < w; x++) {
            const int d = Df[(size_t)y * w + x];
            int xl = x - lutL[d], xr = x - lutR[d];
            if (xl < 0 || xl >= w) xl = x;
            if (xr < 0 || xr >= w) xr = x;
            const uint8_t *sl = frame + ((size_t)y * w + xl) * 3;
            const uint8_t *sr = frame + ((size_t)y * w + xr) * 3;
            const size_t o = ((size_t)y * w + x) * 3;
            for (int c = 0; c < 3; c++) {
                if (out_L) out_L[o + c] = sl[c];
                if (out_R) out_R[o + c] = sr[c];
            }
            if (out_A) {
                out_A[o + 0] = sl[0];
                out_A[o + 1] = sr[1];
                out_A[o + 2] = sr[2];
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------ block-iterative inpainting */
/* The inpainting algorithm of Fig. 3 (Section 4), as an alternative to the
 * row fill.  Its pseudocode leaves the neighbourhood, the colour rule, the
 * block size, the update order and the stopping rule open; the reading:
 *   - damaged pixels are the holes of the forward warp (warp[y][x] < 0);
 *   - one block is the whole frame;
 *   - sweeps are simultaneous (Jacobi): in each sweep every pixel that is
 *     damaged at its start and has at least two undamaged pixels among its
 *     8 neighbours (at the sweep's start) becomes undamaged, with the mean of
 *     those neighbours' colours per channel, rounded half up;
 *   - the sweeps stop when one fills nothing; a pixel still damaged then keeps
 *     its own source pixel (as the Fig. 3 code does for a destination whose
 *     source is out of range).
 * frame: source RGB24; warp: winning source x per destination (-1 = hole);
 * out: the inpainted view.  Returns the number of sweeps that filled pixels,
 * or a negative code. */
int oracle_inpaint_blocks(const uint8_t *frame, const int32_t *warp, int w, int h, uint8_t *out) {
    if (!frame || !warp || !out || w < 1 || h < 1) return ORC_E_INVALID;
    const size_t n = (size_t)w * h;
    uint8_t *dmg = (uint8_t *)malloc(n), *dmg2 = (uint8_t *)malloc(n);
    uint8_t *col2 = (uint8_t *)malloc(n * 3);
    if (!dmg || !dmg2 || !col2) {
        free(dmg); free(dmg2); free(col2);
        return ORC_E_NOMEM;
    }
    for (int y = 0; y < h; y++) {
        for (int x = 0; x < w; x++) {
            const size_t i = (size_t)y * w + x;
            const int s = warp[i];
            dmg[i] = s < 0;
            for (int c = 0; c < 3; c++) out[i * 3 + c] = s < 0 ? 0 : frame[((size_t)y * w + s) * 3 + c];
        }
    }
    int sweeps = 0;
    for (;;) {
        int filled = 0;
        memcpy(dmg2, dmg, n);
        memcpy(col2, out, n * 3);
        for (int y = 0; y < h; y++) {
            for (int x = 0; x < w; x++) {
                const size_t i = (size_t)y * w + x;
                if (!dmg[i]) continue;
                int cnt = 0, sum[3] = {0, 0, 0};
                for (int dy = -1; dy <= 1; dy++) {
                    for (int dx = -1; dx <= 1; dx++) {
                        if (!dx && !dy) continue;
                        const int yy = y + dy, xx = x + dx;
                        if (yy < 0 || yy >= h || xx < 0 || xx >= w) continue;
                        const size_t j = (size_t)yy * w + xx;
                        if (dmg[j]) continue;
                        cnt++;
                        for (int c = 0; c < 3; c++) sum[c] += out[j * 3 + c];
                    }
                }
                if (cnt >= 2) {
                    for (int c = 0; c < 3; c++) col2[i * 3 + c] = (uint8_t)((sum[c] + cnt / 2) / cnt);
                    dmg2[i] = 0;
                    filled++;
                }
            }
        }
        if (!filled) break;
        memcpy(dmg, dmg2, n);
        memcpy(out, col2, n * 3);
        sweeps++;
    }
    for (size_t i = 0; i < n; i++)
        if (dmg[i])
            for (int c = 0; c < 3; c++) out[i * 3 + c] = frame[i * 3 + c];
    free(dmg); free(dmg2); free(col2);
    return sweeps;
}
