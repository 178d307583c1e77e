// C ABI of the batched form: many frames of uneven size through one
// persistent kernel launch (kernels_batch.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pstereo.h"
#include "pstereo_batch.h"
#include "pstereo_internal.h"

using pstereo::BatchDesc;
using pstereo::BatchSeg;
using pstereo::FrameDesc;

struct pstereo_batch {
    pstereo_ctx* ctx = nullptr;
    int device = 0;
    int max_jobs = 0;
    int64_t max_pixels = 0;
    int grid = 0;
    // device tables and per-frame scratch
    FrameDesc* d_frames = nullptr;
    BatchSeg* d_segs = nullptr;
    int* d_need = nullptr;
    uint32_t* d_ctr = nullptr;
    uint32_t* d_stats = nullptr;
    uint2* d_binfo = nullptr;
    int32_t* d_labels = nullptr;
    uint8_t* d_df = nullptr;
    // pinned staging of the tables
    FrameDesc* h_frames = nullptr;
    BatchSeg* h_segs = nullptr;
    int* h_need = nullptr;
    hipEvent_t staged = nullptr;
    bool staged_pending = false;
    // the prepared batch
    int n = 0, ntask = 0, r = 2;
    int qseg[pstereo::kXcds + 1] = {};  // fused form: segments of each XCD's queue
    int qntask[pstereo::kXcds] = {};
    bool prepared = false;
    // tuning and the staged form's tables
    pstereo_batch_tuning tune{PSTEREO_BATCH_STAGED, 256, 1, 0, 0};
    int cus = 0;
    int* d_first = nullptr;
    int* h_first = nullptr;
    pstereo::StagedPlan plan;
    hipStream_t stream = nullptr;
    std::string err;
};

namespace {

int bfail(pstereo_batch* b, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    b->err = buf;
    return code;
}

int dev_ptr_ok(const void* p, int device) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == device;
}

int auto_block_size(int w, int h) {
    static const int cand[4] = {8, 16, 32, 64};
    for (int K : cand)
        if ((long long)((w + K - 1) / K) * ((h + K - 1) / K) <= PSTEREO_MAX_BLOCKS) return K;
    return -1;
}

void batch_free(pstereo_batch* b) {
    (void)hipSetDevice(b->device);
    if (b->staged) {
        (void)hipEventSynchronize(b->staged);
        (void)hipEventDestroy(b->staged);
    }
    (void)hipFree(b->d_frames);
    (void)hipFree(b->d_segs);
    (void)hipFree(b->d_need);
    (void)hipFree(b->d_ctr);
    (void)hipFree(b->d_first);
    (void)hipHostFree(b->h_first);
    (void)hipFree(b->d_stats);
    (void)hipFree(b->d_binfo);
    (void)hipFree(b->d_labels);
    (void)hipFree(b->d_df);
    (void)hipHostFree(b->h_frames);
    (void)hipHostFree(b->h_segs);
    (void)hipHostFree(b->h_need);
    (void)hipGetLastError();
    delete b;
}

}  // namespace

namespace pstereo {

int batch_create_internal(pstereo_ctx* ctx, int max_jobs, int64_t max_pixels, bool own_scratch, pstereo_batch** out) {
    if (!ctx || !out || max_jobs < 1 || max_jobs > 4096 || max_pixels < 1) return PSTEREO_E_INVALID;
    *out = nullptr;
    pstereo_batch* b = new (std::nothrow) pstereo_batch;
    if (!b) return PSTEREO_E_NOMEM;
    b->ctx = ctx;
    b->device = pstereo::ctx_device(ctx);
    b->max_jobs = max_jobs;
    b->max_pixels = max_pixels;
    if (hipSetDevice(b->device) != hipSuccess) {
        delete b;
        return PSTEREO_E_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->device) != hipSuccess || pstereo::prepare_batch_kernels() != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return PSTEREO_E_DEVICE;
    }
    b->cus = prop.multiProcessorCount;
    b->grid = b->cus;  // fused form: one 1024-lane workgroup per CU
    const size_t first_ints = (size_t)(2 + pstereo::kMaxWarpClasses) * (max_jobs + 1);
    const size_t nb = PSTEREO_MAX_BLOCKS;
    const size_t df_bytes = (size_t)max_pixels + 256 * (size_t)max_jobs;
    bool ok = hipMalloc(&b->d_frames, sizeof(FrameDesc) * max_jobs) == hipSuccess &&
              hipMalloc(&b->d_segs, sizeof(BatchSeg) * 4 * max_jobs) == hipSuccess &&
              hipMalloc(&b->d_need, sizeof(int) * 4 * max_jobs) == hipSuccess &&
              hipMalloc(&b->d_ctr, sizeof(uint32_t) * (pstereo::kXcds + 1 + 4 * max_jobs)) == hipSuccess &&
              hipMalloc(&b->d_first, sizeof(int) * first_ints) == hipSuccess &&
              hipHostMalloc(&b->h_first, sizeof(int) * first_ints, hipHostMallocDefault) == hipSuccess &&
              (!own_scratch || (hipMalloc(&b->d_stats, sizeof(uint32_t) * nb * max_jobs) == hipSuccess &&
                                hipMalloc(&b->d_binfo, sizeof(uint2) * nb * max_jobs) == hipSuccess &&
                                hipMalloc(&b->d_labels, sizeof(int32_t) * nb * max_jobs) == hipSuccess &&
                                hipMalloc(&b->d_df, df_bytes) == hipSuccess)) &&
              hipHostMalloc(&b->h_frames, sizeof(FrameDesc) * max_jobs, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&b->h_segs, sizeof(BatchSeg) * 4 * max_jobs, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&b->h_need, sizeof(int) * 4 * max_jobs, hipHostMallocDefault) == hipSuccess &&
              hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        batch_free(b);
        return PSTEREO_E_NOMEM;
    }
    *out = b;
    return PSTEREO_OK;
}

}  // namespace pstereo

extern "C" {

int pstereo_batch_create(pstereo_ctx* ctx, int max_jobs, int64_t max_pixels, pstereo_batch** out) {
    return pstereo::batch_create_internal(ctx, max_jobs, max_pixels, true, out);
}

int pstereo_batch_destroy(pstereo_batch* b) {
    if (!b) return PSTEREO_OK;
    batch_free(b);
    return PSTEREO_OK;
}

const char* pstereo_batch_last_error(const pstereo_batch* b) { return b ? b->err.c_str() : ""; }

int pstereo_batch_prepare(pstereo_batch* b, const pstereo_job* jobs, int n, const pstereo_params* pin) {
    return pstereo::batch_prepare_internal(b, jobs, n, pin, nullptr, true);
}

}  // extern "C"

namespace pstereo {

int batch_prepare_internal(pstereo_batch* b, const pstereo_job* jobs, int n, const pstereo_params* pin,
                           const JobScratch* scratch, bool check_ptrs) {
    if (!b) return PSTEREO_E_INVALID;
    b->err.clear();
    b->prepared = false;
    if (!jobs || n < 1 || n > b->max_jobs) return bfail(b, PSTEREO_E_INVALID, "job count %d outside 1..%d", n, b->max_jobs);
    pstereo_params p;
    pstereo_params_init(&p);
    if (pin) {
        if (pin->struct_size != sizeof(pstereo_params)) return bfail(b, PSTEREO_E_INVALID, "params.struct_size mismatch");
        p = *pin;
    }
    if (p.flags & (PSTEREO_DEPTH_EXTERNAL | PSTEREO_WARP_GATHER | PSTEREO_INPAINT_BLOCKS))
        return bfail(b, PSTEREO_E_UNSUPPORTED, "batches generate their depth maps and warp");
    if (p.out_depth || p.out_depth_raw || p.out_hsbs)
        return bfail(b, PSTEREO_E_UNSUPPORTED, "batches take no depth dumps or half side-by-side output");
    if (p.depth_threshold < -1 || p.depth_threshold > 255) return bfail(b, PSTEREO_E_INVALID, "depth_threshold out of range");
    if (p.cbf_radius < 0 || p.cbf_radius > 3) return bfail(b, PSTEREO_E_INVALID, "cbf_radius out of range");
    if (p.edge_thresh < 0 || p.edge_thresh > 255) return bfail(b, PSTEREO_E_INVALID, "edge_thresh out of range");
    if (p.link_thresh < 0 || p.link_thresh > 765) return bfail(b, PSTEREO_E_INVALID, "link_thresh out of range");
    if (p.block_size && p.block_size != 2 && p.block_size != 4 && p.block_size != 8 && p.block_size != 16 &&
        p.block_size != 32 && p.block_size != 64)
        return bfail(b, PSTEREO_E_INVALID, "block_size %d not in {2,4,8,16,32,64}", p.block_size);
    (void)hipSetDevice(b->device);
    // the staging buffers may still feed the previous prepare's copies
    if (b->staged_pending) {
        if (hipEventSynchronize(b->staged) != hipSuccess) return bfail(b, PSTEREO_E_DEVICE, "event synchronize");
        b->staged_pending = false;
    }
    int64_t px_total = 0;
    size_t df_off = 0;
    for (int i = 0; i < n; ++i) {
        const pstereo_job& j = jobs[i];
        if (!j.frame || j.w < 1 || j.h < 1) return bfail(b, PSTEREO_E_INVALID, "job %d: bad frame or size", i);
        if (j.w % 4 != 0) return bfail(b, PSTEREO_E_UNSUPPORTED, "job %d: width %d not a multiple of 4", i, j.w);
        if (b->tune.mode == PSTEREO_BATCH_FUSED && !pstereo::batch_width_ok(j.w))
            return bfail(b, PSTEREO_E_UNSUPPORTED, "job %d: width %d too large for the fused form", i, j.w);
        const uintptr_t al = (uintptr_t)j.frame | (uintptr_t)j.out_left | (uintptr_t)j.out_right | (uintptr_t)j.out_anaglyph;
        if (al % 4) return bfail(b, PSTEREO_E_UNSUPPORTED, "job %d: buffers must be 4-byte aligned", i);
        const int B = j.max_disparity < 0 ? (2 * j.w + 50) / 100 : j.max_disparity;
        if (j.max_disparity < -1 || B > 255) return bfail(b, PSTEREO_E_INVALID, "job %d: max_disparity out of range", i);
        const int K = p.block_size ? p.block_size : auto_block_size(j.w, j.h);
        if (K < 0) return bfail(b, PSTEREO_E_INVALID, "job %d: frame too large for the block grid", i);
        const int gw = (j.w + K - 1) / K, gh = (j.h + K - 1) / K;
        if ((long long)gw * gh > PSTEREO_MAX_BLOCKS) return bfail(b, PSTEREO_E_INVALID, "job %d: too many blocks", i);
        if (check_ptrs) {
            if (!dev_ptr_ok(j.frame, b->device)) return bfail(b, PSTEREO_E_INVALID, "job %d: frame is not device memory", i);
            const uint8_t* outs[3] = {j.out_left, j.out_right, j.out_anaglyph};
            for (const uint8_t* o : outs)
                if (o && !dev_ptr_ok(o, b->device))
                    return bfail(b, PSTEREO_E_INVALID, "job %d: output is not device memory", i);
        }
        px_total += (int64_t)j.w * j.h;
        if (!scratch && px_total > b->max_pixels)
            return bfail(b, PSTEREO_E_INVALID, "batch exceeds %lld pixels", (long long)b->max_pixels);
        FrameDesc f{};
        f.frame = j.frame;
        f.out_l = j.out_left;
        f.out_r = j.out_right;
        f.out_a = j.out_anaglyph;
        if (scratch) {
            f.stats = scratch[i].stats;
            f.binfo = scratch[i].binfo;
            f.labels = scratch[i].labels;
            f.df = scratch[i].df;
        } else {
            f.stats = b->d_stats + (size_t)i * PSTEREO_MAX_BLOCKS;
            f.binfo = b->d_binfo + (size_t)i * PSTEREO_MAX_BLOCKS;
            f.labels = b->d_labels + (size_t)i * PSTEREO_MAX_BLOCKS;
            f.df = b->d_df + df_off;
            df_off += ((size_t)j.w * j.h + 255) / 256 * 256;
        }
        f.w = j.w;
        f.h = j.h;
        f.K = K;
        f.gw = gw;
        f.gh = gh;
        f.B = B;
        f.T = p.depth_threshold;
        f.g = p.edge_thresh;
        f.tau = p.link_thresh;
        f.r = p.cbf_radius;
        f.aligned = 1;
        b->h_frames[i] = f;
    }
    // outputs must not overlap any frame or other output of the batch
    // (a server checks each request once, when it is submitted)
    struct Rng { const uint8_t* p; size_t n; };
    std::vector<Rng> ins, outs;
    for (int i = 0; i < n; ++i) {
        const size_t img = (size_t)jobs[i].w * jobs[i].h * 3;
        ins.push_back({jobs[i].frame, img});
        const uint8_t* o[3] = {jobs[i].out_left, jobs[i].out_right, jobs[i].out_anaglyph};
        for (const uint8_t* x : o) if (x) outs.push_back({x, img});
    }
    if (!check_ptrs) outs.clear();
    for (size_t a = 0; a < outs.size(); ++a) {
        for (const Rng& r : ins)
            if (outs[a].p < r.p + r.n && r.p < outs[a].p + outs[a].n) return bfail(b, PSTEREO_E_ALIAS, "an output overlaps a frame");
        for (size_t c = a + 1; c < outs.size(); ++c)
            if (outs[a].p < outs[c].p + outs[c].n && outs[c].p < outs[a].p + outs[a].n)
                return bfail(b, PSTEREO_E_ALIAS, "two outputs overlap");
    }
    b->n = n;
    b->r = p.cbf_radius;
    b->stream = (hipStream_t)p.stream;  // NULL: the HIP null stream
    hipStream_t st = b->stream;
    hipError_t e;
    if (b->tune.mode == PSTEREO_BATCH_FUSED) {
        // frames to the XCDs' queues, largest first onto the queue with the
        // fewest pixels; per queue, tasks in claim order: (blockstats,
        // regions) of each of its frames, then (depth filter, warp) of each
        constexpr int X = pstereo::kXcds;
        std::vector<int> order(n), owner(n);
        for (int i = 0; i < n; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
            return (int64_t)jobs[a].w * jobs[a].h > (int64_t)jobs[c].w * jobs[c].h;
        });
        int64_t load[X] = {};
        for (int i : order) {
            int best = 0;
            for (int x = 1; x < X; ++x)
                if (load[x] < load[best]) best = x;
            owner[i] = best;
            load[best] += (int64_t)jobs[i].w * jobs[i].h;
        }
        int s = 0;
        b->ntask = 0;
        for (int x = 0; x < X; ++x) {
            b->qseg[x] = s;
            int task = 0;
            for (int pass = 0; pass < 2; ++pass) {
                for (int i = 0; i < n; ++i) {
                    if (owner[i] != x) continue;
                    for (int ph = 2 * pass; ph < 2 * pass + 2; ++ph) {
                        BatchSeg sg;
                        sg.frame = i;
                        sg.phase = ph;
                        sg.first = task;
                        sg.ntask = pstereo::batch_tasks(b->h_frames[i], ph, &sg.items, &sg.gx);
                        b->h_need[4 * i + ph] = sg.ntask;
                        b->h_segs[s++] = sg;
                        task += sg.ntask;
                    }
                }
            }
            b->qntask[x] = task;
            b->ntask += task;
        }
        b->qseg[X] = s;
        b->grid = b->tune.fused_grid > 0 ? b->tune.fused_grid : b->cus;
        if ((e = hipMemcpyAsync(b->d_frames, b->h_frames, sizeof(FrameDesc) * n, hipMemcpyHostToDevice, st)) != hipSuccess ||
            (e = hipMemcpyAsync(b->d_segs, b->h_segs, sizeof(BatchSeg) * 4 * n, hipMemcpyHostToDevice, st)) != hipSuccess ||
            (e = hipMemcpyAsync(b->d_need, b->h_need, sizeof(int) * 4 * n, hipMemcpyHostToDevice, st)) != hipSuccess ||
            (e = hipEventRecord(b->staged, st)) != hipSuccess)
            return bfail(b, PSTEREO_E_DEVICE, "table upload: %s", hipGetErrorString(e));
    } else {
        // staged form: per-stage first-workgroup tables and the warp shapes
        pstereo::StagedPlan& pl = b->plan;
        pl = pstereo::StagedPlan();
        pl.n = n;
        pl.r = p.cbf_radius;
        pl.k2 = p.block_size == 2;
        pl.warp_rows = b->tune.warp_rows;
        pl.bs_rows = b->tune.bs_rows;
        int* fb = b->h_first;
        int* fc = b->h_first + (n + 1);
        int nb_max = 1;
        std::vector<int> cls(n);
        for (int i = 0; i < n; ++i) {
            const FrameDesc& f = b->h_frames[i];
            int items, gx;
            fb[i] = pl.tiles_bs;
            (void)pstereo::batch_tasks(f, 0, &items, &gx, pl.bs_rows);  // block-statistics tiles
            pl.tiles_bs += items;
            fc[i] = pl.tiles_cbf;
            (void)pstereo::batch_tasks(f, 2, &items, &gx);  // depth-filter tiles
            pl.tiles_cbf += items;
            nb_max = std::max(nb_max, f.gw * f.gh);
            pstereo::WarpShape ws;
            if (!pstereo::warp_shape_cap(f.w, b->tune.warp_lanes, &ws))
                return bfail(b, PSTEREO_E_UNSUPPORTED, "job %d: width %d too large for the row warp", i, f.w);
            int c = 0;
            while (c < pl.nclass && !(pl.cls_threads[c] == ws.threads && pl.cls_q[c] == ws.quads)) ++c;
            if (c == pl.nclass) {
                if (pl.nclass == pstereo::kMaxWarpClasses) return bfail(b, PSTEREO_E_UNSUPPORTED, "too many row shapes");
                pl.cls_threads[c] = ws.threads;
                pl.cls_q[c] = ws.quads;
                pl.cls_lds[c] = 0;
                ++pl.nclass;
            }
            pl.cls_lds[c] = std::max(pl.cls_lds[c], ws.lds_bytes);
            cls[i] = c;
        }
        fb[n] = pl.tiles_bs;
        fc[n] = pl.tiles_cbf;
        pl.regions_lds = pstereo::regions_lds_bytes(nb_max);
        for (int c = 0; c < pl.nclass; ++c) {
            int* fw = b->h_first + (size_t)(2 + c) * (n + 1);
            int acc = 0;
            for (int i = 0; i < n; ++i) {
                fw[i] = acc;
                if (cls[i] == c) acc += (b->h_frames[i].h + pl.warp_rows - 1) / pl.warp_rows;
            }
            fw[n] = acc;
            pl.cls_rows[c] = acc;
        }
        b->ntask = pl.tiles_bs + n + pl.tiles_cbf;
        if ((e = hipMemcpyAsync(b->d_frames, b->h_frames, sizeof(FrameDesc) * n, hipMemcpyHostToDevice, st)) != hipSuccess ||
            (e = hipMemcpyAsync(b->d_first, b->h_first, sizeof(int) * (2 + pl.nclass) * (n + 1), hipMemcpyHostToDevice,
                                st)) != hipSuccess ||
            (e = hipEventRecord(b->staged, st)) != hipSuccess)
            return bfail(b, PSTEREO_E_DEVICE, "table upload: %s", hipGetErrorString(e));
    }
    b->staged_pending = true;
    b->prepared = true;
    return PSTEREO_OK;
}

size_t job_scratch_bytes(int w, int h, int K) {
    const size_t nb = (size_t)((w + K - 1) / K) * ((h + K - 1) / K);
    const size_t tab = (nb * (4 + 8 + 4) + 255) / 256 * 256;
    return tab + ((size_t)w * h + 255) / 256 * 256;
}

JobScratch job_scratch_carve(uint8_t* base, int w, int h, int K) {
    const size_t nb = (size_t)((w + K - 1) / K) * ((h + K - 1) / K);
    JobScratch s;
    s.binfo = reinterpret_cast<uint2*>(base);
    s.stats = reinterpret_cast<uint32_t*>(base + nb * 8);
    s.labels = reinterpret_cast<int32_t*>(base + nb * 12);
    s.df = base + (nb * 16 + 255) / 256 * 256;
    return s;
}

}  // namespace pstereo

extern "C" {

int pstereo_batch_launch(pstereo_batch* b, void* stream) {
    if (!b) return PSTEREO_E_INVALID;
    b->err.clear();
    if (!b->prepared) return bfail(b, PSTEREO_E_INVALID, "no prepared batch");
    (void)hipSetDevice(b->device);
    BatchDesc bd;
    bd.frames = b->d_frames;
    bd.segs = b->d_segs;
    bd.need = b->d_need;
    bd.ctr = b->d_ctr;
    bd.nframes = b->n;
    for (int x = 0; x <= pstereo::kXcds; ++x) bd.qseg[x] = b->qseg[x];
    for (int x = 0; x < pstereo::kXcds; ++x) bd.qntask[x] = b->qntask[x];
    hipStream_t st = stream ? (hipStream_t)stream : b->stream;
    hipError_t e = b->tune.mode == PSTEREO_BATCH_FUSED ? pstereo::launch_batch(bd, b->r, b->grid, st)
                                                        : pstereo::launch_staged(b->d_frames, b->d_first, b->plan, st);
    if (e != hipSuccess) return bfail(b, PSTEREO_E_DEVICE, "batch launch: %s", hipGetErrorString(e));
    return PSTEREO_OK;
}

int pstereo_batch_run(pstereo_batch* b, const pstereo_job* jobs, int n, const pstereo_params* p) {
    int rc = pstereo_batch_prepare(b, jobs, n, p);
    if (rc != PSTEREO_OK) return rc;
    rc = pstereo_batch_launch(b, nullptr);
    if (rc != PSTEREO_OK) return rc;
    if (p && (p->flags & PSTEREO_SYNC)) {
        if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, PSTEREO_E_DEVICE, "stream synchronize");
        uint32_t aborted = 0;
        if (b->tune.mode == PSTEREO_BATCH_FUSED &&
            hipMemcpy(&aborted, b->d_ctr + pstereo::kXcds + 4 * b->n, sizeof(aborted), hipMemcpyDeviceToHost) != hipSuccess)
            return bfail(b, PSTEREO_E_DEVICE, "abort word read-back");
        if (aborted) return bfail(b, PSTEREO_E_DEVICE, "a dependency wait timed out; outputs are incomplete");
    }
    return PSTEREO_OK;
}

int pstereo_batch_set_tuning(pstereo_batch* b, const pstereo_batch_tuning* t) {
    if (!b || !t) return PSTEREO_E_INVALID;
    b->err.clear();
    if (t->mode != PSTEREO_BATCH_STAGED && t->mode != PSTEREO_BATCH_FUSED)
        return bfail(b, PSTEREO_E_INVALID, "unknown batch mode %d", t->mode);
    if (t->warp_lanes < 64 || t->warp_lanes > 1024 || t->warp_lanes % 64)
        return bfail(b, PSTEREO_E_INVALID, "warp_lanes %d not a multiple of 64 in 64..1024", t->warp_lanes);
    if (t->warp_rows < 1 || t->warp_rows > 8) return bfail(b, PSTEREO_E_INVALID, "warp_rows %d outside 1..8", t->warp_rows);
    if (t->fused_grid < 0 || (t->fused_grid > 0 && t->fused_grid < pstereo::kXcds) || t->fused_grid > 65536)
        return bfail(b, PSTEREO_E_INVALID, "fused_grid %d: 0 or 8..65536 (every XCD serves a queue)", t->fused_grid);
    if (t->bs_rows != 0 && t->bs_rows != 16 && t->bs_rows != 32 && t->bs_rows != 64)
        return bfail(b, PSTEREO_E_INVALID, "bs_rows %d: 0, 16, 32 or 64", t->bs_rows);
    b->tune = *t;
    b->prepared = false;  // the tables depend on the tuning
    return PSTEREO_OK;
}

int pstereo_batch_get_tuning(const pstereo_batch* b, pstereo_batch_tuning* t) {
    if (!b || !t) return PSTEREO_E_INVALID;
    *t = b->tune;
    return PSTEREO_OK;
}

int pstereo_batch_autotune(pstereo_batch* b, const pstereo_job* jobs, int n, const pstereo_params* p, int reps,
                           pstereo_batch_tuning* best, double* best_ms, pstereo_batch_trial* trials, int cap,
                           int* n_trials) {
    if (!b || reps < 1 || reps > 1000 || cap < 0 || (cap > 0 && !trials)) return PSTEREO_E_INVALID;
    // candidates: the staged form over row-workgroup lane caps and rows per
    // workgroup, and the fused form with one workgroup per compute unit;
    // then, if the staged form won, its block-statistics tile heights
    std::vector<pstereo_batch_tuning> cand;
    static const int lanes[4] = {128, 256, 512, 1024};
    static const int rows[3] = {1, 2, 4};
    for (int l : lanes)
        for (int r : rows) cand.push_back({PSTEREO_BATCH_STAGED, l, r, 0, 0});
    cand.push_back({PSTEREO_BATCH_FUSED, 256, 1, 0, 0});
    const pstereo_batch_tuning saved = b->tune;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipSetDevice(b->device);
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        if (e0) (void)hipEventDestroy(e0);
        return bfail(b, PSTEREO_E_DEVICE, "event create");
    }
    double best_t = -1;
    pstereo_batch_tuning best_c = saved;
    int nt = 0, rc = PSTEREO_OK;
    // time one candidate; false once an error ends the search
    auto trial = [&](const pstereo_batch_tuning& c) -> bool {
        b->tune = c;
        int r = pstereo_batch_prepare(b, jobs, n, p);
        if (r == PSTEREO_E_UNSUPPORTED) return true;  // e.g. a width the fused form cannot take
        if (r != PSTEREO_OK) { rc = r; return false; }
        hipStream_t st = b->stream;
        if ((r = pstereo_batch_launch(b, nullptr)) != PSTEREO_OK) { rc = r; return false; }  // warm-up
        if (hipEventRecord(e0, st) != hipSuccess) { rc = bfail(b, PSTEREO_E_DEVICE, "event record"); return false; }
        for (int k = 0; k < reps && r == PSTEREO_OK; ++k) r = pstereo_batch_launch(b, nullptr);
        if (r != PSTEREO_OK) { rc = r; return false; }
        float ms = 0;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = bfail(b, PSTEREO_E_DEVICE, "event timing");
            return false;
        }
        const double t = ms / reps;
        if (nt < cap) {
            trials[nt].tuning = c;
            trials[nt].ms = t;
        }
        ++nt;
        if (best_t < 0 || t < best_t) {
            best_t = t;
            best_c = c;
        }
        return true;
    };
    bool going = true;
    for (size_t ci = 0; ci < cand.size() && going; ++ci) going = trial(cand[ci]);
    if (going && best_t >= 0 && best_c.mode == PSTEREO_BATCH_STAGED) {
        const pstereo_batch_tuning base = best_c;
        for (int h : {16, 32, 64}) {
            pstereo_batch_tuning d = base;
            d.bs_rows = h;
            if (!(going = trial(d))) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (n_trials) *n_trials = nt;
    if (rc != PSTEREO_OK || best_t < 0) {
        b->tune = saved;
        b->prepared = false;
        return rc != PSTEREO_OK ? rc : bfail(b, PSTEREO_E_UNSUPPORTED, "no candidate could run this batch");
    }
    // leave the batch prepared with the winner
    b->tune = best_c;
    rc = pstereo_batch_prepare(b, jobs, n, p);
    if (best) *best = best_c;
    if (best_ms) *best_ms = best_t;
    return rc;
}

int pstereo_synthesize_batch(pstereo_ctx* ctx, const pstereo_job* jobs, int n, const pstereo_params* p) {
    if (!ctx) return PSTEREO_E_INVALID;
    pstereo::ctx_set_error(ctx, "");
    if (!jobs || n < 1 || n > 4096) {
        pstereo::ctx_set_error(ctx, "job count outside 1..4096 or jobs is NULL");
        return PSTEREO_E_INVALID;
    }
    int64_t px = 0;
    for (int i = 0; i < n; ++i) {
        if (jobs[i].w < 1 || jobs[i].h < 1) {
            pstereo::ctx_set_error(ctx, "a job has a non-positive size");
            return PSTEREO_E_INVALID;
        }
        px += (int64_t)jobs[i].w * jobs[i].h;
    }
    pstereo_batch** slot = pstereo::ctx_batch(ctx);
    pstereo_batch* b = *slot;
    if (!b || b->max_jobs < n || b->max_pixels < px) {
        // (re)made for at least this many jobs and pixels; the old object's
        // scratch may still be read by launches in flight on any stream
        if (b) {
            (void)hipSetDevice(b->device);
            (void)hipDeviceSynchronize();
            batch_free(b);
            *slot = nullptr;
        }
        const int jobs_cap = std::max(n, 64);
        const int64_t px_cap = std::max<int64_t>(px, (int64_t)3840 * 2160);
        const int rc = pstereo::batch_create_internal(ctx, jobs_cap, px_cap, true, &b);
        if (rc != PSTEREO_OK) {
            pstereo::ctx_set_error(ctx, "batch scratch allocation failed");
            return rc;
        }
        // the staged form with 512-lane row workgroups of 4 rows, the tuning
        // the autotuner picks for the uneven 720p..8K mix
        b->tune = {PSTEREO_BATCH_STAGED, 512, 4, 0, 0};
        *slot = b;
    }
    const int rc = pstereo_batch_run(b, jobs, n, p);
    if (rc != PSTEREO_OK) pstereo::ctx_set_error(ctx, b->err.c_str());
    return rc;
}

}  // extern "C"
