// C ABI of the pseudo-stereo library: context, argument validation, launch
// sequence of one frame, per-kernel event timing.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pstereo.h"
#include "pstereo_internal.h"

using pstereo::FrameDesc;
using pstereo::WarpShape;

namespace {

constexpr int kProfSets = 4096;
constexpr int kProfEvents = 5;  // before blockstats, after blockstats, after regions, after cbf, after warp

thread_local std::string g_create_error;

}  // namespace

struct pstereo_ctx {
    int device = 0;
    int max_w = 0, max_h = 0;
    hipStream_t stream = nullptr;
    uint32_t* d_stats = nullptr;
    uint2* d_binfo = nullptr;
    int32_t* d_labels = nullptr;
    uint8_t* d_df = nullptr;  // filtered depth, max_w * max_h bytes
    std::string err;
    // last generated-depth call, for pstereo_debug_blocks
    bool have_blocks = false;
    int last_gw = 0, last_gh = 0;
    hipStream_t last_stream = nullptr;
    // profiling ring
    std::vector<hipEvent_t> prof_ev;
    std::vector<uint8_t> prof_has_depth;
    long long prof_head = 0;
};

namespace {

int fail(pstereo_ctx* c, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else g_create_error = buf;
    return code;
}

// A device pointer of this context's GPU, or an error.
int check_device_ptr(pstereo_ctx* c, const void* p, const char* name) {
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, PSTEREO_E_INVALID, "%s is not a device pointer (%s)", name, hipGetErrorString(e));
    }
    if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
        return fail(c, PSTEREO_E_INVALID, "%s is not device memory", name);
    if (a.device != c->device)
        return fail(c, PSTEREO_E_INVALID, "%s lives on device %d, context is on device %d", name, a.device,
                    c->device);
    return PSTEREO_OK;
}

struct Range {
    const uint8_t* p;
    size_t n;
    const char* name;
};

bool overlap(const Range& a, const Range& b) {
    return a.p && b.p && a.p < b.p + b.n && b.p < a.p + a.n;
}

bool legal_block(int K) { return K == 4 || K == 8 || K == 16 || K == 32 || K == 64; }

int auto_block(int w, int h) {
    static const int cand[4] = {8, 16, 32, 64};
    for (int K : cand) {
        const long long gw = (w + K - 1) / K, gh = (h + K - 1) / K;
        if (gw * gh <= PSTEREO_MAX_BLOCKS) return K;
    }
    return -1;
}

}  // namespace

extern "C" {

int pstereo_params_init(pstereo_params* p) {
    if (!p) return PSTEREO_E_INVALID;
    std::memset(p, 0, sizeof *p);
    p->struct_size = sizeof(pstereo_params);
    p->max_disparity = -1;
    p->depth_threshold = 150;
    p->block_size = 0;
    p->edge_thresh = 24;
    p->link_thresh = 24;
    p->cbf_radius = 2;
    return PSTEREO_OK;
}

int pstereo_create(pstereo_ctx** out, int device, int max_w, int max_h) {
    g_create_error.clear();
    if (!out) return fail(nullptr, PSTEREO_E_INVALID, "out is NULL");
    *out = nullptr;
    if (max_w < 1 || max_w > 65535 || max_h < 1 || max_h > 65535)
        return fail(nullptr, PSTEREO_E_INVALID, "max size %dx%d out of range", max_w, max_h);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return fail(nullptr, PSTEREO_E_INVALID, "device %d not available (%d devices)", device, ndev);
    }
    pstereo_ctx* c = new (std::nothrow) pstereo_ctx;
    if (!c) return fail(nullptr, PSTEREO_E_NOMEM, "host allocation failed");
    c->device = device;
    c->max_w = max_w;
    c->max_h = max_h;
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = pstereo::prepare_depth_kernels();
    if (e == hipSuccess) e = pstereo::prepare_render_kernels();
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete c;
        return fail(nullptr, PSTEREO_E_DEVICE, "device setup failed: %s", hipGetErrorString(e));
    }
    const size_t nb = PSTEREO_MAX_BLOCKS;
    if (hipMalloc(&c->d_stats, nb * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&c->d_binfo, nb * sizeof(uint2)) != hipSuccess ||
        hipMalloc(&c->d_labels, nb * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&c->d_df, (size_t)max_w * max_h) != hipSuccess) {
        (void)hipGetLastError();
        pstereo_destroy(c);
        return fail(nullptr, PSTEREO_E_NOMEM, "scratch allocation failed");
    }
    *out = c;
    return PSTEREO_OK;
}

int pstereo_destroy(pstereo_ctx* c) {
    if (!c) return PSTEREO_OK;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t ev : c->prof_ev) (void)hipEventDestroy(ev);
    (void)hipFree(c->d_stats);
    (void)hipFree(c->d_binfo);
    (void)hipFree(c->d_labels);
    (void)hipFree(c->d_df);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    (void)hipGetLastError();
    delete c;
    return PSTEREO_OK;
}

const char* pstereo_last_error(const pstereo_ctx* c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

int pstereo_synthesize(pstereo_ctx* c, const uint8_t* frame, int w, int h, const pstereo_params* pin,
                       uint8_t* out_l, uint8_t* out_r, uint8_t* out_a) {
    if (!c) return PSTEREO_E_INVALID;
    c->err.clear();
    pstereo_params p;
    pstereo_params_init(&p);
    if (pin) {
        if (pin->struct_size != sizeof(pstereo_params))
            return fail(c, PSTEREO_E_INVALID, "params.struct_size %u != %zu", pin->struct_size,
                        sizeof(pstereo_params));
        p = *pin;
    }
    if (!frame) return fail(c, PSTEREO_E_INVALID, "frame is NULL");
    if (w < 1 || h < 1 || w > c->max_w || h > c->max_h)
        return fail(c, PSTEREO_E_INVALID, "frame %dx%d outside 1..%d x 1..%d", w, h, c->max_w, c->max_h);
    const int B = p.max_disparity < 0 ? (2 * w + 50) / 100 : p.max_disparity;
    if (p.max_disparity < -1 || B > 255) return fail(c, PSTEREO_E_INVALID, "max_disparity %d outside -1..255", p.max_disparity);
    if (p.depth_threshold < -1 || p.depth_threshold > 255)
        return fail(c, PSTEREO_E_INVALID, "depth_threshold %d outside -1..255", p.depth_threshold);
    if (p.cbf_radius < 0 || p.cbf_radius > 3) return fail(c, PSTEREO_E_INVALID, "cbf_radius %d outside 0..3", p.cbf_radius);
    if (p.edge_thresh < 0 || p.edge_thresh > 255) return fail(c, PSTEREO_E_INVALID, "edge_thresh %d outside 0..255", p.edge_thresh);
    if (p.link_thresh < 0 || p.link_thresh > 765) return fail(c, PSTEREO_E_INVALID, "link_thresh %d outside 0..765", p.link_thresh);
    const bool ext = (p.flags & PSTEREO_DEPTH_EXTERNAL) != 0;
    if (ext && !p.depth_in) return fail(c, PSTEREO_E_INVALID, "PSTEREO_DEPTH_EXTERNAL without depth_in");
    const int K = p.block_size ? p.block_size : auto_block(w, h);
    if (!legal_block(K)) return fail(c, PSTEREO_E_INVALID, "block_size %d not in {4,8,16,32,64}", p.block_size);
    const int gw = (w + K - 1) / K, gh = (h + K - 1) / K;
    if (!ext && (long long)gw * gh > PSTEREO_MAX_BLOCKS)
        return fail(c, PSTEREO_E_INVALID, "%dx%d blocks of %d px exceed %d", gw, gh, K, PSTEREO_MAX_BLOCKS);

    int rc;
    if ((rc = check_device_ptr(c, frame, "frame")) != PSTEREO_OK) return rc;
    if (out_l && (rc = check_device_ptr(c, out_l, "out_left")) != PSTEREO_OK) return rc;
    if (out_r && (rc = check_device_ptr(c, out_r, "out_right")) != PSTEREO_OK) return rc;
    if (out_a && (rc = check_device_ptr(c, out_a, "out_anaglyph")) != PSTEREO_OK) return rc;
    if (ext && (rc = check_device_ptr(c, p.depth_in, "depth_in")) != PSTEREO_OK) return rc;
    if (p.out_depth && (rc = check_device_ptr(c, p.out_depth, "out_depth")) != PSTEREO_OK) return rc;
    if (p.out_depth_raw && (rc = check_device_ptr(c, p.out_depth_raw, "out_depth_raw")) != PSTEREO_OK) return rc;

    const size_t img = (size_t)w * h * 3, pl = (size_t)w * h;
    const Range rin[2] = {{frame, img, "frame"}, {ext ? p.depth_in : nullptr, pl, "depth_in"}};
    const Range rout[5] = {{out_l, img, "out_left"}, {out_r, img, "out_right"}, {out_a, img, "out_anaglyph"},
                           {p.out_depth, pl, "out_depth"}, {p.out_depth_raw, pl, "out_depth_raw"}};
    for (int i = 0; i < 5; ++i) {
        for (int j = 0; j < 2; ++j)
            if (overlap(rout[i], rin[j])) return fail(c, PSTEREO_E_ALIAS, "%s overlaps %s", rout[i].name, rin[j].name);
        for (int j = i + 1; j < 5; ++j)
            if (overlap(rout[i], rout[j])) return fail(c, PSTEREO_E_ALIAS, "%s overlaps %s", rout[i].name, rout[j].name);
    }

    WarpShape ws;
    if (!pstereo::warp_shape(w, &ws))
        return fail(c, PSTEREO_E_UNSUPPORTED, "width %d exceeds the warp kernel's LDS budget", w);

    FrameDesc f{};
    f.frame = frame;
    f.out_l = out_l;
    f.out_r = out_r;
    f.out_a = out_a;
    f.depth_in = ext ? p.depth_in : nullptr;
    f.out_df = p.out_depth;
    f.out_d0 = p.out_depth_raw;
    f.stats = c->d_stats;
    f.binfo = c->d_binfo;
    f.labels = c->d_labels;
    f.df = c->d_df;
    f.w = w;
    f.h = h;
    f.K = K;
    f.gw = gw;
    f.gh = gh;
    f.B = B;
    f.T = p.depth_threshold;
    f.g = p.edge_thresh;
    f.tau = p.link_thresh;
    f.r = p.cbf_radius;
    uintptr_t al = (uintptr_t)frame | (uintptr_t)out_l | (uintptr_t)out_r | (uintptr_t)out_a;
    f.aligned = (w % 4 == 0) && (al % 4 == 0);

    hipStream_t s = p.stream ? (hipStream_t)p.stream : c->stream;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return fail(c, PSTEREO_E_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));

    const bool prof = (p.flags & PSTEREO_PROFILE) != 0;
    hipEvent_t* ev = nullptr;
    if (prof) {
        if (c->prof_ev.empty()) {
            c->prof_ev.resize((size_t)kProfSets * kProfEvents, nullptr);
            c->prof_has_depth.resize(kProfSets, 0);
            for (auto& x : c->prof_ev)
                if ((e = hipEventCreate(&x)) != hipSuccess)
                    return fail(c, PSTEREO_E_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
        }
        const int slot = (int)(c->prof_head % kProfSets);
        ev = &c->prof_ev[(size_t)slot * kProfEvents];
        c->prof_has_depth[slot] = !ext;
        c->prof_head++;
    }

    if (prof) (void)hipEventRecord(ev[0], s);
    if (!ext) {
        if ((e = pstereo::launch_blockstats(f, s)) != hipSuccess)
            return fail(c, PSTEREO_E_DEVICE, "block statistics launch: %s", hipGetErrorString(e));
        if (prof) (void)hipEventRecord(ev[1], s);
        if ((e = pstereo::launch_regions(f, s)) != hipSuccess)
            return fail(c, PSTEREO_E_DEVICE, "region grouping launch: %s", hipGetErrorString(e));
        if (prof) (void)hipEventRecord(ev[2], s);
    } else if (prof) {
        (void)hipEventRecord(ev[1], s);
        (void)hipEventRecord(ev[2], s);
    }
    if ((e = pstereo::launch_cbf(f, s)) != hipSuccess)
        return fail(c, PSTEREO_E_DEVICE, "depth filter launch: %s", hipGetErrorString(e));
    if (prof) (void)hipEventRecord(ev[3], s);
    if ((e = pstereo::launch_warp(f, ws, s)) != hipSuccess)
        return fail(c, PSTEREO_E_DEVICE, "warp launch: %s", hipGetErrorString(e));
    if (prof) (void)hipEventRecord(ev[4], s);
    if (!ext) {
        c->have_blocks = true;
        c->last_gw = gw;
        c->last_gh = gh;
        c->last_stream = s;
    }
    if (p.flags & PSTEREO_SYNC) {
        if ((e = hipStreamSynchronize(s)) != hipSuccess)
            return fail(c, PSTEREO_E_DEVICE, "stream synchronize: %s", hipGetErrorString(e));
    }
    return PSTEREO_OK;
}

int pstereo_debug_blocks(pstereo_ctx* c, uint32_t* stats, int32_t* labels, uint8_t* dblk, int cap, int* gw,
                         int* gh) {
    if (!c) return PSTEREO_E_INVALID;
    c->err.clear();
    if (!c->have_blocks) return fail(c, PSTEREO_E_INVALID, "no generated-depth synthesis yet");
    const int nb = c->last_gw * c->last_gh;
    if (gw) *gw = c->last_gw;
    if (gh) *gh = c->last_gh;
    if (cap < nb) return fail(c, PSTEREO_E_INVALID, "capacity %d < %d blocks", cap, nb);
    (void)hipSetDevice(c->device);
    hipError_t e = hipStreamSynchronize(c->last_stream);
    if (e != hipSuccess) return fail(c, PSTEREO_E_DEVICE, "stream synchronize: %s", hipGetErrorString(e));
    std::vector<uint2> bi(nb);
    if ((e = hipMemcpy(bi.data(), c->d_binfo, nb * sizeof(uint2), hipMemcpyDeviceToHost)) != hipSuccess)
        return fail(c, PSTEREO_E_DEVICE, "copy: %s", hipGetErrorString(e));
    if (labels && (e = hipMemcpy(labels, c->d_labels, nb * sizeof(int32_t), hipMemcpyDeviceToHost)) != hipSuccess)
        return fail(c, PSTEREO_E_DEVICE, "copy: %s", hipGetErrorString(e));
    for (int i = 0; i < nb; ++i) {
        if (stats) stats[i] = bi[i].x;
        if (dblk) dblk[i] = (uint8_t)bi[i].y;
    }
    return PSTEREO_OK;
}

int pstereo_profile_collect(pstereo_ctx* c, double ms_sum[4], int* count, double* per_call_ms, int cap) {
    if (!c || !ms_sum || !count) return PSTEREO_E_INVALID;
    c->err.clear();
    ms_sum[0] = ms_sum[1] = ms_sum[2] = ms_sum[3] = 0.0;
    *count = 0;
    if (c->prof_head == 0) return PSTEREO_OK;
    (void)hipSetDevice(c->device);
    const long long n = c->prof_head < kProfSets ? c->prof_head : kProfSets;
    for (long long k = c->prof_head - n; k < c->prof_head; ++k) {
        const int slot = (int)(k % kProfSets);
        hipEvent_t* ev = &c->prof_ev[(size_t)slot * kProfEvents];
        hipError_t e = hipEventSynchronize(ev[4]);
        if (e != hipSuccess) return fail(c, PSTEREO_E_DEVICE, "event synchronize: %s", hipGetErrorString(e));
        float a = 0.f, b = 0.f, d = 0.f, q = 0.f;
        if (c->prof_has_depth[slot]) {
            (void)hipEventElapsedTime(&a, ev[0], ev[1]);
            (void)hipEventElapsedTime(&b, ev[1], ev[2]);
        }
        (void)hipEventElapsedTime(&d, ev[2], ev[3]);
        (void)hipEventElapsedTime(&q, ev[3], ev[4]);
        ms_sum[0] += a;
        ms_sum[1] += b;
        ms_sum[2] += d;
        ms_sum[3] += q;
        if (per_call_ms && *count < cap) {
            float tot = 0.f;
            (void)hipEventElapsedTime(&tot, ev[0], ev[4]);
            per_call_ms[*count] = tot;
        }
        ++*count;
    }
    c->prof_head = 0;
    return PSTEREO_OK;
}

}  // extern "C"
