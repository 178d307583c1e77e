// C ABI of the pseudo-stereo library: context, argument validation, launch
// sequence of one frame, per-kernel event timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pstereo.h"
#include "pstereo_internal.h"

using pstereo::FrameDesc;
using pstereo::WarpShape;

namespace {

// Profiling ring: per profiled call, a start and a stop event per kernel.
constexpr int kProfSets = 4096;
constexpr int kMaxKernels = 6;
constexpr int kProfEvents = 2 * kMaxKernels;

// message of the last failed create or context-free call on this thread
thread_local char g_create_error[512];

// The per-frame tables of the depth-map stages (block statistics, region
// grouping) that the filter reads: one set per frame in flight.
struct BlockScratch {
    uint8_t* mem = nullptr;  // one allocation, carved below
    uint32_t* stats = nullptr;
    uint2* binfo = nullptr;
    int32_t* labels = nullptr;
    uint2* rent = nullptr;
    uint32_t* rrow = nullptr;
    uint32_t* rfin = nullptr;
    uint2* rbnd = nullptr;
    uint32_t* rctl = nullptr;
};

constexpr size_t align256(size_t n) { return (n + 255) / 256 * 256; }

// Byte sizes of the tables of one set, in carving order: statistics, block
// info, labels, slot entries, slot rows, slot finals, boundary candidates,
// control words.
constexpr size_t kBlkTableBytes[8] = {
    PSTEREO_MAX_BLOCKS * 4, PSTEREO_MAX_BLOCKS * 8, PSTEREO_MAX_BLOCKS * 4, pstereo::kRegionSlots * 8,
    pstereo::kRegionSlots * 4, pstereo::kRegionSlots * 4, pstereo::kBoundSlots * 8, 4 * 4};

constexpr size_t block_scratch_bytes() {
    size_t tot = 0;
    for (size_t b : kBlkTableBytes) tot += align256(b);
    return tot;
}

// Lay one set out in `mem` (block_scratch_bytes() bytes, 256-byte aligned).
void block_scratch_carve(BlockScratch& b, uint8_t* mem) {
    size_t off[8], tot = 0;
    for (int i = 0; i < 8; ++i) {
        off[i] = tot;
        tot += align256(kBlkTableBytes[i]);
    }
    b.mem = mem;
    b.stats = reinterpret_cast<uint32_t*>(mem + off[0]);
    b.binfo = reinterpret_cast<uint2*>(mem + off[1]);
    b.labels = reinterpret_cast<int32_t*>(mem + off[2]);
    b.rent = reinterpret_cast<uint2*>(mem + off[3]);
    b.rrow = reinterpret_cast<uint32_t*>(mem + off[4]);
    b.rfin = reinterpret_cast<uint32_t*>(mem + off[5]);
    b.rbnd = reinterpret_cast<uint2*>(mem + off[6]);
    b.rctl = reinterpret_cast<uint32_t*>(mem + off[7]);
}

// Allocate and carve one set; the control words start at zero (the merge
// kernel leaves them zero after each frame).
hipError_t block_scratch_alloc(BlockScratch& b) {
    uint8_t* mem = nullptr;
    hipError_t e = hipMalloc(&mem, block_scratch_bytes());
    if (e != hipSuccess) return e;
    block_scratch_carve(b, mem);
    return hipMemset(b.rctl, 0, 4 * sizeof(uint32_t));
}

// One filtered-depth image, rounded up so that the second one stays aligned.
size_t df_image_bytes(int w, int h) { return align256((size_t)w * h); }

}  // namespace

struct pstereo_ctx {
    int device = 0;
    int max_w = 0, max_h = 0;
    // block tables: set 0 for every call; pipelined calls alternate sets 0
    // and 1 so that one frame's depth-map stages can run while the previous
    // frame's filter still reads its set
    BlockScratch blk[2];
    uint8_t* d_df = nullptr;  // filtered depth, max_w * max_h bytes
    // second filtered-depth image (three-stage pipelined calls alternate the
    // two), in the same allocation
    uint8_t* d_df2 = nullptr;
    // pipelined calls (PSTEREO_PIPELINE): the depth-map stages go on `side`;
    // three-stage calls (PSTEREO_PIPELINE_DEEP) put the filter on `mid`
    hipStream_t side = nullptr;
    hipStream_t mid = nullptr;
    // ev_before: the caller's stream at the start of a pipelined call with no
    // pipelined call before it on that stream; pipelined video: the video's
    // stream before the previous frame
    hipEvent_t ev_before = nullptr;
    // pipelined calls, call numbers: [0] the last call whose depth map is
    // done, [1] the last call whose depth filter has started; three-stage
    // calls also [2] the last call whose filter is done, [3] the last call
    // whose warp has started
    unsigned long long* d_sig = nullptr;
    bool pipe_valid = false;  // the previous pipelined call was on pipe_stream and its launches all went out
    bool pipe_deep = false;   // the previous pipelined call was a three-stage one
    bool pipe_drained = false;  // no kernel of an earlier pipelined call is still to store a mark
    // the caller's stream the context's streams were last checked against
    // (and whether for three stages), and the check's probe number
    bool overlap_checked = false;
    bool overlap_deep = false;
    hipStream_t overlap_stream = nullptr;
    unsigned long long probe_token = 0;
    hipStream_t pipe_stream = nullptr;
    long long pipe_n = 0;
    // block-iterative inpainting scratch, allocated on first use
    uint32_t* d_ipc = nullptr;
    uint16_t* d_ipt = nullptr;
    uint32_t* d_ipn = nullptr;
    uint32_t* h_ipn = nullptr;  // pinned read-back of one sweep counter
    pstereo_batch* batch = nullptr;  // pstereo_synthesize_batch's batch object, made on first use
    char err[512] = {0};  // message of the last failure
    // last generated-depth call, for pstereo_debug_blocks
    bool have_blocks = false;
    int last_gw = 0, last_gh = 0;
    hipStream_t last_stream = nullptr;
    FrameDesc last_fd{};         // descriptor of the last generated-depth frame
    bool blocks_final = false;   // its per-block labels and depths are final
    // profiling ring: events of kProfSets calls; per call the kernel count
    // and each kernel's stage
    std::vector<hipEvent_t> prof_ev;
    std::vector<int8_t> prof_stage;  // [kProfSets][kMaxKernels], -1 past the last kernel
    long long prof_head = 0;
};

namespace {

// 1 if kernels on streams a and b ran at the same time, 0 if one ran after
// the other, -1 on a HIP error.  Both streams are drained first; the probe
// uses context words 4 and 5.
int streams_overlap(pstereo_ctx* c, hipStream_t a, hipStream_t b) {
    unsigned long long res = 0;
    const unsigned long long token = ++c->probe_token;
    if (hipStreamSynchronize(a) != hipSuccess || hipStreamSynchronize(b) != hipSuccess ||
        pstereo::launch_probe(c->d_sig + 4, token, a, b) != hipSuccess || hipStreamSynchronize(a) != hipSuccess ||
        hipStreamSynchronize(b) != hipSuccess ||
        hipMemcpy(&res, c->d_sig + 5, sizeof res, hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    return res == 1 ? 1 : 0;
}

// Pipelined calls overlap only if the context's second stream (and, for
// three stages, its third) runs beside the caller's stream and beside each
// other.  HIP maps streams onto a few hardware queues (GPU_MAX_HW_QUEUES),
// fixed when a stream is created; streams that share a queue run their
// kernels one after the other.  So the first pipelined call on a caller
// stream probes each pair and replaces a context stream that does not
// overlap by a newly created one -- the rejected one stays alive meanwhile,
// so that the new one is placed on another queue -- a few times at most.
// Where none is found the calls stay correct, only not overlapped.  Drains
// every stream involved.
void ensure_overlap(pstereo_ctx* c, hipStream_t s, bool deep) {
    if (c->overlap_checked && c->overlap_stream == s && (c->overlap_deep || !deep)) return;
    std::vector<hipStream_t> rejected;
    for (int attempt = 0; attempt < 8; ++attempt) {
        hipStream_t* bad = nullptr;
        if (streams_overlap(c, c->side, s) == 0) bad = &c->side;
        else if (deep && streams_overlap(c, c->mid, s) == 0) bad = &c->mid;
        else if (deep && streams_overlap(c, c->mid, c->side) == 0) bad = &c->mid;
        if (!bad) break;
        hipStream_t fresh = nullptr;
        if (hipStreamCreateWithFlags(&fresh, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            break;
        }
        rejected.push_back(*bad);
        *bad = fresh;
    }
    for (hipStream_t r : rejected) (void)hipStreamDestroy(r);
    c->overlap_checked = true;
    c->overlap_stream = s;
    c->overlap_deep = deep;
}

}  // namespace

namespace pstereo {
int ctx_device(const pstereo_ctx* c) { return c->device; }
pstereo_batch** ctx_batch(pstereo_ctx* c) { return &c->batch; }
void ctx_set_error(pstereo_ctx* c, const char* msg) { snprintf(c->err, sizeof c->err, "%s", msg ? msg : ""); }
}  // namespace pstereo

namespace {

int fail(pstereo_ctx* c, int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    if (c) vsnprintf(c->err, sizeof c->err, fmt, ap);
    else vsnprintf(g_create_error, sizeof g_create_error, fmt, ap);
    va_end(ap);
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

bool legal_block(int K) { return K == 2 || K == 4 || K == 8 || K == 16 || K == 32 || K == 64; }

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
    g_create_error[0] = '\0';
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
    if (e != hipSuccess) {
        delete c;
        return fail(nullptr, PSTEREO_E_DEVICE, "device setup failed: %s", hipGetErrorString(e));
    }
    if (block_scratch_alloc(c->blk[0]) != hipSuccess || block_scratch_alloc(c->blk[1]) != hipSuccess ||
        hipMalloc(&c->d_df, 2 * df_image_bytes(max_w, max_h)) != hipSuccess || hipMalloc(&c->d_sig, 64) != hipSuccess ||
        hipMemset(c->d_sig, 0, 64) != hipSuccess) {
        (void)hipGetLastError();
        pstereo_destroy(c);
        return fail(nullptr, PSTEREO_E_NOMEM, "scratch allocation failed");
    }
    c->d_df2 = c->d_df + df_image_bytes(max_w, max_h);
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->mid, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_before, hipEventDisableTiming) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        pstereo_destroy(c);
        return fail(nullptr, PSTEREO_E_DEVICE, "stream or event creation failed");
    }
    *out = c;
    return PSTEREO_OK;
}

int pstereo_destroy(pstereo_ctx* c) {
    if (!c) return PSTEREO_OK;
    (void)hipSetDevice(c->device);
    // the context's work may sit on any stream of the caller's: wait for the
    // device before its scratch goes
    (void)hipDeviceSynchronize();
    if (c->batch) (void)pstereo_batch_destroy(c->batch);
    for (hipEvent_t ev : c->prof_ev) (void)hipEventDestroy(ev);
    for (BlockScratch& b : c->blk) (void)hipFree(b.mem);
    (void)hipFree(c->d_df);
    (void)hipFree(c->d_sig);
    if (c->ev_before) (void)hipEventDestroy(c->ev_before);
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->mid) (void)hipStreamDestroy(c->mid);
    (void)hipFree(c->d_ipc);
    (void)hipFree(c->d_ipt);
    (void)hipFree(c->d_ipn);
    if (c->h_ipn) (void)hipHostFree(c->h_ipn);
    (void)hipGetLastError();
    delete c;
    return PSTEREO_OK;
}

const char* pstereo_last_error(const pstereo_ctx* c) {
    return c ? c->err : g_create_error;
}

}  // extern "C"

namespace {

// Validate one synthesis request and build its frame descriptor.  Returns a
// status code; on success *f, *ws and *stream are filled.
int build_desc(pstereo_ctx* c, const uint8_t* frame, int w, int h, const pstereo_params* pin, uint8_t* out_l,
               uint8_t* out_r, uint8_t* out_a, FrameDesc* fd, WarpShape* ws, hipStream_t* stream, uint32_t* flags,
               bool check_ptrs = true) {
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
    if (!legal_block(K)) return fail(c, PSTEREO_E_INVALID, "block_size %d not in {2,4,8,16,32,64}", p.block_size);
    const int gw = (w + K - 1) / K, gh = (h + K - 1) / K;
    if (!ext && (long long)gw * gh > PSTEREO_MAX_BLOCKS)
        return fail(c, PSTEREO_E_INVALID, "%dx%d blocks of %d px exceed %d", gw, gh, K, PSTEREO_MAX_BLOCKS);

    int rc;
    if (check_ptrs && (rc = check_device_ptr(c, frame, "frame")) != PSTEREO_OK) return rc;
    if (check_ptrs) {
        if (out_l && (rc = check_device_ptr(c, out_l, "out_left")) != PSTEREO_OK) return rc;
        if (out_r && (rc = check_device_ptr(c, out_r, "out_right")) != PSTEREO_OK) return rc;
        if (out_a && (rc = check_device_ptr(c, out_a, "out_anaglyph")) != PSTEREO_OK) return rc;
        if (ext && (rc = check_device_ptr(c, p.depth_in, "depth_in")) != PSTEREO_OK) return rc;
        if (p.out_depth && (rc = check_device_ptr(c, p.out_depth, "out_depth")) != PSTEREO_OK) return rc;
        if (p.out_depth_raw && (rc = check_device_ptr(c, p.out_depth_raw, "out_depth_raw")) != PSTEREO_OK) return rc;
        if (p.out_hsbs && (rc = check_device_ptr(c, p.out_hsbs, "out_hsbs")) != PSTEREO_OK) return rc;
    }

    const size_t img = (size_t)w * h * 3, pl = (size_t)w * h;
    const Range rin[2] = {{frame, img, "frame"}, {ext ? p.depth_in : nullptr, pl, "depth_in"}};
    const Range rout[6] = {{out_l, img, "out_left"}, {out_r, img, "out_right"}, {out_a, img, "out_anaglyph"},
                           {p.out_depth, pl, "out_depth"}, {p.out_depth_raw, pl, "out_depth_raw"},
                           {p.out_hsbs, img, "out_hsbs"}};
    for (int i = 0; check_ptrs && i < 6; ++i) {
        for (int j = 0; j < 2; ++j)
            if (overlap(rout[i], rin[j])) return fail(c, PSTEREO_E_ALIAS, "%s overlaps %s", rout[i].name, rin[j].name);
        for (int j = i + 1; j < 6; ++j)
            if (overlap(rout[i], rout[j])) return fail(c, PSTEREO_E_ALIAS, "%s overlaps %s", rout[i].name, rout[j].name);
    }
    const bool gather = (p.flags & PSTEREO_WARP_GATHER) != 0;
    if (gather && (p.flags & PSTEREO_INPAINT_BLOCKS))
        return fail(c, PSTEREO_E_INVALID, "PSTEREO_WARP_GATHER leaves no holes to inpaint");
    if (!gather && !pstereo::warp_shape(w, ws))
        return fail(c, PSTEREO_E_UNSUPPORTED, "width %d exceeds the warp kernel's LDS budget", w);
    if (gather && !pstereo::gather_fits(w))
        return fail(c, PSTEREO_E_UNSUPPORTED, "width %d exceeds the gather kernel's LDS budget", w);

    FrameDesc f{};
    f.frame = frame;
    f.out_l = out_l;
    f.out_r = out_r;
    f.out_a = out_a;
    f.depth_in = ext ? p.depth_in : nullptr;
    f.out_df = p.out_depth;
    f.out_d0 = p.out_depth_raw;
    f.out_h = p.out_hsbs;
    const BlockScratch& bs = c->blk[0];
    f.stats = bs.stats;
    f.binfo = bs.binfo;
    f.labels = bs.labels;
    f.df = c->d_df;
    f.rent = bs.rent;
    f.rrow = bs.rrow;
    f.rfin = bs.rfin;
    f.rbnd = bs.rbnd;
    f.rctl = bs.rctl;
    f.rstrip = pstereo::strip_rows(gw);
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
    const uintptr_t al = (uintptr_t)frame | (uintptr_t)out_l | (uintptr_t)out_r | (uintptr_t)out_a;
    f.aligned = (w % 4 == 0) && (al % 4 == 0);
    f.gather = gather ? 1 : 0;
    *fd = f;
    *stream = (hipStream_t)p.stream;  // NULL: the HIP null stream
    *flags = p.flags;
    return PSTEREO_OK;
}

// The launch sequence of one frame (block statistics and region grouping
// only with a generated depth map).
constexpr int kMaxSpecs = 6;
static_assert(kMaxSpecs <= kMaxKernels, "profiling ring holds every kernel of a call");

// stage[i]: which of the four profiled stages kernel i belongs to (block
// statistics, region grouping, depth filter, warp)
void frame_specs(const FrameDesc& f, const WarpShape& ws, pstereo::LaunchSpec (&ls)[kMaxSpecs], int& n,
                 int (*stage)[kMaxSpecs] = nullptr) {
    n = 0;
    int st[kMaxSpecs];
    if (!f.depth_in) {
        st[n] = 0;
        ls[n++] = pstereo::spec_blockstats(f);
        if (f.rstrip > 0) {
            // the per-block final labels and depths (k_rg_final) are only
            // materialised on request (pstereo_debug_blocks): the depth filter
            // resolves the depths it needs from the slot table
            st[n] = 1;
            ls[n++] = pstereo::spec_rg_strip(f);
            st[n] = 1;
            ls[n++] = pstereo::spec_rg_merge(f);
        } else {
            st[n] = 1;
            ls[n++] = pstereo::spec_regions(f);
        }
    }
    st[n] = 2;
    ls[n++] = pstereo::spec_cbf(f);
    st[n] = 3;
    ls[n++] = f.gather ? pstereo::spec_gather(f) : pstereo::spec_warp(f, ws);
    if (stage)
        for (int i = 0; i < n; ++i) (*stage)[i] = st[i];
}

}  // namespace

extern "C" {

int pstereo_synthesize(pstereo_ctx* c, const uint8_t* frame, int w, int h, const pstereo_params* pin,
                       uint8_t* out_l, uint8_t* out_r, uint8_t* out_a) {
    if (!c) return PSTEREO_E_INVALID;
    c->err[0] = '\0';
    FrameDesc f;
    WarpShape ws{};
    hipStream_t s;
    uint32_t flags;
    int rc = build_desc(c, frame, w, h, pin, out_l, out_r, out_a, &f, &ws, &s, &flags);
    if (rc != PSTEREO_OK) return rc;
    const bool ext = f.depth_in != nullptr;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return fail(c, PSTEREO_E_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));

    const bool inpaint = (flags & PSTEREO_INPAINT_BLOCKS) != 0;
    if (inpaint) {
        if (!c->d_ipc) {
            const size_t px = (size_t)c->max_w * c->max_h;
            if (hipMalloc(&c->d_ipc, 2 * px * sizeof(uint32_t)) != hipSuccess ||
                hipMalloc(&c->d_ipt, 2 * px * sizeof(uint16_t)) != hipSuccess ||
                hipMalloc(&c->d_ipn, (pstereo::kMaxSweeps + 1) * sizeof(uint32_t)) != hipSuccess ||
                hipHostMalloc(&c->h_ipn, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                (void)hipFree(c->d_ipc);
                (void)hipFree(c->d_ipt);
                (void)hipFree(c->d_ipn);
                c->d_ipc = nullptr;
                c->d_ipt = nullptr;
                c->d_ipn = nullptr;
                return fail(c, PSTEREO_E_NOMEM, "inpainting scratch allocation failed");
            }
        }
        f.ipc = c->d_ipc;
        f.ipt = c->d_ipt;
        f.ipn = c->d_ipn;
    }

    const bool prof = (flags & PSTEREO_PROFILE) != 0;
    hipEvent_t* ev = nullptr;
    int8_t* ev_stage = nullptr;
    if (prof) {
        if (c->prof_ev.empty()) {
            // created once, on the first profiled call
            std::vector<hipEvent_t> evs((size_t)kProfSets * kProfEvents, nullptr);
            for (auto& x : evs) {
                if ((e = hipEventCreate(&x)) != hipSuccess) {
                    for (hipEvent_t y : evs)
                        if (y) (void)hipEventDestroy(y);
                    return fail(c, PSTEREO_E_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
                }
            }
            c->prof_ev.swap(evs);
            c->prof_stage.assign((size_t)kProfSets * kMaxKernels, -1);
        }
        const int slot = (int)(c->prof_head % kProfSets);
        ev = &c->prof_ev[(size_t)slot * kProfEvents];
        ev_stage = &c->prof_stage[(size_t)slot * kMaxKernels];
        c->prof_head++;
    }

    // Pipelined call: the depth-map stages (block statistics, region
    // grouping) run on the context's side stream into block-table set
    // pipe_n % 2 once the depth filter of the previous pipelined call has
    // started.  Two stages: that is after everything the caller's stream
    // held before the previous call's filter, when the caller promises the
    // frame was complete; the filter and warp follow on the caller's stream
    // once the depth map is done.  So this frame's depth map is built while
    // the previous frame's filter and warp run, and the set it writes was
    // last read by the filter two calls back, which has finished by then.
    // Three stages: the filter goes on the context's third stream once the
    // depth map is done and the previous call's warp has started (so the warp
    // two calls back, the last reader of the filtered-depth image pipe_n % 2
    // that it writes, has finished); a small kernel after it marks its end,
    // and the warp follows on the caller's stream once that mark is there.
    // Then the depth map of frame i+2, the filter of frame i+1 and the warp
    // of frame i run together, and a filter's start implies the warp's start
    // one call earlier, so everything the caller's stream held before the
    // call two back.  The orderings go through words of the context that a
    // wait-value packet polls (a few us, where an event pair between streams
    // costs ~12 us, and an event recorded on the caller's stream at every
    // call holds that stream up); every wait's releasing kernel was enqueued
    // before the wait, so the orderings also hold where streams share a
    // hardware queue.  The words only grow: each is written by one stream in
    // call order, and the first call on a stream, or in a mode, (whose depth
    // stages wait for its own start, an event) first waits until the last
    // pipelined call's last mark -- its filter's start, or its warp's start
    // for three stages -- is stored, so no kernel of an older call is still
    // to store one.  A call that fails once its work has begun drains the
    // streams and gives up its number.
    const bool deep = (flags & PSTEREO_PIPELINE_DEEP) != 0;
    const bool pipe = (flags & (PSTEREO_PIPELINE | PSTEREO_PIPELINE_DEEP)) && !ext && !inpaint;
    const unsigned long long pv = (unsigned long long)c->pipe_n + 1;  // this call's number
    bool first = false;
    auto pipe_fail = [&](const char* what, hipError_t err) {
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamSynchronize(c->mid);
        (void)hipStreamSynchronize(s);
        (void)hipGetLastError();
        c->pipe_n = (long long)pv;
        c->pipe_drained = true;
        if (prof) ev_stage[0] = -1;  // nothing of this call is collected
        return fail(c, PSTEREO_E_DEVICE, "%s: %s", what, hipGetErrorString(err));
    };
    if (pipe) {
        const BlockScratch& bs = c->blk[c->pipe_n % 2];
        f.stats = bs.stats;
        f.binfo = bs.binfo;
        f.labels = bs.labels;
        f.rent = bs.rent;
        f.rrow = bs.rrow;
        f.rfin = bs.rfin;
        f.rbnd = bs.rbnd;
        f.rctl = bs.rctl;
        if (deep) f.df = c->pipe_n % 2 ? c->d_df2 : c->d_df;
        ensure_overlap(c, s, deep);
        first = !c->pipe_valid || c->pipe_stream != s || c->pipe_deep != deep;
        c->pipe_valid = false;  // until this call's launches are all enqueued
        if (first) {
            if ((c->pipe_n > 0 && !c->pipe_drained &&
                 (e = hipStreamWaitValue64(s, c->d_sig + (c->pipe_deep ? 3 : 1), (unsigned long long)c->pipe_n,
                                           hipStreamWaitValueGte, ~0ull)) != hipSuccess) ||
                (e = hipEventRecord(c->ev_before, s)) != hipSuccess ||
                (e = hipStreamWaitEvent(c->side, c->ev_before, 0)) != hipSuccess)
                return pipe_fail("pipeline ordering", e);
        } else if ((e = hipStreamWaitValue64(c->side, c->d_sig + 1, pv - 1, hipStreamWaitValueGte, ~0ull)) !=
                   hipSuccess) {
            return pipe_fail("pipeline ordering", e);
        }
        f.sig = c->d_sig;
        f.sig_value = pv;
        f.mark = c->d_sig + 1;
        f.mark_value = pv;
        if (deep) {
            f.wmark = c->d_sig + 3;
            f.wmark_value = pv;
        }
    } else {
        c->pipe_valid = false;
    }

    pstereo::LaunchSpec ls[kMaxSpecs];
    int stage[kMaxSpecs];
    int n;
    frame_specs(f, ws, ls, n, &stage);
    static const char* names[4] = {"block statistics", "region grouping", "depth filter", "warp"};
    for (int i = 0; i < n; ++i) {
        hipStream_t si = s;
        if (pipe && stage[i] <= 1) si = c->side;
        if (pipe && stage[i] == 2) {
            if (deep) si = c->mid;
            if ((e = hipStreamWaitValue64(si, c->d_sig, pv, hipStreamWaitValueGte, ~0ull)) != hipSuccess ||
                (deep && !first &&
                 (e = hipStreamWaitValue64(si, c->d_sig + 3, pv - 1, hipStreamWaitValueGte, ~0ull)) != hipSuccess))
                return pipe_fail("pipeline ordering", e);
        }
        if (pipe && deep && stage[i] == 3 &&
            (e = hipStreamWaitValue64(s, c->d_sig + 2, pv, hipStreamWaitValueGte, ~0ull)) != hipSuccess)
            return pipe_fail("pipeline ordering", e);
        // a profiled call takes each kernel's own start and stop times
        e = prof ? pstereo::launch_timed(ls[i], f, si, ev[2 * i], ev[2 * i + 1]) : pstereo::launch(ls[i], f, si);
        if (e == hipSuccess && pipe && deep && stage[i] == 2) e = pstereo::launch_signal(c->d_sig + 2, pv, si);
        if (e != hipSuccess) {
            if (pipe) return pipe_fail(names[stage[i]], e);
            if (prof) ev_stage[0] = -1;  // nothing of this call is collected
            return fail(c, PSTEREO_E_DEVICE, "%s launch: %s", names[stage[i]], hipGetErrorString(e));
        }
    }
    if (pipe) {
        c->pipe_valid = true;
        c->pipe_deep = deep;
        c->pipe_drained = false;
        c->pipe_stream = s;
        c->pipe_n++;
    }
    if (prof)
        for (int i = 0; i < kMaxKernels; ++i) ev_stage[i] = (int8_t)(i < n ? stage[i] : -1);
    if (inpaint) {
        // sweeps in chunks of 8 until one fills nothing (each sweep returns at
        // once after a sweep that filled nothing); a frame still filling
        // pixels at the last allowed sweep is reported, not composed
        if ((e = pstereo::launch_inpaint_reset(f, s)) != hipSuccess)
            return fail(c, PSTEREO_E_DEVICE, "inpainting launch: %s", hipGetErrorString(e));
        bool converged = false;
        for (int sw = 1; sw <= pstereo::kMaxSweeps && !converged; sw += 8) {
            const int last = std::min(sw + 7, pstereo::kMaxSweeps);
            for (int k = sw; k <= last; ++k)
                if ((e = pstereo::launch_inpaint_sweep(f, k, s)) != hipSuccess)
                    return fail(c, PSTEREO_E_DEVICE, "inpainting sweep: %s", hipGetErrorString(e));
            if ((e = hipMemcpyAsync(c->h_ipn, f.ipn + last, sizeof(uint32_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return fail(c, PSTEREO_E_DEVICE, "inpainting convergence check: %s", hipGetErrorString(e));
            converged = *c->h_ipn == 0;
        }
        if (!converged)
            return fail(c, PSTEREO_E_UNSUPPORTED,
                        "block inpainting still filled pixels at its last allowed sweep (%d); outputs not written",
                        pstereo::kMaxSweeps);
        if ((e = pstereo::launch_inpaint_final(f, s)) != hipSuccess)
            return fail(c, PSTEREO_E_DEVICE, "inpainting composition: %s", hipGetErrorString(e));
    }
    if (!ext) {
        c->have_blocks = true;
        c->last_fd = f;
        c->blocks_final = f.rstrip == 0;
        c->last_gw = f.gw;
        c->last_gh = f.gh;
        c->last_stream = s;
    }
    if (flags & PSTEREO_SYNC) {
        if ((e = hipStreamSynchronize(s)) != hipSuccess)
            return fail(c, PSTEREO_E_DEVICE, "stream synchronize: %s", hipGetErrorString(e));
    }
    return PSTEREO_OK;
}

int pstereo_debug_blocks(pstereo_ctx* c, uint32_t* stats, int32_t* labels, uint8_t* dblk, int cap, int* gw,
                         int* gh) {
    if (!c) return PSTEREO_E_INVALID;
    c->err[0] = '\0';
    if (!c->have_blocks) return fail(c, PSTEREO_E_INVALID, "no generated-depth synthesis yet");
    const int nb = c->last_gw * c->last_gh;
    if (gw) *gw = c->last_gw;
    if (gh) *gh = c->last_gh;
    if (cap < nb) return fail(c, PSTEREO_E_INVALID, "capacity %d < %d blocks", cap, nb);
    (void)hipSetDevice(c->device);
    c->pipe_valid = false;  // the next pipelined call waits for this one
    hipError_t e;
    if (!c->blocks_final) {
        // turn the blocks' slots into final labels and depths
        if ((e = pstereo::launch(pstereo::spec_rg_final(c->last_fd), c->last_fd, c->last_stream)) != hipSuccess)
            return fail(c, PSTEREO_E_DEVICE, "block resolution launch: %s", hipGetErrorString(e));
        c->blocks_final = true;
    }
    e = hipStreamSynchronize(c->last_stream);
    if (e != hipSuccess) return fail(c, PSTEREO_E_DEVICE, "stream synchronize: %s", hipGetErrorString(e));
    std::vector<uint2> bi(nb);
    if ((e = hipMemcpy(bi.data(), c->last_fd.binfo, nb * sizeof(uint2), hipMemcpyDeviceToHost)) != hipSuccess)
        return fail(c, PSTEREO_E_DEVICE, "copy: %s", hipGetErrorString(e));
    if (labels && (e = hipMemcpy(labels, c->last_fd.labels, nb * sizeof(int32_t), hipMemcpyDeviceToHost)) != hipSuccess)
        return fail(c, PSTEREO_E_DEVICE, "copy: %s", hipGetErrorString(e));
    for (int i = 0; i < nb; ++i) {
        if (stats) stats[i] = bi[i].x;
        if (dblk) dblk[i] = (uint8_t)bi[i].y;
    }
    return PSTEREO_OK;
}

int pstereo_profile_collect(pstereo_ctx* c, double ms_sum[4], int* count, double* per_call_ms, int cap) {
    if (!c || !ms_sum || !count) return PSTEREO_E_INVALID;
    c->err[0] = '\0';
    ms_sum[0] = ms_sum[1] = ms_sum[2] = ms_sum[3] = 0.0;
    *count = 0;
    if (c->prof_head == 0) return PSTEREO_OK;
    (void)hipSetDevice(c->device);
    const long long n = c->prof_head < kProfSets ? c->prof_head : kProfSets;
    for (long long k = c->prof_head - n; k < c->prof_head; ++k) {
        const int slot = (int)(k % kProfSets);
        hipEvent_t* ev = &c->prof_ev[(size_t)slot * kProfEvents];
        const int8_t* st = &c->prof_stage[(size_t)slot * kMaxKernels];
        int nk = 0;
        while (nk < kMaxKernels && st[nk] >= 0) ++nk;
        if (nk == 0) continue;  // a call whose launch failed
        hipError_t e = hipEventSynchronize(ev[2 * nk - 1]);
        if (e != hipSuccess) return fail(c, PSTEREO_E_DEVICE, "event synchronize: %s", hipGetErrorString(e));
        // a stage runs from its first kernel's start to its last kernel's stop
        for (int i = 0; i < nk;) {
            int j = i;
            while (j + 1 < nk && st[j + 1] == st[i]) ++j;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev[2 * i], ev[2 * j + 1]);
            ms_sum[st[i]] += ms;
            i = j + 1;
        }
        if (per_call_ms && *count < cap) {
            float tot = 0.f;
            (void)hipEventElapsedTime(&tot, ev[0], ev[2 * nk - 1]);
            per_call_ms[*count] = tot;
        }
        ++*count;
    }
    c->prof_head = 0;
    return PSTEREO_OK;
}


// ------------------------------------------------------------------ video
// The frame's launch sequence as HIP graphs, replayed per frame with the
// frame and output pointers written into the kernel nodes' arguments.  A ring
// of kRing instantiated copies lets the host prepare frame n+1 while frame n
// runs; copy k is rewritten only after its previous replay (frame n - kRing)
// has finished: completion events are recorded after every kEvery-th frame,
// alternating between two events.  The region grouping reads only the
// block tables and keeps its template arguments.
//
// Pipelined video (PSTEREO_PIPELINE at begin): each copy is two graphs, the
// depth-map stages (replayed on the context's side stream) and the filter +
// warp (on the video's stream, after the depth graph of the same frame), and
// copy k works in block-table set k % 2; frame n's depth graph waits only for
// what the video's stream held before frame n-1's call, so it runs during
// frame n-1's filter and warp.
struct pstereo_video {
    static constexpr int kRing = 8;
    static constexpr int kEvery = 4;
    static_assert(kRing % 2 == 0, "ring copy k uses block-table set k % 2");
    pstereo_ctx* ctx = nullptr;
    int w = 0, h = 0;
    pstereo_params params{};
    hipStream_t stream = nullptr;
    bool pipe = false;
    bool pipe_started = false;  // the previous frame went through the pipelined graphs
    // pipelined: frame numbers, [0] the last frame whose depth map is done,
    // [1] the last frame whose depth filter has started (both only grow)
    unsigned long long* d_sig = nullptr;
    FrameDesc tmpl{};
    WarpShape ws{};
    pstereo::LaunchSpec ls[kMaxSpecs];
    int stage[kMaxSpecs] = {};
    bool per_frame[kMaxSpecs] = {};  // node i reads the frame / output pointers or a frame number
    int gidx[kMaxSpecs] = {};        // node i's graph: 0, or 1 for the filter + warp of a pipelined video
    int nk = 0;
    hipGraph_t graph[2][kRing] = {};
    hipGraphExec_t exec[2][kRing] = {};
    hipGraphNode_t node[kRing][kMaxSpecs] = {};
    hipEvent_t done[2] = {};
    long long waited = -1;  // last event group known complete
    long long count = 0;
};

static void video_free(pstereo_video* v) {
    for (int g = 0; g < 2; ++g) {
        for (int k = 0; k < pstereo_video::kRing; ++k) {
            if (v->exec[g][k]) (void)hipGraphExecDestroy(v->exec[g][k]);
            if (v->graph[g][k]) (void)hipGraphDestroy(v->graph[g][k]);
        }
    }
    for (int k = 0; k < 2; ++k)
        if (v->done[k]) (void)hipEventDestroy(v->done[k]);
    (void)hipFree(v->d_sig);
    delete v;
}

static hipKernelNodeParams node_params(const pstereo::LaunchSpec& ls, void** args) {
    hipKernelNodeParams kp{};
    kp.blockDim = ls.block;
    kp.gridDim = ls.grid;
    kp.func = const_cast<void*>(ls.func);
    kp.kernelParams = args;
    kp.extra = nullptr;
    kp.sharedMemBytes = (unsigned)ls.lds;
    return kp;
}

// The descriptor of ring copy k: f with the block tables of its set.
static FrameDesc video_desc(const pstereo_video* v, const FrameDesc& f, int k) {
    FrameDesc d = f;
    const BlockScratch& bs = v->ctx->blk[v->pipe ? k % 2 : 0];
    d.stats = bs.stats;
    d.binfo = bs.binfo;
    d.labels = bs.labels;
    d.rent = bs.rent;
    d.rrow = bs.rrow;
    d.rfin = bs.rfin;
    d.rbnd = bs.rbnd;
    d.rctl = bs.rctl;
    return d;
}

int pstereo_video_begin(pstereo_ctx* c, int w, int h, const pstereo_params* p, pstereo_video** out) {
    if (!c) return PSTEREO_E_INVALID;
    c->err[0] = '\0';
    if (!out) return fail(c, PSTEREO_E_INVALID, "out is NULL");
    *out = nullptr;
    pstereo_params pp;
    pstereo_params_init(&pp);
    if (p) {
        if (p->struct_size != sizeof(pstereo_params))
            return fail(c, PSTEREO_E_INVALID, "params.struct_size %u != %zu", p->struct_size, sizeof(pstereo_params));
        pp = *p;
    }
    if (pp.flags & (PSTEREO_DEPTH_EXTERNAL | PSTEREO_WARP_GATHER | PSTEREO_INPAINT_BLOCKS))
        return fail(c, PSTEREO_E_UNSUPPORTED, "video replay generates the depth map and warps (no "
                                              "PSTEREO_DEPTH_EXTERNAL / PSTEREO_WARP_GATHER)");
    if (pp.out_depth || pp.out_depth_raw || pp.out_hsbs)
        return fail(c, PSTEREO_E_UNSUPPORTED, "video replay takes no depth dumps");
    if (pp.flags & PSTEREO_PIPELINE_DEEP)
        return fail(c, PSTEREO_E_UNSUPPORTED, "video replay pipelines two stages (PSTEREO_PIPELINE), not three");
    pstereo_video* v = new (std::nothrow) pstereo_video;
    if (!v) return fail(c, PSTEREO_E_NOMEM, "host allocation failed");
    v->ctx = c;
    v->w = w;
    v->h = h;
    v->params = pp;
    v->pipe = (pp.flags & PSTEREO_PIPELINE) != 0;
    uint32_t flags;
    // template descriptor: aligned placeholders stand in for the frame buffers
    // (the graphs run on p->stream, NULL = the HIP null stream)
    uint8_t* ph = c->d_df;
    int rc = build_desc(c, ph, w, h, &pp, ph + 4, ph + 8, ph + 12, &v->tmpl, &v->ws, &v->stream, &flags, false);
    if (rc != PSTEREO_OK) {
        delete v;
        return rc;
    }
    v->tmpl.out_l = v->tmpl.out_r = v->tmpl.out_a = nullptr;
    v->tmpl.frame = nullptr;
    v->tmpl.aligned = (w % 4 == 0);
    frame_specs(v->tmpl, v->ws, v->ls, v->nk, &v->stage);
    for (int i = 0; i < v->nk; ++i) {
        // a pipelined video's last grouping kernel signals the frame's number
        const bool signals = v->pipe && v->stage[i] == 1 && (i + 1 == v->nk || v->stage[i + 1] != 1);
        v->per_frame[i] = v->stage[i] != 1 || signals;
        v->gidx[i] = v->pipe && v->stage[i] >= 2 ? 1 : 0;
    }
    hipError_t e = hipSetDevice(c->device);
    if (v->pipe && e == hipSuccess) ensure_overlap(c, v->stream, false);
    if (v->pipe && e == hipSuccess && (e = hipMalloc(&v->d_sig, 16)) == hipSuccess) e = hipMemset(v->d_sig, 0, 16);
    for (int k = 0; k < pstereo_video::kRing && e == hipSuccess; ++k) {
        FrameDesc arg = video_desc(v, v->tmpl, k);
        void* args[] = {&arg};
        for (int g = 0; g < (v->pipe ? 2 : 1) && e == hipSuccess; ++g) e = hipGraphCreate(&v->graph[g][k], 0);
        int prev[2] = {-1, -1};  // last node added to each graph
        for (int i = 0; i < v->nk && e == hipSuccess; ++i) {
            const int g = v->gidx[i];
            hipKernelNodeParams kp = node_params(v->ls[i], args);
            hipGraphNode_t* dep = prev[g] >= 0 ? &v->node[k][prev[g]] : nullptr;
            e = hipGraphAddKernelNode(&v->node[k][i], v->graph[g][k], dep, dep ? 1 : 0, &kp);
            prev[g] = i;
        }
        for (int g = 0; g < (v->pipe ? 2 : 1) && e == hipSuccess; ++g)
            e = hipGraphInstantiate(&v->exec[g][k], v->graph[g][k], nullptr, nullptr, 0);
    }
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&v->done[k], hipEventDisableTiming);
    if (e != hipSuccess) {
        video_free(v);
        return fail(c, PSTEREO_E_DEVICE, "graph setup: %s", hipGetErrorString(e));
    }
    *out = v;
    return PSTEREO_OK;
}

int pstereo_video_frame(pstereo_video* v, const uint8_t* frame, uint8_t* out_l, uint8_t* out_r, uint8_t* out_a) {
    if (!v) return PSTEREO_E_INVALID;
    pstereo_ctx* c = v->ctx;
    c->err[0] = '\0';
    FrameDesc f;
    WarpShape ws{};
    hipStream_t s;
    uint32_t flags;
    int rc = build_desc(c, frame, v->w, v->h, &v->params, out_l, out_r, out_a, &f, &ws, &s, &flags);
    if (rc != PSTEREO_OK) return rc;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return fail(c, PSTEREO_E_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    c->pipe_valid = false;  // a later plain pipelined call waits for this frame
    if (f.aligned != v->tmpl.aligned) {
        // the captured kernels assume the first frame's alignment; launch
        // directly on the stream, in set 0, after everything before
        pstereo::LaunchSpec ls[kMaxSpecs];
        int n;
        frame_specs(f, ws, ls, n);
        for (int i = 0; i < n; ++i)
            if ((e = pstereo::launch(ls[i], f, s)) != hipSuccess)
                return fail(c, PSTEREO_E_DEVICE, "launch: %s", hipGetErrorString(e));
        v->pipe_started = false;  // the next frame's depth graph waits for this one
        return PSTEREO_OK;
    }
    constexpr int R = pstereo_video::kRing, E = pstereo_video::kEvery;
    const long long n = v->count;
    const int k = (int)(n % R);
    if (n >= R) {
        // the previous replay of copy k (frame n - R) is covered by the event
        // recorded after frame ((n - R) / E) * E + E - 1 < n
        const long long g = (n - R) / E;
        if (g > v->waited) {
            if ((e = hipEventSynchronize(v->done[g % 2])) != hipSuccess)
                return fail(c, PSTEREO_E_DEVICE, "event synchronize: %s", hipGetErrorString(e));
            v->waited = g;
        }
    }
    FrameDesc arg = video_desc(v, f, k);
    const unsigned long long fn = (unsigned long long)n + 1;  // this frame's number
    if (v->pipe) {
        arg.sig = v->d_sig;
        arg.sig_value = fn;
        arg.mark = v->d_sig + 1;
        arg.mark_value = fn;
    }
    void* args[] = {&arg};
    for (int i = 0; i < v->nk; ++i) {
        if (!v->per_frame[i]) continue;
        hipKernelNodeParams kp = node_params(v->ls[i], args);
        if ((e = hipGraphExecKernelNodeSetParams(v->exec[v->gidx[i]][k], v->node[k][i], &kp)) != hipSuccess)
            return fail(c, PSTEREO_E_DEVICE, "graph node update: %s", hipGetErrorString(e));
    }
    if (v->pipe) {
        // the depth graph once the previous frame's filter has started, so
        // after what the stream held before that frame's call (for the first
        // frame: after everything, an event); the filter and warp once the
        // depth graph's grouping has signalled this frame's number (both
        // through the video's words, polled by wait-value packets)
        if ((!v->pipe_started && ((e = hipEventRecord(c->ev_before, v->stream)) != hipSuccess ||
                                  (e = hipStreamWaitEvent(c->side, c->ev_before, 0)) != hipSuccess)) ||
            (v->pipe_started &&
             (e = hipStreamWaitValue64(c->side, v->d_sig + 1, fn - 1, hipStreamWaitValueGte, ~0ull)) != hipSuccess) ||
            (e = hipGraphLaunch(v->exec[0][k], c->side)) != hipSuccess ||
            (e = hipStreamWaitValue64(v->stream, v->d_sig, fn, hipStreamWaitValueGte, ~0ull)) != hipSuccess ||
            (e = hipGraphLaunch(v->exec[1][k], v->stream)) != hipSuccess) {
            v->pipe_started = false;
            return fail(c, PSTEREO_E_DEVICE, "pipelined graph launch: %s", hipGetErrorString(e));
        }
        v->pipe_started = true;
    } else if ((e = hipGraphLaunch(v->exec[0][k], v->stream)) != hipSuccess) {
        return fail(c, PSTEREO_E_DEVICE, "graph launch: %s", hipGetErrorString(e));
    }
    if (n % E == E - 1 && (e = hipEventRecord(v->done[(n / E) % 2], v->stream)) != hipSuccess)
        return fail(c, PSTEREO_E_DEVICE, "event record: %s", hipGetErrorString(e));
    v->count++;
    c->have_blocks = true;
    c->last_fd = arg;
    c->blocks_final = f.rstrip == 0;
    c->last_gw = f.gw;
    c->last_gh = f.gh;
    c->last_stream = v->stream;
    return PSTEREO_OK;
}

int pstereo_video_end(pstereo_video* v) {
    if (!v) return PSTEREO_OK;
    (void)hipSetDevice(v->ctx->device);
    (void)hipStreamSynchronize(v->stream);
    video_free(v);
    return PSTEREO_OK;
}

}  // extern "C"

// ------------------------------------------------------------ no-alloc call
// pstereo_synthesize_noalloc: the plain call with its scratch (one set of
// block tables and the filtered depth of a frame of up to
// PSTEREO_NOALLOC_MAX_PIXELS pixels) in a file-scope device array, so that a
// call allocates nothing.  Each GPU the library runs on holds its own copy of
// the array until the process ends; host code reaches it only through the
// device address hipGetSymbolAddress gives on that device.
namespace {

constexpr size_t kNoAllocBytes = block_scratch_bytes() + align256(PSTEREO_NOALLOC_MAX_PIXELS);
constexpr int kNoAllocDevices = 64;

__device__ __align__(256) uint8_t scratch[kNoAllocBytes];

struct NoAllocDevice {
    std::mutex mu;
    bool ready = false;
    uint8_t* ptr = nullptr;  // this device's address of `scratch`
    pstereo_ctx ctx;         // sizes, device and the scratch carved from ptr
};

NoAllocDevice g_noalloc[kNoAllocDevices];

// Once per device, with the device current: its address of the array, and
// the kernels' launch attributes.
int noalloc_setup(int device, NoAllocDevice** out) {
    if (device < 0 || device >= kNoAllocDevices)
        return fail(nullptr, PSTEREO_E_INVALID, "device %d outside 0..%d", device, kNoAllocDevices - 1);
    NoAllocDevice& d = g_noalloc[device];
    std::lock_guard<std::mutex> g(d.mu);
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(nullptr, PSTEREO_E_INVALID, "device %d not available: %s", device, hipGetErrorString(e));
    }
    if (!d.ready) {
        void* ptr = nullptr;
        if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(nullptr, PSTEREO_E_DEVICE, "static scratch address on device %d: %s", device,
                        hipGetErrorString(e));
        }
        if ((e = pstereo::prepare_depth_kernels()) != hipSuccess || (e = pstereo::prepare_render_kernels()) != hipSuccess)
            return fail(nullptr, PSTEREO_E_DEVICE, "device setup failed: %s", hipGetErrorString(e));
        d.ptr = static_cast<uint8_t*>(ptr);
        d.ctx.device = device;
        d.ctx.max_w = 65535;
        d.ctx.max_h = 65535;
        block_scratch_carve(d.ctx.blk[0], d.ptr);
        d.ctx.d_df = d.ptr + block_scratch_bytes();
        d.ready = true;
    }
    *out = &d;
    return PSTEREO_OK;
}

}  // namespace

extern "C" int pstereo_synthesize_noalloc(int device, const uint8_t* frame, int w, int h, const pstereo_params* pin,
                                          uint8_t* out_l, uint8_t* out_r, uint8_t* out_a) {
    g_create_error[0] = '\0';
    NoAllocDevice* d = nullptr;
    int rc = noalloc_setup(device, &d);
    if (rc != PSTEREO_OK) return rc;
    if (pin && pin->struct_size == sizeof(pstereo_params) &&
        (pin->flags & (PSTEREO_PROFILE | PSTEREO_INPAINT_BLOCKS | PSTEREO_PIPELINE | PSTEREO_PIPELINE_DEEP)))
        return fail(nullptr, PSTEREO_E_UNSUPPORTED,
                    "PSTEREO_PROFILE, PSTEREO_INPAINT_BLOCKS and PSTEREO_PIPELINE(_DEEP) need a context");
    if (w < 1 || h < 1 || (int64_t)w * h > (int64_t)PSTEREO_NOALLOC_MAX_PIXELS)
        return fail(nullptr, PSTEREO_E_INVALID, "frame %dx%d outside 1..%d pixels of the static scratch", w, h,
                    PSTEREO_NOALLOC_MAX_PIXELS);
    std::lock_guard<std::mutex> g(d->mu);  // the per-device descriptor state
    pstereo_ctx* c = &d->ctx;
    FrameDesc f;
    WarpShape ws{};
    hipStream_t s;
    uint32_t flags;
    rc = build_desc(c, frame, w, h, pin, out_l, out_r, out_a, &f, &ws, &s, &flags);
    if (rc != PSTEREO_OK) {
        snprintf(g_create_error, sizeof g_create_error, "%s", c->err);
        return rc;
    }
    hipError_t e = hipSetDevice(device);
    // the grouping's control words start at zero on every call: an earlier
    // call on this GPU may have stopped between its strips and its merge
    if (e == hipSuccess && !f.depth_in) e = pstereo::launch_clear_words(f.rctl, 4, s);
    if (e != hipSuccess) return fail(nullptr, PSTEREO_E_DEVICE, "launch: %s", hipGetErrorString(e));
    pstereo::LaunchSpec ls[kMaxSpecs];
    int n;
    frame_specs(f, ws, ls, n);
    for (int i = 0; i < n; ++i)
        if ((e = pstereo::launch(ls[i], f, s)) != hipSuccess)
            return fail(nullptr, PSTEREO_E_DEVICE, "launch: %s", hipGetErrorString(e));
    if ((flags & PSTEREO_SYNC) && (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail(nullptr, PSTEREO_E_DEVICE, "stream synchronize: %s", hipGetErrorString(e));
    return PSTEREO_OK;
}
