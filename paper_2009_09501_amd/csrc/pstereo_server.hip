// Continuous-batching server: frames of several concurrent video streams,
// admitted as device slots free up, launched as batches on a few HIP streams
// ("lanes") so that a batch formed from late arrivals runs while earlier ones
// drain.
//
// Host-side only; the device work is the persistent batch kernel (policy
// BATCH) or the plain per-frame kernel sequence (policy PLAIN, the baseline
// the batch policy is compared with).  One scheduler thread per server owns
// every HIP call after create; clients only queue requests and read
// completions, under one mutex.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "pstereo.h"
#include "pstereo_batch.h"
#include "pstereo_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t id = 0;
    int sid = 0;
    const uint8_t* frame = nullptr;  // caller's (device, or host for a host-I/O stream)
    uint8_t* out[3] = {nullptr, nullptr, nullptr};
    int slot = -1;
    double t_submit = 0, t_launch = 0;
};

struct StreamState {
    bool open = false;
    int w = 0, h = 0, B = 0, K = 0;
    bool host_io = false;
    int nslots = 0;
    size_t slot_bytes = 0, scratch_bytes = 0;
    uint8_t* mem = nullptr;  // nslots slots: [scratch][frame 3wh][L 3wh][R 3wh][A 3wh] (images only for host I/O)
    std::vector<int> free_slots;
    std::deque<Request> pending;
    int inflight = 0;
};

struct Lane {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    pstereo_batch* batch = nullptr;
    // the lane's own context for batches of one frame (made on first need,
    // remade larger for a larger frame), its largest frame and HBM bytes
    pstereo_ctx* ctx = nullptr;
    int cw = 0, ch = 0;
    int64_t ctx_bytes = 0;
    std::vector<Request> reqs;
    bool busy = false;
    std::string err;  // message of the lane's last launch failure
};

int auto_block(int w, int h) {
    static const int cand[4] = {8, 16, 32, 64};
    for (int K : cand)
        if ((long long)((w + K - 1) / K) * ((h + K - 1) / K) <= PSTEREO_MAX_BLOCKS) return K;
    return -1;
}

bool is_device_ptr(const void* p, int device) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == device;
}

}  // namespace

struct pstereo_server {
    int device = 0;
    int policy = PSTEREO_SERVE_BATCH;
    int64_t budget = 0, in_use = 0;
    int max_streams = 0, max_batch = 0, queue_cap = 0;
    pstereo_ctx* ctx = nullptr;  // own context: its stream, and the plain path's scratch
    std::vector<StreamState> streams;
    std::vector<Lane> lanes;
    std::deque<pstereo_completion> done;
    uint64_t next_id = 1, submitted = 0, completed = 0;
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    size_t rr = 0;  // stream to look at first when forming the next batch
    std::string err;
    std::atomic<int> device_error{0};

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

int sfail(pstereo_server* s, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    s->err = buf;
    return code;
}

int lfail(Lane& ln, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ln.err = buf;
    return code;
}

// Device pointers of slot k of stream st: scratch, then (host I/O) staging
// images in the order frame, left, right, anaglyph.
uint8_t* slot_base(const StreamState& st, int k) { return st.mem + (size_t)k * st.slot_bytes; }

uint8_t* slot_image(const StreamState& st, int k, int which) {
    return slot_base(st, k) + st.scratch_bytes + (size_t)which * 3 * st.w * st.h;
}

// Complete a lane whose event has fired (called with the lock held).
void retire(pstereo_server* s, Lane& ln, int status) {
    const double t = s->now();
    for (const Request& r : ln.reqs) {
        StreamState& st = s->streams[r.sid];
        st.free_slots.push_back(r.slot);
        --st.inflight;
        pstereo_completion c;
        c.req_id = r.id;
        c.stream_id = r.sid;
        c.status = status;
        c.t_submit = r.t_submit;
        c.t_launch = r.t_launch;
        c.t_done = t;
        s->done.push_back(c);
        ++s->completed;
    }
    ln.reqs.clear();
    ln.busy = false;
}

// Take the requests of the next batch: oldest first across streams, each
// needing a free slot of its stream.  Lock held.
void take_batch(pstereo_server* s, std::vector<Request>& out, int limit) {
    out.clear();
    while ((int)out.size() < limit) {
        int best = -1;
        double tb = 0;
        const size_t n = s->streams.size();
        for (size_t i = 0; i < n; ++i) {
            const size_t k = (s->rr + i) % n;
            const StreamState& st = s->streams[k];
            if (!st.open || st.pending.empty() || st.free_slots.empty()) continue;
            if (best < 0 || st.pending.front().t_submit < tb) {
                best = (int)k;
                tb = st.pending.front().t_submit;
            }
        }
        if (best < 0) break;
        StreamState& st = s->streams[best];
        Request r = st.pending.front();
        st.pending.pop_front();
        r.slot = st.free_slots.back();
        st.free_slots.pop_back();
        ++st.inflight;
        out.push_back(r);
        s->rr = (best + 1) % n;
    }
}

// The lane's context for a frame of w x h, made (or remade) for the largest
// frame of the open streams if the HBM budget allows it (lock NOT held;
// takes it to read the streams and the budget).  False: none.
bool lane_context(pstereo_server* s, Lane& ln, int w, int h) {
    if (ln.ctx && ln.cw >= w && ln.ch >= h) return true;
    int cw = std::max(ln.cw, w), ch = std::max(ln.ch, h);
    int64_t need;
    {
        std::lock_guard<std::mutex> g(s->mu);
        for (const StreamState& st : s->streams)
            if (st.open) {
                cw = std::max(cw, st.w);
                ch = std::max(ch, st.h);
            }
        // filtered depth, and two sets of block tables of ~20 bytes per block
        need = (int64_t)cw * ch + (int64_t)PSTEREO_MAX_BLOCKS * 40;
        if (s->in_use - ln.ctx_bytes + need > s->budget) return false;
        s->in_use += need - ln.ctx_bytes;
    }
    if (ln.ctx) pstereo_destroy(ln.ctx);  // waits for the device
    ln.ctx = nullptr;
    if (pstereo_create(&ln.ctx, s->device, cw, ch) != PSTEREO_OK) {
        ln.ctx = nullptr;
        std::lock_guard<std::mutex> g(s->mu);
        s->in_use -= need;
        ln.cw = ln.ch = 0;
        ln.ctx_bytes = 0;
        return false;
    }
    ln.cw = cw;
    ln.ch = ch;
    ln.ctx_bytes = need;
    return true;
}

// Enqueue one lane's requests (lock NOT held: only the scheduler thread
// touches lanes and slot memory).  Returns a status code.
int launch_lane(pstereo_server* s, Lane& ln) {
    const int n = (int)ln.reqs.size();
    std::vector<pstereo_job> jobs(n);
    std::vector<pstereo::JobScratch> scr(n);
    hipError_t e = hipSuccess;
    for (int i = 0; i < n; ++i) {
        const Request& r = ln.reqs[i];
        const StreamState& st = s->streams[r.sid];
        const size_t img = (size_t)3 * st.w * st.h;
        pstereo_job& j = jobs[i];
        j.w = st.w;
        j.h = st.h;
        j.max_disparity = st.B;
        if (st.host_io) {
            j.frame = slot_image(st, r.slot, 0);
            j.out_left = r.out[0] ? slot_image(st, r.slot, 1) : nullptr;
            j.out_right = r.out[1] ? slot_image(st, r.slot, 2) : nullptr;
            j.out_anaglyph = r.out[2] ? slot_image(st, r.slot, 3) : nullptr;
            if ((e = hipMemcpyAsync(const_cast<uint8_t*>(j.frame), r.frame, img, hipMemcpyHostToDevice, ln.st)) != hipSuccess)
                return lfail(ln, PSTEREO_E_DEVICE, "frame upload: %s", hipGetErrorString(e));
        } else {
            j.frame = r.frame;
            j.out_left = r.out[0];
            j.out_right = r.out[1];
            j.out_anaglyph = r.out[2];
        }
        scr[i] = pstereo::job_scratch_carve(slot_base(st, r.slot), st.w, st.h, st.K);
    }
    pstereo_params p;
    pstereo_params_init(&p);
    p.stream = ln.st;
    int rc = PSTEREO_OK;
    if (s->policy == PSTEREO_SERVE_BATCH && n == 1 && lane_context(s, ln, jobs[0].w, jobs[0].h)) {
        // a batch of one frame: the per-frame launch sequence, whose
        // strip-parallel grouping beats the batch's one-workgroup grouping of
        // a whole frame
        p.max_disparity = jobs[0].max_disparity;
        rc = pstereo_synthesize(ln.ctx, jobs[0].frame, jobs[0].w, jobs[0].h, &p, jobs[0].out_left, jobs[0].out_right,
                                jobs[0].out_anaglyph);
        if (rc != PSTEREO_OK) return lfail(ln, rc, "frame: %s", pstereo_last_error(ln.ctx));
    } else if (s->policy == PSTEREO_SERVE_BATCH) {
        rc = pstereo::batch_prepare_internal(ln.batch, jobs.data(), n, &p, scr.data(), false);
        if (rc == PSTEREO_OK) rc = pstereo_batch_launch(ln.batch, ln.st);
        if (rc != PSTEREO_OK) return lfail(ln, rc, "batch: %s", pstereo_batch_last_error(ln.batch));
    } else {
        for (int i = 0; i < n && rc == PSTEREO_OK; ++i) {
            p.max_disparity = jobs[i].max_disparity;
            rc = pstereo_synthesize(s->ctx, jobs[i].frame, jobs[i].w, jobs[i].h, &p, jobs[i].out_left,
                                    jobs[i].out_right, jobs[i].out_anaglyph);
        }
        if (rc != PSTEREO_OK) return lfail(ln, rc, "plain: %s", pstereo_last_error(s->ctx));
    }
    for (int i = 0; i < n; ++i) {
        const Request& r = ln.reqs[i];
        const StreamState& st = s->streams[r.sid];
        if (!st.host_io) continue;
        const size_t img = (size_t)3 * st.w * st.h;
        for (int v = 0; v < 3; ++v)
            if (r.out[v] && (e = hipMemcpyAsync(r.out[v], slot_image(st, r.slot, 1 + v), img, hipMemcpyDeviceToHost,
                                                ln.st)) != hipSuccess)
                return lfail(ln, PSTEREO_E_DEVICE, "result download: %s", hipGetErrorString(e));
    }
    if ((e = hipEventRecord(ln.done, ln.st)) != hipSuccess)
        return lfail(ln, PSTEREO_E_DEVICE, "event record: %s", hipGetErrorString(e));
    return PSTEREO_OK;
}

void scheduler(pstereo_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        bool progress = false;
        // retire finished lanes
        for (Lane& ln : s->lanes) {
            if (!ln.busy) continue;
            const hipError_t q = hipEventQuery(ln.done);
            if (q == hipErrorNotReady) continue;
            retire(s, ln, q == hipSuccess ? PSTEREO_OK : PSTEREO_E_DEVICE);
            if (q != hipSuccess) s->device_error = 1;
            progress = true;
        }
        if (progress) s->cv_done.notify_all();
        if (s->stop && s->submitted == s->completed) break;
        // fill idle lanes with what is waiting
        for (Lane& ln : s->lanes) {
            if (ln.busy) continue;
            take_batch(s, ln.reqs, s->max_batch);
            if (ln.reqs.empty()) break;
            const double t = s->now();
            for (Request& r : ln.reqs) r.t_launch = t;
            ln.busy = true;
            lk.unlock();
            const int rc = launch_lane(s, ln);
            lk.lock();
            if (rc != PSTEREO_OK) {
                // nothing (more) of this lane was enqueued after the failure:
                // wait for what was, then report the requests as failed
                (void)hipStreamSynchronize(ln.st);
                (void)hipGetLastError();
                s->err = ln.err;
                s->device_error = 1;
                retire(s, ln, rc);
                s->cv_done.notify_all();
            }
            progress = true;
        }
        if (progress) continue;
        bool any_busy = false;
        for (const Lane& ln : s->lanes) any_busy |= ln.busy;
        if (any_busy) {
            // a lane is running: poll its event at a short interval
            s->cv_work.wait_for(lk, std::chrono::microseconds(20));
        } else {
            s->cv_work.wait(lk, [s] {
                if (s->stop) return true;
                for (const StreamState& st : s->streams)
                    if (st.open && !st.pending.empty() && !st.free_slots.empty()) return true;
                return false;
            });
        }
    }
}

void server_free(pstereo_server* s) {
    (void)hipSetDevice(s->device);
    for (Lane& ln : s->lanes) {
        if (ln.st) (void)hipStreamSynchronize(ln.st);
        if (ln.batch) pstereo_batch_destroy(ln.batch);
        if (ln.ctx) pstereo_destroy(ln.ctx);
        if (ln.done) (void)hipEventDestroy(ln.done);
        if (ln.st) (void)hipStreamDestroy(ln.st);
    }
    for (StreamState& st : s->streams) (void)hipFree(st.mem);
    if (s->ctx) pstereo_destroy(s->ctx);
    (void)hipGetLastError();
    delete s;
}

}  // namespace

extern "C" {

int pstereo_server_create(int device, int64_t hbm_budget_bytes, int max_streams, int lanes, int policy,
                          pstereo_server** out) {
    if (!out || hbm_budget_bytes < 1 || max_streams < 1 || max_streams > 1024 || lanes < 1 || lanes > 16)
        return PSTEREO_E_INVALID;
    if (policy != PSTEREO_SERVE_BATCH && policy != PSTEREO_SERVE_PLAIN) return PSTEREO_E_INVALID;
    *out = nullptr;
    pstereo_server* s = new (std::nothrow) pstereo_server;
    if (!s) return PSTEREO_E_NOMEM;
    s->device = device;
    s->policy = policy;
    s->budget = hbm_budget_bytes;
    s->max_streams = max_streams;
    s->max_batch = 64;
    s->queue_cap = 256;
    s->t0 = Clock::now();
    s->streams.resize(max_streams);
    // the plain policy runs one frame after another on one stream, with the
    // context's scratch; batches bring their own (the streams' slots)
    if (policy == PSTEREO_SERVE_PLAIN) lanes = 1;
    const int cw = policy == PSTEREO_SERVE_PLAIN ? 7680 : 64, ch = policy == PSTEREO_SERVE_PLAIN ? 4320 : 64;
    s->in_use = (int64_t)cw * ch + (int64_t)PSTEREO_MAX_BLOCKS * 16;
    if (s->in_use > s->budget) {
        delete s;
        return PSTEREO_E_NOMEM;
    }
    int rc = pstereo_create(&s->ctx, device, cw, ch);
    if (rc != PSTEREO_OK) {
        s->ctx = nullptr;
        server_free(s);
        return rc;
    }
    s->lanes.resize(lanes);
    for (Lane& ln : s->lanes) {
        if (hipStreamCreateWithFlags(&ln.st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ln.done, hipEventDisableTiming) != hipSuccess) {
            server_free(s);
            return PSTEREO_E_DEVICE;
        }
        if (policy == PSTEREO_SERVE_BATCH &&
            (rc = pstereo::batch_create_internal(s->ctx, s->max_batch, 1, false, &ln.batch)) != PSTEREO_OK) {
            ln.batch = nullptr;
            server_free(s);
            return rc;
        }
    }
    s->worker = std::thread(scheduler, s);
    *out = s;
    return PSTEREO_OK;
}

int pstereo_server_open_stream(pstereo_server* s, int w, int h, int max_disparity, int slots, uint32_t flags,
                               int* stream_id) {
    if (!s || !stream_id) return PSTEREO_E_INVALID;
    std::lock_guard<std::mutex> g(s->mu);
    s->err.clear();
    if (w < 1 || h < 1 || w > 7680 || h > 4320) return sfail(s, PSTEREO_E_INVALID, "frame size %dx%d outside 1..7680 x 1..4320", w, h);
    if (slots < 1 || slots > 64) return sfail(s, PSTEREO_E_INVALID, "slots %d outside 1..64", slots);
    if (flags & ~PSTEREO_STREAM_HOST_IO) return sfail(s, PSTEREO_E_INVALID, "unknown stream flags");
    const int B = max_disparity < 0 ? (2 * w + 50) / 100 : max_disparity;
    if (max_disparity < -1 || B > 255) return sfail(s, PSTEREO_E_INVALID, "max_disparity out of range");
    const int K = auto_block(w, h);
    if (K < 0) return sfail(s, PSTEREO_E_INVALID, "frame too large for the block grid");
    if (s->policy == PSTEREO_SERVE_BATCH && (w % 4 != 0 || !pstereo::batch_width_ok(w)))
        return sfail(s, PSTEREO_E_UNSUPPORTED, "width %d: batched frames need a width divisible by 4", w);
    int sid = -1;
    for (int i = 0; i < s->max_streams; ++i)
        if (!s->streams[i].open && s->streams[i].inflight == 0) { sid = i; break; }
    if (sid < 0) return sfail(s, PSTEREO_E_BUSY, "all %d stream slots are open", s->max_streams);
    StreamState& st = s->streams[sid];
    const size_t scratch = pstereo::job_scratch_bytes(w, h, K);
    const size_t images = (flags & PSTEREO_STREAM_HOST_IO) ? (size_t)12 * w * h : 0;
    const size_t slot_bytes = (scratch + images + 255) / 256 * 256;
    const int64_t need = (int64_t)slot_bytes * slots;
    if (s->in_use + need > s->budget)
        return sfail(s, PSTEREO_E_NOMEM, "stream needs %lld B, %lld B of the %lld B budget left", (long long)need,
                     (long long)(s->budget - s->in_use), (long long)s->budget);
    (void)hipSetDevice(s->device);
    uint8_t* mem = nullptr;
    if (hipMalloc(&mem, need) != hipSuccess) {
        (void)hipGetLastError();
        return sfail(s, PSTEREO_E_NOMEM, "device allocation of %lld B failed", (long long)need);
    }
    (void)hipFree(st.mem);
    st = StreamState();
    st.open = true;
    st.w = w;
    st.h = h;
    st.B = B;
    st.K = K;
    st.host_io = (flags & PSTEREO_STREAM_HOST_IO) != 0;
    st.nslots = slots;
    st.slot_bytes = slot_bytes;
    st.scratch_bytes = scratch;
    st.mem = mem;
    for (int k = slots - 1; k >= 0; --k) st.free_slots.push_back(k);
    s->in_use += need;
    *stream_id = sid;
    return PSTEREO_OK;
}

int pstereo_server_close_stream(pstereo_server* s, int stream_id) {
    if (!s) return PSTEREO_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    if (stream_id < 0 || stream_id >= s->max_streams || !s->streams[stream_id].open)
        return sfail(s, PSTEREO_E_INVALID, "stream %d is not open", stream_id);
    StreamState& st = s->streams[stream_id];
    s->cv_done.wait(lk, [&] { return st.pending.empty() && st.inflight == 0; });
    (void)hipSetDevice(s->device);
    (void)hipFree(st.mem);
    s->in_use -= (int64_t)st.slot_bytes * st.nslots;
    st = StreamState();
    return PSTEREO_OK;
}

int pstereo_server_submit(pstereo_server* s, int stream_id, const uint8_t* frame, uint8_t* out_left,
                          uint8_t* out_right, uint8_t* out_anaglyph, uint64_t* req_id) {
    if (!s) return PSTEREO_E_INVALID;
    std::lock_guard<std::mutex> g(s->mu);
    s->err.clear();
    if (s->stop) return sfail(s, PSTEREO_E_INVALID, "server is shutting down");
    if (stream_id < 0 || stream_id >= s->max_streams || !s->streams[stream_id].open)
        return sfail(s, PSTEREO_E_INVALID, "stream %d is not open", stream_id);
    StreamState& st = s->streams[stream_id];
    if (!frame) return sfail(s, PSTEREO_E_INVALID, "null frame");
    if ((int)st.pending.size() >= s->queue_cap)
        return sfail(s, PSTEREO_E_BUSY, "stream %d has %d requests waiting", stream_id, s->queue_cap);
    uint8_t* outs[3] = {out_left, out_right, out_anaglyph};
    const size_t img = (size_t)3 * st.w * st.h;
    if (st.host_io) {
        // host buffers: they must not be device memory of this GPU
        if (is_device_ptr(frame, s->device)) return sfail(s, PSTEREO_E_INVALID, "host-I/O stream got a device frame");
        for (uint8_t* o : outs)
            if (o && is_device_ptr(o, s->device)) return sfail(s, PSTEREO_E_INVALID, "host-I/O stream got a device output");
    } else {
        if (!is_device_ptr(frame, s->device)) return sfail(s, PSTEREO_E_INVALID, "frame is not device memory");
        for (uint8_t* o : outs)
            if (o && !is_device_ptr(o, s->device)) return sfail(s, PSTEREO_E_INVALID, "output is not device memory");
        if (((uintptr_t)frame | (uintptr_t)out_left | (uintptr_t)out_right | (uintptr_t)out_anaglyph) % 4 &&
            s->policy == PSTEREO_SERVE_BATCH)
            return sfail(s, PSTEREO_E_UNSUPPORTED, "batched buffers must be 4-byte aligned");
    }
    for (int a = 0; a < 3; ++a) {
        if (!outs[a]) continue;
        if (outs[a] < frame + img && frame < outs[a] + img) return sfail(s, PSTEREO_E_ALIAS, "an output overlaps the frame");
        for (int c = a + 1; c < 3; ++c)
            if (outs[c] && outs[a] < outs[c] + img && outs[c] < outs[a] + img)
                return sfail(s, PSTEREO_E_ALIAS, "two outputs overlap");
    }
    Request r;
    r.id = s->next_id++;
    r.sid = stream_id;
    r.frame = frame;
    for (int v = 0; v < 3; ++v) r.out[v] = outs[v];
    r.t_submit = s->now();
    st.pending.push_back(r);
    ++s->submitted;
    if (req_id) *req_id = r.id;
    s->cv_work.notify_one();
    return PSTEREO_OK;
}

int pstereo_server_poll(pstereo_server* s, pstereo_completion* out, int max, int* n_out, int wait_us) {
    if (!s || !n_out || max < 0 || (max > 0 && !out)) return PSTEREO_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && wait_us > 0)
        s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), [s] { return !s->done.empty(); });
    int n = 0;
    while (n < max && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    *n_out = n;
    return PSTEREO_OK;
}

int pstereo_server_drain(pstereo_server* s) {
    if (!s) return PSTEREO_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_work.notify_one();
    s->cv_done.wait(lk, [s] { return s->submitted == s->completed; });
    return s->device_error ? PSTEREO_E_DEVICE : PSTEREO_OK;
}

int pstereo_server_info(const pstereo_server* s, int64_t* budget, int64_t* in_use, uint64_t* submitted,
                        uint64_t* completed) {
    if (!s) return PSTEREO_E_INVALID;
    std::lock_guard<std::mutex> g(const_cast<pstereo_server*>(s)->mu);
    if (budget) *budget = s->budget;
    if (in_use) *in_use = s->in_use;
    if (submitted) *submitted = s->submitted;
    if (completed) *completed = s->completed;
    return PSTEREO_OK;
}

int pstereo_server_destroy(pstereo_server* s) {
    if (!s) return PSTEREO_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    server_free(s);
    return PSTEREO_OK;
}

const char* pstereo_server_last_error(const pstereo_server* s) { return s ? s->err.c_str() : ""; }

}  // extern "C"
