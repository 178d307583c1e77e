/*
 * pstereo.h -- C ABI of the MI355X (gfx950) pseudo-stereo DIBR library.
 *
 * One 2D RGB frame in, a stereo pair (left view, right view) and a red-cyan
 * anaglyph out, by the conversion scheme of "3D Pseudo Stereo Visualization
 * with GPGPU Support" (Section 3, Fig. 1; Section 4, the seven steps):
 *
 *   depth map from block colour / edge / region cues
 *   -> cross-bilateral filtering of the depth map, guided by luma
 *   -> left and right frame reconstruction by the depth -> shift rule of the
 *      Fig. 3 code (threshold 150, half of the stereo base per view), written
 *      as a row-wise z-buffered forward warp
 *   -> inpainting of the holes (nearest background pixel of the row)
 *   -> stereo formatting (anaglyph: red from the left view, green and blue
 *      from the right view, as the Fig. 3 code builds its result).
 *
 * Conventions shared by every entry point:
 *  - Images are contiguous uint8 RGB24, [h][w][3], row pitch 3*w bytes, in
 *    DEVICE memory of the context's GPU (for example torch uint8 CUDA tensors).
 *    Host pointers are rejected with PSTEREO_E_INVALID.
 *  - The caller owns every image buffer; the context owns all scratch memory,
 *    allocated once in pstereo_create.  No call after create allocates device
 *    memory, so the launch sequence can be captured into a HIP graph.
 *  - Calls enqueue work on params->stream (a hipStream_t; NULL = the HIP null
 *    stream, the legacy default stream, which is also torch's default stream)
 *    and return; outputs are valid once that stream has reached the work
 *    (synchronise it, or set PSTEREO_SYNC).  The work is ordered after what
 *    was enqueued on that stream before the call, like any kernel on it.
 *  - Every call returns a status code; nothing is thrown across the ABI.
 *    Errors are not sticky.  The message of the last failure is kept per
 *    context (pstereo_last_error).  A context is not thread-safe: use one per
 *    host thread.
 */
#ifndef PSTEREO_H
#define PSTEREO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define PSTEREO_OK 0
#define PSTEREO_E_INVALID (-1)     /* bad argument: size, range, null or host pointer */
#define PSTEREO_E_NOMEM (-2)       /* device allocation failed (create only) */
#define PSTEREO_E_DEVICE (-3)      /* a HIP runtime call or kernel launch failed */
#define PSTEREO_E_ALIAS (-4)       /* output buffers overlap each other or an input */
#define PSTEREO_E_UNSUPPORTED (-5) /* valid request the library cannot run (e.g. too wide for LDS) */
#define PSTEREO_E_BUSY (-6)        /* server: request not admitted now, retry later */

/* Flags. */
#define PSTEREO_DEPTH_EXTERNAL 0x1u /* depth_in replaces the generated depth map */
#define PSTEREO_SYNC 0x2u           /* block until the outputs are complete */
#define PSTEREO_PROFILE 0x4u        /* record each kernel's start and stop times in HIP events
                                       (pstereo_profile_collect) */
#define PSTEREO_WARP_GATHER 0x8u    /* reconstruct the views as the Fig. 3 code does (Section 4):
                                       each destination pixel gathers the source pixel its
                                       own filtered depth points back to, its own source
                                       pixel when that lies outside the row; no z-buffer, no
                                       hole filling; the anaglyph takes red from the gathered
                                       left view, green and blue from the gathered right.
                                       Plain calls only */
#define PSTEREO_INPAINT_BLOCKS 0x10u /* fill holes by the block-iterative inpainting of Fig. 3
                                       (Section 4) instead of the row fill: Jacobi sweeps over
                                       the whole frame, a hole with >= 2 undamaged 8-neighbours
                                       taking their mean (rounded half up), until a sweep fills
                                       nothing; pixels never filled keep their own source pixel.
                                       A frame still filling pixels at sweep 4096 is not composed:
                                       the call returns PSTEREO_E_UNSUPPORTED and the outputs are
                                       left unwritten.  Plain calls only.  The first
                                       such call allocates 12 * max_w * max_h bytes of scratch,
                                       and every such call waits for its sweeps (the host checks
                                       convergence), so it is neither asynchronous nor
                                       graph-capturable */

#define PSTEREO_PIPELINE 0x20u      /* pipelined plain calls: this call's depth-map stages (block
                                       statistics, region grouping) run on a second stream the
                                       context owns, so that they overlap the depth filter and
                                       warp of the context's previous pipelined call.  The caller
                                       promises that everything writing this call's frame was
                                       enqueued on params->stream (or had finished) before that
                                       previous pipelined call was made; the filter and warp still
                                       follow everything on params->stream.  Calls on the same
                                       context alternate two sets of block tables.  The two
                                       streams order each other through stream wait-value packets
                                       (which the runtime runs as small polling kernels), so a
                                       profiler that serialises dispatches cannot run such calls.
                                       Streams overlap only on distinct hardware queues: the
                                       first pipelined call on a stream waits for it and checks
                                       (a few hundred microseconds) that the context's streams
                                       run beside it, and replaces one that does not.
                                       Ignored with PSTEREO_DEPTH_EXTERNAL or
                                       PSTEREO_INPAINT_BLOCKS; not for stream capture */
#define PSTEREO_PIPELINE_DEEP 0x40u /* three-stage pipelined plain calls (implies PSTEREO_PIPELINE):
                                       the depth-map stages on the context's second stream, the
                                       depth filter on a third one and the warp on params->stream,
                                       so that this call's depth map, the previous call's filter
                                       and the warp of the call before that run at once.  The
                                       caller promises that everything writing this call's frame
                                       was enqueued on params->stream (or had finished) before the
                                       pipelined call two calls back was made (frames supplied two
                                       ahead); the warp still follows everything on
                                       params->stream.  Calls alternate two sets of block tables
                                       and two filtered-depth images.  A call that changes stream
                                       or mode, or follows another kind of call, starts the
                                       pipeline again.  Same exclusions as PSTEREO_PIPELINE; the
                                       video calls reject it */

/* Largest number of depth blocks per frame (region grouping runs in one
 * workgroup's LDS). */
#define PSTEREO_MAX_BLOCKS 32768

/*
 * Parameters of one synthesis.  Initialise with pstereo_params_init, then
 * override fields.  The paper fixes only the threshold 150 and the half-base
 * per view (Section 4, Fig. 3); every other constant is the library's reading.
 */
typedef struct pstereo_params {
    uint32_t struct_size;     /* must be sizeof(pstereo_params) (ABI version check) */
    int32_t max_disparity;    /* B: maximum total parallax in px, 0..255 ("Base"
                                 of the Fig. 3 code); -1 = round(0.02 * w) */
    int32_t depth_threshold;  /* T: depths above T shift crossed (in front of the
                                 screen), others uncrossed; 150 in the paper;
                                 -1..255, -1 = linear mode (depth 0 at the screen) */
    int32_t block_size;       /* K: depth block edge in px, one of 2, 4, 8, 16, 32, 64;
                                 0 = smallest of 8, 16, 32, 64 giving at most
                                 PSTEREO_MAX_BLOCKS blocks */
    int32_t edge_thresh;      /* g: a block is an edge block when some forward luma
                                 step inside it exceeds g; 0..255, default 24 */
    int32_t link_thresh;      /* tau: neighbouring non-edge blocks join one region
                                 when their mean colours differ by <= tau (sum of
                                 |dR|+|dG|+|dB|); 0..765, default 24 */
    int32_t cbf_radius;       /* r: cross-bilateral window (2r+1)^2, 0..3, default 2;
                                 spatial sigma 1.5 px, range sigma 12 luma levels */
    uint32_t flags;           /* PSTEREO_DEPTH_EXTERNAL | PSTEREO_SYNC | PSTEREO_PROFILE */
    const uint8_t *depth_in;  /* device uint8 [h][w]: depth map (255 = nearest) used
                                 instead of the generated one when
                                 PSTEREO_DEPTH_EXTERNAL is set; filtered like it */
    uint8_t *out_depth;       /* optional device uint8 [h][w]: filtered depth */
    uint8_t *out_depth_raw;   /* optional device uint8 [h][w]: depth before filtering */
    void *stream;             /* hipStream_t to enqueue on; NULL = the HIP null stream */
    uint8_t *out_hsbs;        /* optional device RGB24 [h][w][3]: half side-by-side
                                 frame (Section 5 names it beside the anaglyph):
                                 left half = left view squeezed to floor(w/2)
                                 columns, right half = right view squeezed to the
                                 remaining ceil(w/2); column p of a half is the mean
                                 of view columns 2p, 2p+1 rounded half up (column
                                 w-1 alone for the last one of odd w).  Plain calls
                                 only: the video, batch and server forms reject it */
} pstereo_params;

typedef struct pstereo_ctx pstereo_ctx;

/* Fill *p with the defaults above (B = -1, T = 150, K = 0, g = 24, tau = 24,
 * r = 2, no flags, no optional buffers, stream NULL).  Returns PSTEREO_OK, or
 * PSTEREO_E_INVALID for a null pointer. */
int pstereo_params_init(pstereo_params *p);

/* Create a context on HIP device `device` for frames up to max_w x max_h
 * (1 <= max_w <= 65535, 1 <= max_h <= 65535).  Allocates all scratch memory
 * (the context owns no stream: work goes on the caller's).  On success *out receives the context.  Errors:
 * PSTEREO_E_INVALID (bad device or sizes, out == NULL), PSTEREO_E_NOMEM,
 * PSTEREO_E_DEVICE. */
int pstereo_create(pstereo_ctx **out, int device, int max_w, int max_h);

/* Synthesize the left view, right view and anaglyph of one frame.
 *   frame        device RGB24 [h][w][3], read only
 *   w, h         frame size, 1 <= w <= max_w, 1 <= h <= max_h
 *   p            parameters (NULL = defaults)
 *   out_left     device RGB24 [h][w][3] (may be NULL to skip)
 *   out_right    device RGB24 [h][w][3] (may be NULL to skip)
 *   out_anaglyph device RGB24 [h][w][3] (may be NULL to skip)
 * Outputs must not overlap each other, the frame or the depth buffers
 * (PSTEREO_E_ALIAS).  Returns PSTEREO_E_UNSUPPORTED when the frame is wider
 * than the warp kernel's row buffers allow (16384 px). */
int pstereo_synthesize(pstereo_ctx *ctx, const uint8_t *frame, int w, int h,
                       const pstereo_params *p, uint8_t *out_left,
                       uint8_t *out_right, uint8_t *out_anaglyph);

/* Release the context and its scratch memory.  NULL is a no-op.  Waits for
 * the device first (the context's work may sit on any of the caller's
 * streams). */
int pstereo_destroy(pstereo_ctx *ctx);

/* Message of the last failed call on ctx ("" if none); ctx may be NULL for
 * failures of pstereo_create.  The string lives until the next call on ctx. */
const char *pstereo_last_error(const pstereo_ctx *ctx);

/*
 * Per-block intermediate results of the last pstereo_synthesize on ctx with a
 * generated depth map (for inspection and parity tests); no other call may
 * have used the context since.  The per-block labels and depths are
 * materialised here (one small kernel on that call's stream, the first time),
 * then the call waits for the stream.  Host buffers of `cap` entries each
 * (any may be NULL):
 *   stats   uint32 per block: mean R | mean G << 8 | mean B << 16 | edge << 24
 *   labels  int32 per block: region label = smallest block index of the region
 *   dblk    uint8 per block: region depth
 * *gw, *gh receive the block grid (row-major, gw blocks per row).  Returns
 * PSTEREO_E_INVALID if cap < gw*gh or no generated-depth call was made.
 */
int pstereo_debug_blocks(pstereo_ctx *ctx, uint32_t *stats, int32_t *labels,
                         uint8_t *dblk, int cap, int *gw, int *gh);

/*
 * Kernel timing.  Each pstereo_synthesize with PSTEREO_PROFILE launches its
 * kernels with a start and a stop HIP event each, which take the times of the
 * kernel's own dispatch (no marker packets between the kernels).  The events
 * are created by the first profiled call on the context.  This call waits
 * for the recorded events, writes the summed durations in milliseconds of the
 * four stages (block statistics, region grouping, depth filter, warp; a stage
 * runs from its first kernel's start to its last kernel's stop) to
 * ms_sum[0..3] and the number of profiled calls to *count, and clears the
 * record.  If per_call_ms is not NULL it receives, in call order, up to cap
 * per-call durations (first kernel's start to last kernel's stop, ms).  At
 * most 4096 calls are kept between collections; older ones are dropped and
 * not counted.  Block-inpainting sweeps are not timed.
 */
int pstereo_profile_collect(pstereo_ctx *ctx, double ms_sum[4], int *count,
                            double *per_call_ms, int cap);

/*
 * pstereo_synthesize_noalloc: pstereo_synthesize without a context, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Its scratch (one
 * set of block tables and one filtered-depth image, about 9 MB) is a static
 * device array that each GPU the library runs on holds until the process
 * ends; the first call on a device takes that array's address there.  The
 * call allocates nothing (no hipMalloc, hipFree or allocating library call):
 *   device       HIP device of the frame and outputs (0..63)
 *   frame, w, h, p, out_left, out_right, out_anaglyph: as pstereo_synthesize,
 *                with w * h <= PSTEREO_NOALLOC_MAX_PIXELS (one 4K frame);
 *                larger frames return PSTEREO_E_INVALID
 * PSTEREO_PROFILE, PSTEREO_INPAINT_BLOCKS, PSTEREO_PIPELINE and PSTEREO_PIPELINE_DEEP return
 * PSTEREO_E_UNSUPPORTED (they need a context's events, scratch or stream).
 * Every call on one GPU shares that GPU's array, whose contents the last call
 * left: calls that overlap on one GPU (two host threads, or two streams not
 * ordered with each other) race and must be serialised by the caller.  The
 * message of a failure is read with pstereo_last_error(NULL) on the calling
 * thread.
 */
#define PSTEREO_NOALLOC_MAX_PIXELS (3840 * 2160)
int pstereo_synthesize_noalloc(int device, const uint8_t *frame, int w, int h, const pstereo_params *p,
                               uint8_t *out_left, uint8_t *out_right, uint8_t *out_anaglyph);

/*
 * Video: the frame's launch sequence captured once as a HIP graph and
 * replayed per frame (the paper converts video frame by frame, Section 5;
 * there is no state between frames).  pstereo_video_begin fixes the frame
 * size and parameters (generated depth only: no PSTEREO_DEPTH_EXTERNAL, no
 * depth dumps); the graph runs on p->stream (NULL = context stream).
 * pstereo_video_frame validates the buffers like pstereo_synthesize, writes
 * their pointers into the kernel arguments of one of eight instantiated
 * copies of the graph and launches it; it may wait for the replay made eight
 * to eleven frames earlier.  Frames on one video run in
 * order on its stream and share the context's scratch, so a context drives
 * one video (or plain calls on the same stream) at a time.
 * pstereo_video_end waits for the stream and frees the graphs.
 * With PSTEREO_PIPELINE in p->flags each copy is two graphs: the depth-map
 * stages, replayed on the context's second stream, and the filter and warp,
 * replayed on the video's stream after them; a frame's depth graph waits
 * only for what the video's stream held before the previous frame's call,
 * so it runs during that frame's filter and warp.  The caller then promises
 * that each frame was complete on the stream (or on the host) before the
 * previous pstereo_video_frame call was made -- frames are supplied one
 * ahead, as a decoder does.
 * Errors as for pstereo_synthesize; PSTEREO_E_UNSUPPORTED for the excluded
 * parameters.
 */
typedef struct pstereo_video pstereo_video;
int pstereo_video_begin(pstereo_ctx *ctx, int w, int h, const pstereo_params *p, pstereo_video **out);
int pstereo_video_frame(pstereo_video *v, const uint8_t *frame, uint8_t *out_left, uint8_t *out_right,
                        uint8_t *out_anaglyph);
int pstereo_video_end(pstereo_video *v);

/*
 * Batched form: many frames of uneven size per launch, in one of two forms
 * (PSTEREO_BATCH_STAGED, the default: one kernel per stage over all frames;
 * PSTEREO_BATCH_FUSED: one persistent kernel whose workgroups claim tasks in
 * a dependency order -- see the tuning section below).  Every frame's output
 * is byte-identical to pstereo_synthesize with the same parameters.
 *
 * pstereo_batch_create: a batch object on ctx's device for up to max_jobs
 *   frames of max_pixels pixels in total; allocates all per-frame scratch
 *   (about 0.5 MiB per job plus one byte per pixel) and pinned staging.
 * pstereo_batch_prepare: validates the jobs and uploads the task tables on
 *   p->stream (NULL = context stream).  Shared parameters come from p; each
 *   job has its own max_disparity (-1 = round(0.02 w)).  Requirements:
 *   generated depth (no PSTEREO_DEPTH_EXTERNAL, no depth dumps), widths a
 *   multiple of 4 and at most 16384, 4-byte aligned device buffers, outputs
 *   disjoint from every frame and from each other (PSTEREO_E_ALIAS).
 * pstereo_batch_launch: enqueues the prepared batch on `stream` (a
 *   hipStream_t; NULL = the prepare stream): the staged kernels, or a
 *   counter-reset kernel and the persistent kernel; no copies and no
 *   allocation, so it can be captured into a HIP graph and replayed.  A prepared batch can be launched any
 *   number of times; launches of one batch object must not overlap.
 *   Each dependency wait inside the persistent kernel is bounded (1 s of
 *   wall-clock time); should one run out, every workgroup leaves early, the
 *   outputs are incomplete and the abort word is raised.
 * pstereo_batch_run: prepare + launch; with PSTEREO_SYNC it also waits for
 *   the stream and returns PSTEREO_E_DEVICE if the abort word was raised.
 * pstereo_batch_last_error: message of the last failure on the batch.
 */
typedef struct pstereo_job {
    const uint8_t *frame;   /* device RGB24 [h][w][3] */
    int32_t w, h;
    uint8_t *out_left;      /* device RGB24 [h][w][3] or NULL */
    uint8_t *out_right;
    uint8_t *out_anaglyph;
    int32_t max_disparity;  /* -1 = round(0.02 w) */
} pstereo_job;

typedef struct pstereo_batch pstereo_batch;
int pstereo_batch_create(pstereo_ctx *ctx, int max_jobs, int64_t max_pixels, pstereo_batch **out);
int pstereo_batch_prepare(pstereo_batch *b, const pstereo_job *jobs, int n, const pstereo_params *p);
int pstereo_batch_launch(pstereo_batch *b, void *stream);
int pstereo_batch_run(pstereo_batch *b, const pstereo_job *jobs, int n, const pstereo_params *p);
int pstereo_batch_destroy(pstereo_batch *b);
const char *pstereo_batch_last_error(const pstereo_batch *b);

/*
 * pstereo_synthesize_batch: the views of n frames (sizes may differ) in one
 * batched launch on p->stream (NULL = the HIP null stream), with a batch
 * object the context keeps.  Same requirements and results as
 * pstereo_batch_run (per-job max_disparity; p's other fields shared); the
 * form is the staged one with 512-lane row-warp workgroups of 4 rows.  The
 * first call, and any call with more jobs (above 64) or pixels (above one 4K
 * frame) than the context's batch object holds, synchronises the device and
 * allocates that object's scratch; later calls allocate nothing.  The call
 * uploads its job tables from pinned staging on the stream, so it is not
 * meant for graph capture (use pstereo_batch_prepare + pstereo_batch_launch).
 * With PSTEREO_SYNC it waits for the stream.  Errors as for
 * pstereo_batch_run; the message is kept on the context.  The paper converts
 * frames one at a time (Section 5); running many frames per launch is this
 * library's form for throughput.
 */
int pstereo_synthesize_batch(pstereo_ctx *ctx, const pstereo_job *jobs, int n, const pstereo_params *p);

/*
 * Batch forms and their tuning.
 *  PSTEREO_BATCH_STAGED (default): one launch per stage over all frames of
 *    the batch (block statistics, region grouping with one workgroup per
 *    frame, depth filter, then one row-warp launch per distinct row shape);
 *    kernel boundaries order the stages.
 *  PSTEREO_BATCH_FUSED: one persistent kernel: its workgroups claim tasks
 *    (per frame: block statistics, region grouping, depth filter, warp) in a
 *    dependency order from one queue per XCD -- each frame belongs to one
 *    XCD, so a task and the tasks it waits for share that XCD's L2 and
 *    synchronise without cache write-back -- so one frame's region grouping
 *    overlaps the streaming work of the others.
 * Tuning fields: warp_lanes (64..1024, multiple of 64) caps the lanes of a
 * row-warp workgroup before quads per lane grow (1, 2, 4); warp_rows (1..8)
 * rows per row-warp workgroup; fused_grid = persistent workgroups (0 = one
 * per compute unit, else 8..65536: every XCD needs workgroups for its
 * queue); bs_rows (staged form) = rows of a block-statistics tile, 256 px
 * wide (0 = 32 for blocks up to 16 px, 64 above; else 16, 32 or 64, raised
 * to the block size).  A new tuning takes effect at the next prepare.
 * pstereo_batch_autotune: runs the jobs (outputs are written) under each
 *   candidate tuning -- staged with warp_lanes in {128, 256, 512, 1024} x
 *   warp_rows in {1, 2, 4}, and fused; then, if a staged candidate won, that
 *   one with bs_rows 16, 32 and 64 -- timing `reps` launches of each with
 *   HIP events on the prepare stream, and leaves the batch prepared with the
 *   fastest; every timed candidate is reported in trials (up to cap).  The
 *   call synchronises with the stream.
 */
#define PSTEREO_BATCH_STAGED 0
#define PSTEREO_BATCH_FUSED 1

typedef struct pstereo_batch_tuning {
    int32_t mode;
    int32_t warp_lanes;
    int32_t warp_rows;
    int32_t fused_grid;
    int32_t bs_rows;
} pstereo_batch_tuning;

typedef struct pstereo_batch_trial {
    pstereo_batch_tuning tuning;
    double ms;  /* mean launch time */
} pstereo_batch_trial;

int pstereo_batch_set_tuning(pstereo_batch *b, const pstereo_batch_tuning *t);
int pstereo_batch_get_tuning(const pstereo_batch *b, pstereo_batch_tuning *t);
int pstereo_batch_autotune(pstereo_batch *b, const pstereo_job *jobs, int n, const pstereo_params *p, int reps,
                           pstereo_batch_tuning *best, double *best_ms, pstereo_batch_trial *trials, int cap,
                           int *n_trials);

/*
 * Serving: frames of several concurrent video streams with continuous
 * batching (the paper converts each frame independently, Section 5, so a
 * stream's device state is its buffers only).
 *
 * pstereo_server_create(device, hbm_budget_bytes, max_streams, lanes, policy):
 *   a server with its own context and `lanes` HIP streams (1..16, default
 *   priority).  policy PSTEREO_SERVE_BATCH forms batches of waiting frames
 *   (up to 64) and runs each as one persistent launch on an idle lane, so a
 *   batch of frames that arrived meanwhile runs while earlier ones drain;
 *   PSTEREO_SERVE_PLAIN runs the frames one at a time through the plain
 *   per-frame kernels on a single lane (the comparison baseline).  A
 *   scheduler thread owns all device work of the server.
 * pstereo_server_open_stream(s, w, h, max_disparity (-1 = 2 % of w), slots,
 *   flags, &stream_id): admits a stream if its device state fits in what is
 *   left of the HBM budget (else PSTEREO_E_NOMEM): `slots` (1..64) slots of
 *   per-frame scratch (block tables + filtered depth, w*h bytes), each also
 *   holding the frame and the three output images (12*w*h bytes) with
 *   PSTEREO_STREAM_HOST_IO.  Frames of a stream run in at most `slots`
 *   requests at once; more wait in the stream's queue (up to 256; beyond
 *   that submit returns PSTEREO_E_BUSY).  Under PSTEREO_SERVE_BATCH the
 *   width must be divisible by 4 (PSTEREO_E_UNSUPPORTED otherwise).
 * pstereo_server_submit(s, stream_id, frame, out_left, out_right,
 *   out_anaglyph, &req_id): queues one frame of the stream's size.  Without
 *   PSTEREO_STREAM_HOST_IO every buffer is device memory of the server's GPU,
 *   4-byte aligned under the batch policy; with it every buffer is host
 *   memory (pinned memory makes the copies asynchronous), staged through the
 *   stream's slots.  The caller keeps the buffers valid and untouched until
 *   the request's completion is reported; outputs may be NULL.
 * pstereo_server_poll(s, out, max, &n, wait_us): takes up to `max`
 *   completions (request id, stream, status, host times of submit, launch and
 *   observed completion in seconds since create), waiting up to wait_us
 *   microseconds for the first.
 * pstereo_server_drain(s): waits until every submitted request has completed.
 * pstereo_server_close_stream(s, id): waits for the stream's requests, frees
 *   its slots and returns their bytes to the budget.
 * pstereo_server_info(s, &budget, &in_use, &submitted, &completed).
 * pstereo_server_destroy(s): completes all submitted requests, then frees.
 * A server is thread-safe: any host thread may submit and poll.
 */
#define PSTEREO_SERVE_BATCH 0
#define PSTEREO_SERVE_PLAIN 1
#define PSTEREO_STREAM_HOST_IO 0x1u

typedef struct pstereo_completion {
    uint64_t req_id;
    int32_t stream_id;
    int32_t status;      /* PSTEREO_OK or the failure's code */
    double t_submit;     /* host seconds since pstereo_server_create */
    double t_launch;
    double t_done;
} pstereo_completion;

typedef struct pstereo_server pstereo_server;
int pstereo_server_create(int device, int64_t hbm_budget_bytes, int max_streams, int lanes, int policy,
                          pstereo_server **out);
int pstereo_server_open_stream(pstereo_server *s, int w, int h, int max_disparity, int slots, uint32_t flags,
                               int *stream_id);
int pstereo_server_close_stream(pstereo_server *s, int stream_id);
int pstereo_server_submit(pstereo_server *s, int stream_id, const uint8_t *frame, uint8_t *out_left,
                          uint8_t *out_right, uint8_t *out_anaglyph, uint64_t *req_id);
int pstereo_server_poll(pstereo_server *s, pstereo_completion *out, int max, int *n_out, int wait_us);
int pstereo_server_drain(pstereo_server *s);
int pstereo_server_info(const pstereo_server *s, int64_t *budget, int64_t *in_use, uint64_t *submitted,
                        uint64_t *completed);
int pstereo_server_destroy(pstereo_server *s);
const char *pstereo_server_last_error(const pstereo_server *s);

#ifdef __cplusplus
}
#endif
#endif /* PSTEREO_H */
