"""Benchmark: 4K stereo frames/s of the pseudo-stereo pipeline on one MI355X.

One step = one 3840x2160 RGB24 frame through the whole per-frame pipeline
(block statistics, region grouping, raw depth and cross-bilateral filter, both
warps with hole fill and the anaglyph) with inputs already resident in HBM.
Prints ONE JSON line with throughput, the HBM roofline fraction of the
dominant kernel -- the warp, which moves the path's algorithmic bytes (HIP
events on the launch stream, inside the timed region) -- and the CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "4K stereo frames/s + % HBM roofline; p99 frame latency (served vs plain)"
HBM_PEAK_GBS = 8000.0
BYTES_PER_PX = 12  # 3 B read (RGB24) + 9 B written (left, right, anaglyph)
KERNELS = ["k_blockstats", "k_regions", "k_cbf", "k_warp"]
# Algorithmic bytes per pixel charged to each kernel: the frame read and the
# three output images; intermediates (block tables, the filtered-depth byte)
# are not counted.
KERNEL_BYTES_PER_PX = {"k_blockstats": 3, "k_regions": 0, "k_cbf": 3, "k_warp": 12}


def _kernel_source_sha() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2009_09501_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if there is none for the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = data.get(f"{kernel}@{workload}")
    if not rec or rec.get("source_sha") != _kernel_source_sha():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(frames, B, budget_s: float = 12.0, max_frames: int = 60):
    """The oracle as it stands (single thread, plain C) on a bounded sample."""
    import oracle
    oracle.load()
    n, t0 = 0, time.perf_counter()
    while n < max_frames and (n == 0 or time.perf_counter() - t0 < budget_s):
        oracle.synthesize_views(frames[n % len(frames)], B)
        n += 1
    dt = time.perf_counter() - t0
    return {"value": round(n / dt, 4), "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} 3840x2160 frames of the same workload, full pipeline, one thread, {dt:.1f} s"}


def _pct(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, int(q * len(xs)))]


def video_leg(torch, synth, ctx, steps: int, warmup: int, bank: int):
    """4K moving-ellipse video through the replayed kernel graphs: a bank of
    ``bank`` frames spread over the 300-frame clip, cycled."""
    from paper_2009_09501_amd import pstereo_params_init
    from paper_2009_09501_amd.pstereo import pstereo_video_begin, pstereo_video_end, pstereo_video_frame
    W, H = 3840, 2160
    spec = synth.VideoSpec(4, W, H, frames=300, n=40, sigma=3.0)
    ts = [round(i * 299 / max(bank - 1, 1)) for i in range(bank)]
    dev = torch.device("cuda:0")
    frames = [torch.from_numpy(spec.frame(t)).to(dev) for t in ts]
    outs = [torch.empty_like(frames[0]) for _ in range(3)]
    stream = torch.cuda.current_stream(dev)
    p = pstereo_params_init(max_disparity=synth.default_disparity(W))
    p.stream = stream.cuda_stream
    v = pstereo_video_begin(ctx.handle, W, H, p)
    try:
        for i in range(warmup):
            pstereo_video_frame(v, frames[i % bank], *outs)
        # per-frame GPU time on every 8th frame only: an event record costs
        # stream time, as in the plain leg
        sampled = list(range(0, steps, 8))
        ev = {i: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for i in sampled}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            if i in ev:
                ev[i][0].record(stream)
            pstereo_video_frame(v, frames[i % bank], *outs)
            if i in ev:
                ev[i][1].record(stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        pstereo_video_end(v)
    lat = [a.elapsed_time(b) for a, b in ev.values()]
    return {"fps": round(steps / dt, 2), "ms_per_frame": round(dt / steps * 1e3, 4),
            "frame_gpu_ms": {"p50": round(_pct(lat, 0.5), 4), "p99": round(_pct(lat, 0.99), 4)},
            "pipeline_hbm_frac": round(BYTES_PER_PX * W * H * steps / dt / 1e9 / HBM_PEAK_GBS, 4),
            "frames": f"VideoSpec(seed 4, 3840x2160, 300 frames, 40 ellipses, sigma 3) frames {ts} cycled"}


def batch_leg(torch, synth, ctx, steps: int, warmup: int, distinct: int):
    """64 frames of uneven size (the seeded 720p..8K mix) in one persistent
    launch, prepared once and launched ``steps`` times."""
    from paper_2009_09501_amd import pstereo_params_init
    from paper_2009_09501_amd.pstereo import (make_jobs, pstereo_batch_autotune, pstereo_batch_create,
                                              pstereo_batch_destroy, pstereo_batch_launch)
    sizes = synth.batch_mix_sizes(5, 64)
    dev = torch.device("cuda:0")
    bank = {}
    frames = []
    for i, (w, h) in enumerate(sizes):
        lst = bank.setdefault((w, h), [])
        if len(lst) < distinct:
            lst.append(torch.from_numpy(synth.gen_frame(10000 + i, w, h, 40, 4.0)).to(dev))
            frames.append(lst[-1])
        else:
            frames.append(lst[i % distinct])
    outs = [[torch.empty_like(f) for _ in range(3)] for f in frames]
    px = sum(w * h for w, h in sizes)
    stream = torch.cuda.current_stream(dev)
    b = pstereo_batch_create(ctx.handle, len(frames), px)
    try:
        p = pstereo_params_init()
        p.stream = stream.cuda_stream
        best, best_ms, trials = pstereo_batch_autotune(b, make_jobs(frames, outs), len(frames), p, reps=2)
        for _ in range(warmup):
            pstereo_batch_launch(b, stream)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record(stream)
        for i in range(steps):
            pstereo_batch_launch(b, stream)
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        torch.cuda.synchronize()
        pstereo_batch_destroy(b)
    lat = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    mps = px * steps / dt / 1e6
    return {"frames_per_s": round(len(frames) * steps / dt, 2),
            "megapixels_per_s": round(mps, 1),
            "fps_4k_equivalent": round(mps / (3840 * 2160 / 1e6), 2),
            "ms_per_batch": round(dt / steps * 1e3, 4),
            "batch_gpu_ms": {"p50": round(_pct(lat, 0.5), 4), "p99": round(_pct(lat, 0.99), 4)},
            "pipeline_hbm_frac": round(BYTES_PER_PX * px * steps / dt / 1e9 / HBM_PEAK_GBS, 4),
            "autotune": {"best": best, "best_ms": round(best_ms, 4),
                         "trials": [dict(t, ms=round(t["ms"], 4)) for t in trials]},
            "frames": f"64 frames, batch_mix_sizes(seed 5) = {px / 1e6:.1f} MP, "
                      f"{distinct} distinct gen_frame inputs per resolution"}


SERVE_SIZES = [(1920, 1080), (3840, 2160), (7680, 4320)]


def _serve_run(torch, srv_mod, policy, streams, banks, arrivals, slots, lanes, closed_loop):
    """Feed one server the arrival schedule (or, closed_loop, everything at
    once) and return per-request latencies and the span."""
    import numpy as np
    m = srv_mod
    dev = torch.device("cuda:0")
    srv = m.pstereo_server_create(0, 32 << 30, len(streams), lanes, policy)
    try:
        sids, rings = [], []
        for (w, h, fps) in streams:
            sids.append(m.pstereo_server_open_stream(srv, w, h, -1, slots))
            rings.append([[torch.empty((h, w, 3), dtype=torch.uint8, device=dev) for _ in range(3)]
                          for _ in range(2 * slots)])
        torch.cuda.synchronize()
        # warm-up: one frame per stream
        for i, (w, h, _) in enumerate(streams):
            m.pstereo_server_submit(srv, sids[i], banks[(w, h)][0], *rings[i][0])
        m.pstereo_server_drain(srv)
        m.pstereo_server_poll(srv, 4096)
        count = [0] * len(streams)
        t0 = time.perf_counter()
        base = None
        for t, i in arrivals:
            if not closed_loop:
                while True:
                    d = t - (time.perf_counter() - t0)
                    if d <= 0:
                        break
                    time.sleep(min(d, 0.0005) if d > 0.0005 else 0)
            k = count[i]
            count[i] += 1
            w, h, _ = streams[i]
            rid = m.pstereo_server_submit(srv, sids[i], banks[(w, h)][k % len(banks[(w, h)])],
                                          *rings[i][k % len(rings[i])])
            if base is None:
                base = rid
        m.pstereo_server_drain(srv)
        span = time.perf_counter() - t0
        done = m.pstereo_server_poll(srv, 1 << 16)
    finally:
        m.pstereo_server_destroy(srv)
    lat = {}
    for c in done:
        w, h, _ = streams[c["stream_id"]]
        lat.setdefault(f"{w}x{h}", []).append((c["t_done"] - c["t_submit"]) * 1e3)
    allv = np.concatenate([np.asarray(v) for v in lat.values()])
    out = {"frames": int(allv.size), "span_s": round(span, 3), "frames_per_s": round(allv.size / span, 1),
           "latency_ms": {"p50": round(float(np.percentile(allv, 50)), 3),
                          "p99": round(float(np.percentile(allv, 99)), 3)},
           "latency_ms_by_size": {k: {"p50": round(float(np.percentile(v, 50)), 3),
                                      "p99": round(float(np.percentile(v, 99)), 3), "n": len(v)}
                                  for k, v in sorted(lat.items())}}
    px = sum(streams[c["stream_id"]][0] * streams[c["stream_id"]][1] for c in done)
    out["fps_4k_equivalent"] = round(px / (3840 * 2160) / span, 1)
    return out


def serve_leg(torch, synth, duration_s: float, burst: int):
    """Eight synthetic video streams (1080p / 4K / 8K, Poisson arrivals at 30
    or 60 frames/s each) through the continuous-batching server and through the
    plain one-frame-at-a-time policy; then a closed-loop burst of ``burst``
    frames per stream (everything submitted at once) for capacity."""
    import numpy as np

    from paper_2009_09501_amd import pstereo as m
    rng = np.random.default_rng(8)
    streams = []
    for i in range(8):
        w, h = SERVE_SIZES[int(rng.integers(0, 3))]
        streams.append((w, h, int(rng.choice([30, 60]))))
    dev = torch.device("cuda:0")
    banks = {}
    for w, h, _ in streams:
        if (w, h) not in banks:
            spec = synth.VideoSpec(20 + w, w, h, frames=300, n=40, sigma=3.0)
            banks[(w, h)] = [torch.from_numpy(spec.frame(t)).to(dev) for t in (0, 150)]
    arrivals = []
    for i, (_, _, fps) in enumerate(streams):
        arrivals += [(float(t), i) for t in synth.poisson_arrivals(100 + i, fps, duration_s)]
    arrivals.sort()
    burst_arr = [(0.0, i) for k in range(burst) for i in range(len(streams))]
    res = {"streams": [f"{w}x{h}@{fps}" for w, h, fps in streams], "duration_s": duration_s,
           "hbm_budget_bytes": 32 << 30}
    for name, pol, lanes in (("served", m.PSTEREO_SERVE_BATCH, 4), ("plain", m.PSTEREO_SERVE_PLAIN, 1)):
        res[name] = _serve_run(torch, m, pol, streams, banks, arrivals, 4, lanes, False)
        res[name + "_burst"] = _serve_run(torch, m, pol, streams, banks, burst_arr, 4, lanes, True)
    return res


def host_leg(torch, synth, frames_n: int, lanes: int):
    """End to end from pinned host memory: 4K frames uploaded, converted and
    the three views downloaded, (i) through the server's host-I/O streams, whose
    lanes overlap one frame's copies with another's compute, and (ii) one frame
    at a time (copy in, convert, copy out, wait) for comparison."""
    from paper_2009_09501_amd import Context
    from paper_2009_09501_amd import pstereo as m
    W, H = 3840, 2160
    spec = synth.VideoSpec(4, W, H, frames=300, n=40, sigma=3.0)
    bank = [torch.from_numpy(spec.frame(t)).pin_memory() for t in (0, 150)]
    ring = 8
    outs = [[torch.empty((H, W, 3), dtype=torch.uint8).pin_memory() for _ in range(3)] for _ in range(ring)]
    res = {"frames": frames_n, "lanes": lanes, "bytes_per_frame": {"h2d": W * H * 3, "d2h": 3 * W * H * 3}}
    srv = m.pstereo_server_create(0, 8 << 30, 1, lanes, m.PSTEREO_SERVE_BATCH)
    try:
        sid = m.pstereo_server_open_stream(srv, W, H, -1, ring // 2, m.PSTEREO_STREAM_HOST_IO)
        m.pstereo_server_submit(srv, sid, bank[0], *outs[0])
        m.pstereo_server_drain(srv)
        m.pstereo_server_poll(srv, 64)
        t0 = time.perf_counter()
        inflight, finished = [], set()
        for k in range(frames_n):
            if len(inflight) == ring:
                # the buffers of request k - ring are reused: wait for it
                while inflight[0] not in finished:
                    finished |= {c["req_id"] for c in m.pstereo_server_poll(srv, 64, wait_us=200)}
                finished.discard(inflight.pop(0))
            inflight.append(m.pstereo_server_submit(srv, sid, bank[k % 2], *outs[k % ring]))
        m.pstereo_server_drain(srv)
        dt = time.perf_counter() - t0
    finally:
        m.pstereo_server_destroy(srv)
    res["overlapped_fps"] = round(frames_n / dt, 1)
    # one frame at a time on one stream
    dev = torch.device("cuda:0")
    ctx = Context(0, W, H)
    dfr = torch.empty((H, W, 3), dtype=torch.uint8, device=dev)
    dout = [torch.empty_like(dfr) for _ in range(3)]
    st = torch.cuda.current_stream(dev)
    B = synth.default_disparity(W)
    n2 = max(frames_n // 2, 4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n2):
        dfr.copy_(bank[k % 2], non_blocking=True)
        ctx.synthesize(dfr, out=dout, stream=st, max_disparity=B)
        for o, hbuf in zip(dout, outs[k % ring]):
            hbuf.copy_(o, non_blocking=True)
        st.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    res["serial_fps"] = round(n2 / dt, 1)
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # steady state: a 30-step warm-up left part of the clock and launch-queue
    # ramp inside the timed region (about 7 % below the rate of a longer run)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--frames", type=int, default=4, help="distinct synthetic frames cycled")
    ap.add_argument("--profile-every", type=int, default=16,
                    help="record per-stage HIP events on every N-th timed step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="video,batch,serve,host",
                    help="extra launch forms measured after the plain path (video, batch, serve, host; "
                         "empty = none)")
    ap.add_argument("--host-frames", type=int, default=120)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run device copies of MIB MiB (to scale HBM byte counters)")
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--serve-burst", type=int, default=16)
    ap.add_argument("--form-steps", type=int, default=60)
    ap.add_argument("--video-bank", type=int, default=8)
    ap.add_argument("--batch-distinct", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(frames and streams shard across GPUs with no exchange; see the design notes)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.calibrate_copy:
        # device-to-device copies of a known size, larger than the 256 MB
        # Infinity Cache: a kernel whose HBM traffic is known (read n + write n)
        n = args.calibrate_copy << 20
        src = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": n, "bytes_written": n, "launches": 10}), flush=True)
        return 0

    import synth
    from paper_2009_09501_amd import PSTEREO_PROFILE, Context, pstereo_profile_collect

    W, H = 3840, 2160
    B = synth.default_disparity(W)
    seeds = [3 + 100 * i for i in range(args.frames)]
    host = [synth.gen_frame(s, W, H, 40, 4.0) for s in seeds]
    dev = torch.device("cuda:0")
    frames = [torch.from_numpy(f).to(dev) for f in host]
    outs = [torch.empty_like(frames[0]) for _ in range(3)]
    ctx = Context(0, W, H)
    # a stream of our own (default priority): torch's current stream would
    # otherwise be the NULL stream, which the library maps to its own stream
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    params = dict(max_disparity=B)

    for i in range(args.warmup):
        ctx.synthesize(frames[i % len(frames)], out=outs, stream=stream, **params)
    torch.cuda.synchronize()
    pstereo_profile_collect(ctx.handle)  # clear
    # what an event pair adds to the kernel it brackets, subtracted from the
    # event-bracketed stage durations: a pair around one tiny kernel, less
    # that kernel's share of a long back-to-back run of it (one pair around
    # 256 launches)
    tiny = torch.zeros(1, dtype=torch.int32, device=dev)
    for _ in range(16):
        tiny.fill_(1)
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(64)]
    for a, b in pairs:
        a.record(stream)
        tiny.fill_(1)
        b.record(stream)
    run0, run1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    run0.record(stream)
    for _ in range(256):
        tiny.fill_(1)
    run1.record(stream)
    torch.cuda.synchronize()
    ev_overhead_ms = max(statistics.median(a.elapsed_time(b) for a, b in pairs) - run0.elapsed_time(run1) / 256,
                         0.0)

    # per-stage HIP events on every `sample`-th timed step: each event record
    # adds a few microseconds of stream time, so recording them on every step
    # would slow the throughput being measured
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        fl = PSTEREO_PROFILE if i % args.profile_every == 0 else 0
        ctx.synthesize(frames[i % len(frames)], out=outs, stream=stream, flags=fl, **params)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_sum, count, per_call = pstereo_profile_collect(ctx.handle)

    fps = args.steps / dt
    px = W * H
    kern_s = {k: ms_sum[i] / count / 1e3 for i, k in enumerate(KERNELS)}
    # the roofline kernel: the one that moves the path's algorithmic bytes
    # (the warp: frame in, three views out).  The depth filter runs about as
    # long but is bound by VALU issue, not HBM (SQ counters in profiles/);
    # the longest stage is reported beside it
    dom = "k_warp"
    longest = max(kern_s, key=kern_s.get)
    dom_s = max(kern_s[dom] - ev_overhead_ms / 1e3, 1e-9)
    achieved = KERNEL_BYTES_PER_PX[dom] * px / dom_s / 1e9
    pipe_s = sum(ms_sum) / count / 1e3
    lat = sorted(per_call)
    traffic = _traffic(dom, "4k")

    out = {
        "metric": METRIC,
        "value": round(fps, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "4K 3840x2160 RGB24 single frames, plain per-frame launch "
                               "(blockstats, regions, cbf, warp), max disparity 77 px",
                   "frames": f"gen_frame seeds {seeds}, 40 shapes, noise sigma 4",
                   "path": "plain"},
        "roofline": {"bound": "hbm", "kernel": dom,
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "duration_us": round(dom_s * 1e6, 3), "event_overhead_us": round(ev_overhead_ms * 1e3, 3),
                     "bytes_per_launch": KERNEL_BYTES_PER_PX[dom] * px,
                     "longest_kernel": longest},
        "kernels_ms": {k: round(v * 1e3, 5) for k, v in kern_s.items()},
        "kernels_hbm_frac": {k: round(KERNEL_BYTES_PER_PX[k] * px / v / 1e9 / HBM_PEAK_GBS, 4)
                             for k, v in kern_s.items()},
        "pipeline_hbm_frac": round(BYTES_PER_PX * px / pipe_s / 1e9 / HBM_PEAK_GBS, 4),
        "latency_ms": {"p50": round(statistics.median(lat), 4),
                       "p99": round(lat[min(len(lat) - 1, int(0.99 * len(lat)))], 4)},
    }
    forms = [f for f in args.forms.split(",") if f]
    if forms:
        out["forms"] = {}
    if "video" in forms:
        out["forms"]["video_graph_4k"] = video_leg(torch, synth, ctx, args.form_steps * 5, 10, args.video_bank)
    if "batch" in forms:
        out["forms"]["batch_uneven_64"] = batch_leg(torch, synth, ctx, args.form_steps, 3, args.batch_distinct)
    if "serve" in forms:
        out["forms"]["serve_8_streams"] = serve_leg(torch, synth, args.serve_seconds, args.serve_burst)
    if "host" in forms:
        out["forms"]["host_pinned_4k"] = host_leg(torch, synth, args.host_frames, 3)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(host, B)
    ctx.close()
    print(json.dumps(out), flush=True)
    _ = np
    return 0


if __name__ == "__main__":
    sys.exit(main())
