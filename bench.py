"""Benchmark: 4K stereo frames/s of the pseudo-stereo pipeline on one MI355X.

One step = one 3840x2160 RGB24 frame through the whole per-frame pipeline
(block statistics, region grouping, raw depth and cross-bilateral filter, both
warps with hole fill and the anaglyph) with inputs already resident in HBM:
one launch sequence per frame in three pipelined stages: the depth-map stages
of frame i+2 on the context's second stream and the depth filter of frame i+1
on its third while frame i is warped (PSTEREO_PIPELINE_DEEP; --stages 2 keeps
the filter with the warp, --serial pipelines nothing).  Prints ONE JSON line with throughput, the HBM roofline
fraction of the kernel that moves the path's algorithmic bytes (the warp; its
duration from its own dispatch timestamps, HIP events taken by the launch
itself over the timed region), the whole-path roofline fraction, latency from
a separate loop of single frames, the 1080p rate, the other launch forms, and
the CPU oracle timed on a bounded sample of the same workloads.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "4K stereo frames/s + % HBM roofline; p99 frame latency (served vs plain)"
HBM_PEAK_GBS = 8000.0
BYTES_PER_PX = 12  # 3 B read (RGB24) + 9 B written (left, right, anaglyph)
STAGES = ["k_blockstats", "k_regions", "k_cbf", "k_warp"]
# Algorithmic bytes per pixel charged to each stage: the frame read and the
# three output images; intermediates (block tables, the filtered-depth byte)
# are not counted.
STAGE_BYTES_PER_PX = {"k_blockstats": 3, "k_regions": 0, "k_cbf": 3, "k_warp": 12}
# Host threads for generating inputs and for the oracle's row-parallel mode:
# the CPUs this process may run on, at most 16 (one GPU's share of the host).
HOST_THREADS = max(1, min(16, len(os.sched_getaffinity(0))))
PATHS = {1: "plain, serial (one stream)",
         2: ("plain, pipelined: frame i+1's block statistics and region grouping on the context's second "
             "stream during frame i's filter and warp (PSTEREO_PIPELINE)"),
         3: ("plain, three-stage pipelined: frame i+2's block statistics and region grouping on the "
             "context's second stream and frame i+1's filter on its third during frame i's warp "
             "(PSTEREO_PIPELINE_DEEP)")}
WORKLOADS = {1: "4k_serial", 2: "4k_pipelined", 3: "4k_pipelined3"}


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
    rec = _profile_record("traffic.json", f"{kernel}@{workload}")
    return rec.get("bytes_per_launch") if rec else None


def _profile_record(name: str, key: str):
    """One entry of a committed rocprofv3 summary (profiles/<name>.json) for
    the current kernel sources, or None (absent, or taken from other
    sources)."""
    try:
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            rec = json.load(fh).get(key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha") != _kernel_source_sha():
        return None
    return rec


def _short_kernel(name: str) -> str:
    """k_warp from 'void pstereo::k_warp<true, 2>(pstereo::FrameDesc)'."""
    base = name.split("(")[0].split("<")[0].replace("void ", "").strip()
    return base.split("::")[-1]


def summarize_trace(csv_dir: str, workload: str) -> None:
    """Record the mean kernel durations of a rocprofv3 --kernel-trace --stats
    run (DIR/run_kernel_stats.csv) in profiles/kernels.json under
    <kernel>@<workload>, with the kernel sources' hash, and print them."""
    import csv
    path = os.path.join(ROOT, "profiles", "kernels.json")
    try:
        data = json.load(open(path))
    except (OSError, ValueError):
        data = {}
    sha = _kernel_source_sha()
    rows = []
    for r in csv.DictReader(open(os.path.join(csv_dir, "run_kernel_stats.csv"))):
        if "pstereo" not in r["Name"]:
            continue
        k = _short_kernel(r["Name"])
        avg = float(r["AverageNs"]) / 1e3
        key = f"{k}@{workload}"
        data[key] = {"avg_us": round(avg, 3), "calls": int(r["Calls"]), "min_us": round(float(r["MinNs"]) / 1e3, 3),
                     "max_us": round(float(r["MaxNs"]) / 1e3, 3), "source_sha": sha}
        rows.append((k, int(r["Calls"]), avg))
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    for k, n, avg in rows:
        print(f"| `{k}` | {n} | {avg:.2f} |")


def summarize_traffic(fetch_dir: str, write_dir: str, workload: str, fetch_factor: float,
                      write_factor: float) -> None:
    """Record HBM bytes per dispatch from two rocprofv3 --pmc runs (FETCH_SIZE,
    WRITE_SIZE; KiB per dispatch, medians per kernel) scaled by the copy
    calibration's factors, in profiles/traffic.json under <kernel>@<workload>."""
    import csv
    import statistics as st
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        data = json.load(open(path))
    except (OSError, ValueError):
        data = {}

    def med(d, counter):
        vals = {}
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            if r["Counter_Name"] == counter and "pstereo" in r["Kernel_Name"]:
                vals.setdefault(_short_kernel(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
        return {k: st.median(v) for k, v in vals.items()}
    fetch, write = med(fetch_dir, "FETCH_SIZE"), med(write_dir, "WRITE_SIZE")
    sha = _kernel_source_sha()
    for k in sorted(set(fetch) & set(write)):
        rd = fetch[k] * 1024 * fetch_factor
        wr = write[k] * 1024 * write_factor
        data[f"{k}@{workload}"] = {"read_bytes": int(rd), "write_bytes": int(wr), "bytes_per_launch": int(rd + wr),
                                   "fetch_factor": fetch_factor, "write_factor": write_factor, "source_sha": sha}
        print(f"| `{k}` | {fetch[k]:.0f} | {write[k]:.0f} | {rd / 1e6:.1f} | {wr / 1e6:.1f} |")
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)


def _pct(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, int(q * len(xs)))]


def _gen_many(fn, args):
    """fn(*a) for every a in args on the host threads (numpy releases the GIL
    in the array work), in order."""
    with ThreadPoolExecutor(HOST_THREADS) as ex:
        return list(ex.map(lambda a: fn(*a), args))


# ----------------------------------------------------------------- CPU oracle
def cpu_baseline(budget_s: float = 4.0):
    """The oracle as it stands (plain C, -O2) on the host cores of this run:
    single thread and row-parallel over HOST_THREADS threads (the
    row-independent stages split into row bands; outputs asserted equal to
    the single-thread ones), on the seeded inputs of each workload: 640x360
    (B = 12), 1080p (B = 38) and 4K (B = 77) stills, and three frames of the
    4K video (extrapolated to its 300 frames).  ``value`` is the 4K
    row-parallel rate."""
    import numpy as np

    import oracle
    import synth
    oracle.load()
    nt = HOST_THREADS

    def timed(fn, frames, B, budget):
        n, t0 = 0, time.perf_counter()
        while n < len(frames) * 4 and (n < len(frames) or time.perf_counter() - t0 < budget):
            fn(frames[n % len(frames)], B)
            n += 1
        return n, time.perf_counter() - t0

    work = {
        "640x360": ([synth.gen_frame(1, 640, 360, 12, 4.0)], 12),
        "1920x1080": ([synth.gen_frame(2, 1920, 1080, 40, 4.0)], 38),
        "3840x2160": ([synth.gen_frame(3, 3840, 2160, 40, 4.0)], 77),
    }
    spec = synth.VideoSpec(4, 3840, 2160, frames=300, n=40, sigma=3.0)
    video = _gen_many(spec.frame, [(t,) for t in (0, 149, 299)])
    res = {}
    for name, (frames, B) in work.items():
        st = oracle.synthesize_views(frames[0], B)
        mt = oracle.synthesize_views_mt(frames[0], B, nt)
        assert all(np.array_equal(a, b) for a, b in zip(st, mt)), f"{name}: threaded oracle differs"
        n1, t1 = timed(oracle.synthesize_views, frames, B, budget_s / 2)
        nm, tm = timed(lambda f, b: oracle.synthesize_views_mt(f, b, nt), frames, B, budget_s / 2)
        res[name] = {"B": B, "single_thread_fps": round(n1 / t1, 4), "single_thread_frames": n1,
                     f"threads_{nt}_fps": round(nm / tm, 4), f"threads_{nt}_frames": nm}
    t0 = time.perf_counter()
    for f in video:
        oracle.synthesize_views(f, 77)
    v1 = (time.perf_counter() - t0) / len(video)
    t0 = time.perf_counter()
    for f in video:
        oracle.synthesize_views_mt(f, 77, nt)
    vm = (time.perf_counter() - t0) / len(video)
    res["video_4k_300"] = {"frames_timed": [0, 149, 299], "extrapolated": True,
                           "single_thread_s_per_clip": round(v1 * 300, 2),
                           f"threads_{nt}_s_per_clip": round(vm * 300, 2)}
    k4 = res["3840x2160"]
    return {"value": k4[f"threads_{nt}_fps"], "unit": "frames/s", "cores": nt, "kind": "oracle",
            "single_thread_value": k4["single_thread_fps"],
            "sample": (f"whole frames through the oracle (all stages), single thread and {nt} threads "
                       f"(row bands), outputs equal; 640x360, 1080p and 4K stills (gen_frame seeds 1, 2, 3) "
                       f"for about {budget_s / 2:.0f} s each, and 3 frames of the 4K video extrapolated to 300"),
            "workloads": res}


# ------------------------------------------------------------- plain path
def plain_run(torch, ctx, stream, frames, outs, B, steps, warmup, prewarm_s, every, stages):
    """`warmup` untimed steps (after `prewarm_s` seconds of the same work to
    bring the clocks up), then `steps` timed steps bracketed by device
    synchronisation, every `every`-th of them (0 = none) with each kernel's
    dispatch timestamps recorded (a profiled launch costs the stream some
    time, so not every step is profiled).  Returns (seconds, per-stage mean
    ms over the profiled steps or None, their count).  stages: 1 = serial
    calls, 2 = PSTEREO_PIPELINE, 3 = PSTEREO_PIPELINE_DEEP."""
    from paper_2009_09501_amd import PSTEREO_PROFILE, pstereo_profile_collect
    from paper_2009_09501_amd.pstereo import PSTEREO_PIPELINE, PSTEREO_PIPELINE_DEEP
    base = {1: 0, 2: PSTEREO_PIPELINE, 3: PSTEREO_PIPELINE_DEEP}[stages]
    nf, no = len(frames), len(outs)
    # one profiled call first: the library creates its profiling events on
    # the first profiled call, which must not fall in the timed region
    ctx.synthesize(frames[0], out=outs[0], stream=stream, flags=base | PSTEREO_PROFILE, max_disparity=B)
    t_end = time.perf_counter() + prewarm_s
    i = 0
    while time.perf_counter() < t_end:
        ctx.synthesize(frames[i % nf], out=outs[i % no], stream=stream, flags=base, max_disparity=B)
        i += 1
        if i % 64 == 0:
            stream.synchronize()
    for i in range(warmup):
        ctx.synthesize(frames[i % nf], out=outs[i % no], stream=stream, flags=base | PSTEREO_PROFILE,
                       max_disparity=B)
    torch.cuda.synchronize()
    pstereo_profile_collect(ctx.handle)  # clear
    prof = base | PSTEREO_PROFILE
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # the profiled steps sit mid-stride: a profiled call costs the host more,
    # which the GPU only sees while the host is not yet ahead of it (as at the
    # first step, right after the synchronisation)
    mid = min(every // 2, (steps - 1) // 2) if steps > 0 else 0
    for i in range(steps):
        fl = prof if every and i % every == mid else base
        ctx.synthesize(frames[i % nf], out=outs[i % no], stream=stream, flags=fl, max_disparity=B)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if not every:
        return dt, None, 0
    ms_sum, count, _ = pstereo_profile_collect(ctx.handle, cap=1)
    return dt, [m / max(count, 1) for m in ms_sum], count


def latency_run(torch, ctx, stream, frames, outs, B, samples):
    """Each frame alone on an idle stream: GPU time from the first kernel's
    start to the last kernel's stop, and host time from the call to the end
    of the stream synchronisation."""
    from paper_2009_09501_amd import PSTEREO_PROFILE, pstereo_profile_collect
    torch.cuda.synchronize()
    pstereo_profile_collect(ctx.handle)
    host = []
    for i in range(samples):
        t0 = time.perf_counter()
        ctx.synthesize(frames[i % len(frames)], out=outs[i % len(outs)], stream=stream, flags=PSTEREO_PROFILE,
                       max_disparity=B)
        stream.synchronize()
        host.append((time.perf_counter() - t0) * 1e3)
    _, count, per = pstereo_profile_collect(ctx.handle, cap=samples)
    return {"samples": count, "gpu_ms": {"p50": round(_pct(per, 0.5), 4), "p99": round(_pct(per, 0.99), 4)},
            "host_ms": {"p50": round(_pct(host, 0.5), 4), "p99": round(_pct(host, 0.99), 4)},
            "what": "one frame alone on an idle stream; gpu = first kernel start to last kernel stop, "
                    "host = call to stream synchronised"}


def plain_leg(torch, synth, W, H, B, n_frames, n_outs, steps, warmup, prewarm_s, every, stages, seed0):
    """Frames/s, per-stage kernel times and roofline figures of the plain
    path at W x H over n_frames distinct inputs and n_outs output triples."""
    from paper_2009_09501_amd import Context
    dev = torch.device("cuda:0")
    seeds = [seed0 + 100 * i for i in range(n_frames)]
    host = _gen_many(synth.gen_frame, [(s, W, H, 40, 4.0) for s in seeds])
    frames = [torch.from_numpy(f).to(dev) for f in host]
    outs = [[torch.empty_like(frames[0]) for _ in range(3)] for _ in range(n_outs)]
    ctx = Context(0, W, H)
    stream = torch.cuda.Stream(device=dev)
    try:
        dt, stage_ms, count = plain_run(torch, ctx, stream, frames, outs, B, steps, warmup, prewarm_s, every,
                                        stages)
    finally:
        torch.cuda.synchronize()
    px = W * H
    res = {"fps": round(steps / dt, 2), "ms_per_frame": round(dt / steps * 1e3, 5), "seconds": dt,
           "working_set_MB": round((n_frames * 3 + n_outs * 9) * px / 1e6, 1),
           "frames": f"gen_frame seeds {seeds}, 40 shapes, noise sigma 4; {n_outs} output triples cycled",
           "path_hbm_frac": round(BYTES_PER_PX * px * steps / dt / 1e9 / HBM_PEAK_GBS, 4)}
    if stage_ms:
        res["stage_ms"] = {k: round(v, 5) for k, v in zip(STAGES, stage_ms)}
        res["stage_count"] = count
        ksum = sum(stage_ms)
        res["kernel_sum_us"] = round(ksum * 1e3, 3)
        res["kernel_sum_hbm_frac"] = round(BYTES_PER_PX * px / (ksum / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    return res, ctx, stream, frames, outs


# ------------------------------------------------------------------ forms
def video_clip(torch, synth, bank: int):
    """The 4K moving-ellipse clip (300 frames) resident in HBM: ``bank``
    frames spread evenly over it (all 300 when bank >= 300), generated on the
    host threads a chunk at a time and uploaded as they are made, so host
    memory holds one chunk."""
    W, H = 3840, 2160
    spec = synth.VideoSpec(4, W, H, frames=300, n=40, sigma=3.0)
    bank = max(1, min(bank, 300))
    ts = [round(i * 299 / max(bank - 1, 1)) for i in range(bank)]
    dev = torch.device("cuda:0")
    frames, chunk = [], 4 * HOST_THREADS
    for k in range(0, bank, chunk):
        frames += [torch.from_numpy(f).to(dev) for f in _gen_many(spec.frame, [(t,) for t in ts[k:k + chunk]])]
    torch.cuda.synchronize()
    return ts, frames


def video_leg(torch, synth, clip, steps: int, warmup: int, n_outs: int, stages: int):
    """4K moving-ellipse video through the replayed kernel graphs (stages 2:
    a frame's depth-map graph on the context's second stream during the
    previous frame's filter and warp; 1: one stream): the frames of ``clip`` (frame numbers,
    device frames) in order, cycled when ``steps`` exceeds them, frame i into
    output triple i % ``n_outs``."""
    from paper_2009_09501_amd import Context, pstereo_params_init
    from paper_2009_09501_amd.pstereo import pstereo_video_begin, pstereo_video_end, pstereo_video_frame
    ts, frames = clip
    bank = len(frames)
    H, W = frames[0].shape[:2]
    outs = [[torch.empty_like(frames[0]) for _ in range(3)] for _ in range(n_outs)]
    ctx = Context(0, W, H)
    stream = torch.cuda.Stream(device=frames[0].device)
    from paper_2009_09501_amd.pstereo import PSTEREO_PIPELINE
    p = pstereo_params_init(max_disparity=synth.default_disparity(W), flags=PSTEREO_PIPELINE if stages == 2 else 0)
    p.stream = stream.cuda_stream
    v = pstereo_video_begin(ctx.handle, W, H, p)
    try:
        for i in range(warmup):
            pstereo_video_frame(v, frames[i % bank], *outs[i % n_outs])
        # per-frame GPU time on every 8th frame only (an event pair costs
        # stream time)
        sampled = list(range(0, steps, 8))
        ev = {i: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for i in sampled}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            if i in ev:
                ev[i][0].record(stream)
            pstereo_video_frame(v, frames[i % bank], *outs[i % n_outs])
            if i in ev:
                ev[i][1].record(stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        pstereo_video_end(v)
        ctx.close()
    del outs
    lat = [a.elapsed_time(b) for a, b in ev.values()]
    span = (f"the whole clip, frames 0..299 in order" if ts == list(range(300))
            else f"frames {ts} cycled")
    return {"fps": round(steps / dt, 2), "ms_per_frame": round(dt / steps * 1e3, 4), "frames_timed": steps,
            "frame_gpu_ms": {"p50": round(_pct(lat, 0.5), 4), "p99": round(_pct(lat, 0.99), 4)},
            "path_hbm_frac": round(BYTES_PER_PX * W * H * steps / dt / 1e9 / HBM_PEAK_GBS, 4),
            "stages": stages,
            "frames": f"VideoSpec(seed 4, 3840x2160, 300 frames, 40 ellipses, sigma 3), {bank} frames resident "
                      f"in HBM ({bank * W * H * 3 / 1e9:.2f} GB): {span}, into {n_outs} output triples"}


def _batch_inputs(torch, synth, sizes, seed0):
    """One distinct device frame per job: two generated frames per
    resolution, each job's a copy of one of them rolled by a seeded offset
    (distinct content and a distinct buffer for every job)."""
    import numpy as np
    dev = torch.device("cuda:0")
    uniq = sorted(set(sizes))
    args = [(seed0 + 10 * k + j, w, h, 40, 4.0) for k, (w, h) in enumerate(uniq) for j in range(2)]
    base = {}
    for a, f in zip(args, _gen_many(synth.gen_frame, args)):
        base.setdefault((a[1], a[2]), []).append(torch.from_numpy(f).to(dev))
    rng = np.random.default_rng(seed0)
    frames = []
    for i, (w, h) in enumerate(sizes):
        dy, dx = int(rng.integers(0, h)), int(rng.integers(0, w))
        frames.append(torch.roll(base[(w, h)][i % 2], shifts=(dy, dx), dims=(0, 1)).contiguous())
    return frames


def batch_leg(torch, synth, steps: int, warmup: int):
    """64 frames of uneven size (the seeded 720p..8K mix), each its own input
    buffer, autotuned, then launched ``steps`` times (the winning form)."""
    from paper_2009_09501_amd import Context, pstereo_params_init
    from paper_2009_09501_amd.pstereo import (make_jobs, pstereo_batch_autotune, pstereo_batch_create,
                                              pstereo_batch_destroy, pstereo_batch_launch)
    sizes = synth.batch_mix_sizes(5, 64)
    frames = _batch_inputs(torch, synth, sizes, 10000)
    outs = [[torch.empty_like(f) for _ in range(3)] for f in frames]
    px = sum(w * h for w, h in sizes)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    ctx = Context(0, 64, 64)
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
        ctx.close()
    lat = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    mps = px * steps / dt / 1e6
    return {"form": "staged" if best["mode"] == 0 else "fused",
            "frames_per_s": round(len(frames) * steps / dt, 2),
            "megapixels_per_s": round(mps, 1),
            "fps_4k_equivalent": round(mps / (3840 * 2160 / 1e6), 2),
            "ms_per_batch": round(dt / steps * 1e3, 4),
            "batch_gpu_ms": {"p50": round(_pct(lat, 0.5), 4), "p99": round(_pct(lat, 0.99), 4)},
            "path_hbm_frac": round(BYTES_PER_PX * px * steps / dt / 1e9 / HBM_PEAK_GBS, 4),
            "autotune": {"best": best, "best_ms": round(best_ms, 4),
                         "trials": [dict(t, ms=round(t["ms"], 4)) for t in trials]},
            "frames": f"64 frames, batch_mix_sizes(seed 5) = {px / 1e6:.1f} MP, one input buffer per job "
                      f"(two gen_frame frames per resolution, each job's rolled by a seeded offset)"}


SERVE_SIZES = [(1920, 1080), (3840, 2160), (7680, 4320)]


def _serve_run(torch, m, policy, streams, banks, arrivals, slots, lanes, closed_loop):
    """Feed one server the arrival schedule (or, closed_loop, everything at
    once) and return per-request latencies and the span."""
    import numpy as np
    dev = torch.device("cuda:0")
    srv = m.pstereo_server_create(0, 32 << 30, len(streams), lanes, policy)
    try:
        sids, rings = [], []
        for (w, h, fps) in streams:
            sids.append(m.pstereo_server_open_stream(srv, w, h, -1, slots))
            rings.append([[torch.empty((h, w, 3), dtype=torch.uint8, device=dev) for _ in range(3)]
                          for _ in range(2 * slots)])
        torch.cuda.synchronize()
        for i, (w, h, _) in enumerate(streams):
            m.pstereo_server_submit(srv, sids[i], banks[(w, h)][0], *rings[i][0])
        m.pstereo_server_drain(srv)
        m.pstereo_server_poll(srv, 4096)
        count = [0] * len(streams)
        t0 = time.perf_counter()
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
            while True:
                rc, _ = m.pstereo_server_submit(srv, sids[i], banks[(w, h)][k % len(banks[(w, h)])],
                                                *rings[i][k % len(rings[i])], check=False)
                if rc != m.PSTEREO_E_BUSY:
                    break
                time.sleep(0.0002)
        m.pstereo_server_drain(srv)
        span = time.perf_counter() - t0
        done = m.pstereo_server_poll(srv, 1 << 17)
    finally:
        m.pstereo_server_destroy(srv)
    lat = {}
    for c in done:
        w, h, _ = streams[c["stream_id"]]
        lat.setdefault(f"{w}x{h}", []).append((c["t_done"] - c["t_submit"]) * 1e3)
    allv = np.concatenate([np.asarray(v) for v in lat.values()])
    out = {"frames": int(allv.size), "span_s": round(span, 4), "frames_per_s": round(allv.size / span, 1),
           "latency_ms": {"p50": round(float(np.percentile(allv, 50)), 3),
                          "p99": round(float(np.percentile(allv, 99)), 3)},
           "latency_ms_by_size": {k: {"p50": round(float(np.percentile(v, 50)), 3),
                                      "p99": round(float(np.percentile(v, 99)), 3), "n": len(v)}
                                  for k, v in sorted(lat.items())}}
    px = sum(streams[c["stream_id"]][0] * streams[c["stream_id"]][1] for c in done)
    out["fps_4k_equivalent"] = round(px / (3840 * 2160) / span, 1)
    return out


def serve_leg(torch, synth, duration_s: float, burst: int, compress):
    """Eight synthetic video streams (1080p / 4K / 8K, Poisson arrivals at 30
    or 60 frames/s each) through the continuous-batching server and through
    the plain one-frame-at-a-time policy: paced in real time, then with the
    same arrival schedule compressed k-fold (saturation sweep, until the
    served rate stops rising), then a closed-loop burst of ``burst`` frames
    per stream (everything submitted at once)."""
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
            banks[(w, h)] = [torch.from_numpy(f).to(dev) for f in _gen_many(spec.frame, [(t,) for t in (0, 75, 150, 225)])]
    arrivals = []
    for i, (_, _, fps) in enumerate(streams):
        arrivals += [(float(t), i) for t in synth.poisson_arrivals(100 + i, fps, duration_s)]
    arrivals.sort()
    burst_arr = [(0.0, i) for k in range(burst) for i in range(len(streams))]
    res = {"streams": [f"{w}x{h}@{fps}" for w, h, fps in streams], "duration_s": duration_s,
           "hbm_budget_bytes": 32 << 30, "slots_per_stream": 4}
    pols = (("served", m.PSTEREO_SERVE_BATCH, 4), ("plain", m.PSTEREO_SERVE_PLAIN, 1))
    for name, pol, lanes in pols:
        res[name] = _serve_run(torch, m, pol, streams, banks, arrivals, 4, lanes, False)
    sweep = []
    for k in compress:
        row = {"compress": k, "offered_fps": round(len(arrivals) * k / duration_s, 1)}
        sched = [(t / k, i) for t, i in arrivals]
        for name, pol, lanes in pols:
            r = _serve_run(torch, m, pol, streams, banks, sched, 4, lanes, False)
            row[name] = {"frames_per_s": r["frames_per_s"], "fps_4k_equivalent": r["fps_4k_equivalent"],
                         "latency_ms": r["latency_ms"], "latency_ms_by_size": r["latency_ms_by_size"]}
        sweep.append(row)
        if len(sweep) >= 2 and row["served"]["frames_per_s"] < 1.05 * sweep[-2]["served"]["frames_per_s"]:
            break
    res["saturation"] = sweep
    for name, pol, lanes in pols:
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
    bank = [torch.from_numpy(f).pin_memory() for f in _gen_many(spec.frame, [(0,), (150,)])]
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
    dev = torch.device("cuda:0")
    ctx = Context(0, W, H)
    dfr = torch.empty((H, W, 3), dtype=torch.uint8, device=dev)
    dout = [torch.empty_like(dfr) for _ in range(3)]
    st = torch.cuda.Stream(device=dev)
    B = synth.default_disparity(W)
    n2 = max(frames_n // 2, 4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n2):
        with torch.cuda.stream(st):
            dfr.copy_(bank[k % 2], non_blocking=True)
        ctx.synthesize(dfr, out=dout, stream=st, max_disparity=B)
        with torch.cuda.stream(st):
            for o, hbuf in zip(dout, outs[k % ring]):
                hbuf.copy_(o, non_blocking=True)
        st.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    res["serial_fps"] = round(n2 / dt, 1)
    return res


def inpaint_leg(torch, synth, reps: int):
    """The paper's block-iterative inpainting (PSTEREO_INPAINT_BLOCKS: Jacobi
    sweeps until one fills nothing, the host checking convergence) against
    the row fill of the hot path, at 1080p and 4K: time per frame and the
    pixels where the two fills' views differ.  There is no ground truth for
    which fill looks better (parity of the two against the oracle is in the
    tests; their quality relative to each other is unpinned)."""
    from paper_2009_09501_amd import Context
    from paper_2009_09501_amd.pstereo import PSTEREO_INPAINT_BLOCKS
    dev = torch.device("cuda:0")
    res = {}
    for (W, H, seed) in ((1920, 1080, 2), (3840, 2160, 3)):
        B = synth.default_disparity(W)
        f = torch.from_numpy(synth.gen_frame(seed, W, H, 40, 4.0)).to(dev)
        ctx = Context(0, W, H)
        st = torch.cuda.Stream(device=dev)
        out = {}
        for name, fl in (("row_fill", 0), ("block_inpaint", PSTEREO_INPAINT_BLOCKS)):
            o = [torch.empty_like(f) for _ in range(3)]
            ctx.synthesize(f, out=o, stream=st, flags=fl, max_disparity=B)
            st.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.synthesize(f, out=o, stream=st, flags=fl, max_disparity=B)
            st.synchronize()
            out[name] = ((time.perf_counter() - t0) / reps * 1e3, o)
        ctx.close()
        diff = [int((a != b).any(-1).sum().item()) for a, b in zip(out["row_fill"][1], out["block_inpaint"][1])]
        res[f"{W}x{H}"] = {"row_fill_ms": round(out["row_fill"][0], 4),
                           "block_inpaint_ms": round(out["block_inpaint"][0], 4),
                           "pixels_differing": {"left": diff[0], "right": diff[1], "anaglyph": diff[2]},
                           "frame": f"gen_frame seed {seed}, B = {B}"}
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--prewarm-ms", type=float, default=300.0,
                    help="untimed seconds*1e-3 of the same work before the warm-up steps (clock ramp)")
    ap.add_argument("--frames", type=int, default=8, help="distinct synthetic 4K frames cycled")
    ap.add_argument("--outs", type=int, default=4, help="output triples cycled")
    ap.add_argument("--profile-every", type=int, default=16,
                    help="record each kernel's dispatch timestamps on every N-th timed step (0 = never)")
    ap.add_argument("--serial", action="store_true", help="headline with serial calls (no pipelining)")
    ap.add_argument("--stages", type=int, choices=(2, 3), default=3,
                    help="pipelined headline: 2 = PSTEREO_PIPELINE, 3 = PSTEREO_PIPELINE_DEEP")
    ap.add_argument("--latency-samples", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="serial,pipelined2,pipelined3,1080p,video,batch,serve,host,inpaint",
                    help="extra measurements after the headline (serial, pipelined2, pipelined3: the plain 4K "
                         "path in the other call modes; 1080p, video, batch, serve, host, inpaint; empty = none)")
    ap.add_argument("--host-frames", type=int, default=120)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run device copies of MIB MiB (to scale HBM byte counters)")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="only record DIR/run_kernel_stats.csv (rocprofv3) in profiles/kernels.json")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="only record two rocprofv3 --pmc runs in profiles/traffic.json")
    ap.add_argument("--workload", default="4k_pipelined", help="workload name for --summarize-*")
    ap.add_argument("--fetch-factor", type=float, default=2.0)
    ap.add_argument("--write-factor", type=float, default=1.0)
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--serve-burst", type=int, default=16)
    ap.add_argument("--serve-compress", default="4,16,64,256")
    ap.add_argument("--form-steps", type=int, default=60)
    ap.add_argument("--video-bank", type=int, default=300,
                    help="frames of the 4K clip resident in HBM for the video legs (300 = the whole clip)")
    ap.add_argument("--video-outs", type=int, default=0,
                    help="output triples the video legs write (0 = one per resident frame)")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.workload)
        return 0
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic, args.workload, args.fetch_factor, args.write_factor)
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(frames and streams shard across GPUs with no exchange; see the design notes)",
              file=sys.stderr)
        return 2

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

    W, H = 3840, 2160
    B = synth.default_disparity(W)
    px = W * H
    every = args.profile_every
    stages = 1 if args.serial else args.stages
    head, ctx, stream, frames, outs = plain_leg(torch, synth, W, H, B, args.frames, args.outs, args.steps,
                                                args.warmup, args.prewarm_ms / 1e3, every, stages, 3)
    lat = latency_run(torch, ctx, stream, frames, outs, B, args.latency_samples)
    ctx.close()
    del frames, outs
    dt = head.pop("seconds")

    out = {
        "metric": METRIC,
        "value": head["fps"],
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
        "config": {"workload": "4K 3840x2160 RGB24 single frames, plain per-frame launch sequence "
                               "(blockstats, region grouping, cbf, warp), max disparity 77 px",
                   "frames": head["frames"], "working_set_MB": head["working_set_MB"],
                   "path": PATHS[stages],
                   "prewarm_ms": args.prewarm_ms},
    }
    if head.get("stage_ms"):
        st = head["stage_ms"]
        dom = "k_warp"
        dom_s = st[dom] / 1e3
        achieved = STAGE_BYTES_PER_PX[dom] * px / dom_s / 1e9
        wl = WORKLOADS[stages]
        trace = _profile_record("kernels.json", f"{dom}@{wl}")
        out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                           "traffic": _traffic(dom, wl), "duration_us": round(dom_s * 1e6, 3),
                           "trace_duration_us": trace["avg_us"] if trace else None,
                           "frac_by_trace": round(STAGE_BYTES_PER_PX[dom] * px / (trace["avg_us"] * 1e-6) / 1e9
                                                  / HBM_PEAK_GBS, 4) if trace else None,
                           "trace": f"profiles/kernels.json {dom}@{wl} (rocprofv3 kernel trace of this command)",
                           "duration_from": "the kernel's own dispatch start/stop timestamps (HIP events "
                                            f"attached to its launch), mean over every {every}-th timed step",
                           "bytes_per_launch": STAGE_BYTES_PER_PX[dom] * px,
                           "longest_kernel": max(st, key=st.get)}
        out["kernels_ms"] = st
        out["kernels_hbm_frac"] = {k: round(STAGE_BYTES_PER_PX[k] * px / (v / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
                                   for k, v in st.items()}
    out["roofline_path"] = {"bytes_per_frame": BYTES_PER_PX * px, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac_by_step_time": head["path_hbm_frac"],
                            "kernel_sum_us": head.get("kernel_sum_us"),
                            "frac_by_kernel_sum": head.get("kernel_sum_hbm_frac")}
    out["latency_ms"] = {"p50": lat["gpu_ms"]["p50"], "p99": lat["gpu_ms"]["p99"]}
    out["latency"] = lat
    forms = [f for f in args.forms.split(",") if f]
    out["forms"] = {}
    for form, st, key in (("serial", 1, "plain_serial_4k"), ("pipelined2", 2, "plain_pipelined2_4k"),
                          ("pipelined3", 3, "plain_pipelined3_4k")):
        if form in forms and st != stages:
            r, c, _, _, _ = plain_leg(torch, synth, W, H, B, args.frames, args.outs, args.steps, 30,
                                      args.prewarm_ms / 1e3, every, st, 3)
            c.close()
            r.pop("seconds")
            r["path"] = PATHS[st]
            out["forms"][key] = r
    if "1080p" in forms:
        # 1080p pipelines two stages: its kernels are short enough that the
        # third stage's extra cross-stream hops cost more than its overlap
        st1080 = min(stages, 2)
        r, c, s, f, o = plain_leg(torch, synth, 1920, 1080, 38, args.frames, args.outs, 2 * args.steps, 100,
                                  args.prewarm_ms / 1e3, every, st1080, 2)
        r["path"] = PATHS[st1080]
        r["latency"] = latency_run(torch, c, s, f, o, 38, args.latency_samples)
        c.close()
        del f, o
        r.pop("seconds")
        out["forms"]["plain_1080p"] = r
    if "video" in forms:
        clip = video_clip(torch, synth, args.video_bank)
        n_outs = args.video_outs or len(clip[1])
        steps = len(clip[1]) * max(1, round(args.form_steps * 5 / len(clip[1])))
        out["forms"]["video_graph_4k"] = video_leg(torch, synth, clip, steps, 10, n_outs, 2)
        out["forms"]["video_graph_4k_serial"] = video_leg(torch, synth, clip, steps, 10, n_outs, 1)
        del clip
        torch.cuda.empty_cache()
    if "batch" in forms:
        out["forms"]["batch_uneven_64"] = batch_leg(torch, synth, args.form_steps // 2, 3)
    if "serve" in forms:
        comp = [float(x) for x in args.serve_compress.split(",") if x]
        out["forms"]["serve_8_streams"] = serve_leg(torch, synth, args.serve_seconds, args.serve_burst, comp)
    if "host" in forms:
        out["forms"]["host_pinned_4k"] = host_leg(torch, synth, args.host_frames, 3)
    if "inpaint" in forms:
        out["forms"]["inpaint_vs_row_fill"] = inpaint_leg(torch, synth, 5)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
