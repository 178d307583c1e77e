"""GPU tests of the launch forms beyond the single call: hipGraph video
replay, batched frames (staged and fused forms, the autotuner, the context's
own batch call).  Every output is compared with the oracle directly, and with
the plain per-frame call."""
import numpy as np
import pytest

import refs
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2009_09501_amd import Context
    c = Context(0, 7680, 4320)
    yield c
    c.close()


def _plain(ctx, frame_t, **params):
    L, R, A = ctx.synthesize(frame_t, **params)
    torch.cuda.synchronize()
    return L.cpu().numpy(), R.cpu().numpy(), A.cpu().numpy()


@pytest.mark.parametrize("pipelined", [False, True])
@pytest.mark.parametrize("w,h", [(1920, 1080), (640, 360), (333, 190)])
def test_video_graph_matches_plain_and_oracle(ctx, oracle_mod, w, h, pipelined):
    from paper_2009_09501_amd import pstereo_params_init
    from paper_2009_09501_amd.pstereo import (PSTEREO_PIPELINE, pstereo_video_begin, pstereo_video_end,
                                              pstereo_video_frame)
    dev = torch.device("cuda:0")
    # 21 frames: the ring of graphs wraps twice, through both completion events
    spec = synth.VideoSpec(4, w, h, frames=21, n=40, sigma=3.0)
    frames = [torch.from_numpy(spec.frame(t)).to(dev) for t in range(21)]
    B = synth.default_disparity(w)
    print(f"video {w}x{h} B={B} pipelined={pipelined}: 21 frames through the graphs", flush=True)
    outs = [[torch.empty_like(frames[0]) for _ in range(3)] for _ in frames]
    p = pstereo_params_init(max_disparity=B, flags=PSTEREO_PIPELINE if pipelined else 0)
    p.stream = torch.cuda.current_stream().cuda_stream
    v = pstereo_video_begin(ctx.handle, w, h, p)
    try:
        for f, o in zip(frames, outs):
            pstereo_video_frame(v, f, *o, ctx=ctx.handle)
        torch.cuda.synchronize()
    finally:
        pstereo_video_end(v)
    for i, (f, o) in enumerate(zip(frames, outs)):
        ref = _plain(ctx, f, max_disparity=B)
        for got, want in zip(o, ref):
            assert np.array_equal(got.cpu().numpy(), want), f"frame {i}"
        refs.assert_views(o, refs.views(("video", 4, w, h, i), spec.frame(i), B), f"video {w}x{h} frame {i}")


def test_video_4k_clip_frames_vs_oracle(ctx):
    """The 4K clip's pipelined replay over 300 frames: frames 0, 149 and 299
    of the moving-ellipse clip against the oracle, the frames in between from
    a bank of four (the graph ring wraps 37 times); every output compared on
    the device with the plain call's output for the same input."""
    from paper_2009_09501_amd import pstereo_params_init
    from paper_2009_09501_amd.pstereo import (PSTEREO_PIPELINE, pstereo_video_begin, pstereo_video_end,
                                              pstereo_video_frame)
    dev = torch.device("cuda:0")
    W, H = 3840, 2160
    B = synth.default_disparity(W)
    spec = synth.VideoSpec(4, W, H, frames=300, n=40, sigma=3.0)
    special = {t: spec.frame(t) for t in (0, 149, 299)}
    bank_t = [37, 75, 187, 262]
    dframes = {t: torch.from_numpy(spec.frame(t)).to(dev) for t in bank_t}
    dframes.update({t: torch.from_numpy(f).to(dev) for t, f in special.items()})
    seq = [t if t in special else bank_t[t % 4] for t in range(300)]
    plain = {}
    for t, f in dframes.items():
        plain[t] = ctx.synthesize(f, max_disparity=B)
    torch.cuda.synchronize()
    p = pstereo_params_init(max_disparity=B, flags=PSTEREO_PIPELINE)
    p.stream = torch.cuda.current_stream().cuda_stream
    v = pstereo_video_begin(ctx.handle, W, H, p)
    kept = {}
    try:
        chunk = 50
        for c0 in range(0, 300, chunk):
            outs = [[torch.empty_like(dframes[0]) for _ in range(3)] for _ in range(chunk)]
            for k in range(chunk):
                pstereo_video_frame(v, dframes[seq[c0 + k]], *outs[k], ctx=ctx.handle)
            torch.cuda.synchronize()
            for k in range(chunk):
                t = c0 + k
                for o, pl in zip(outs[k], plain[seq[t]]):
                    assert torch.equal(o, pl), f"video frame {t} differs from the plain call"
                if t in special:
                    kept[t] = [o.cpu() for o in outs[k]]
            print(f"video 4K frames {c0}..{c0 + chunk - 1} equal the plain call", flush=True)
    finally:
        pstereo_video_end(v)
    for t, f in special.items():
        refs.assert_views(kept[t], refs.views(("video", 4, W, H, t), f, B), f"4K video frame {t}")


def test_video_rejects_external_depth(ctx):
    from paper_2009_09501_amd import PSTEREO_DEPTH_EXTERNAL, pstereo_params_init
    from paper_2009_09501_amd.pstereo import PstereoError, pstereo_video_begin
    p = pstereo_params_init()
    p.flags = PSTEREO_DEPTH_EXTERNAL
    with pytest.raises(PstereoError):
        pstereo_video_begin(ctx.handle, 64, 64, p)


def _batch_frames(sizes, seed0):
    dev = torch.device("cuda:0")
    host = [synth.gen_frame(seed0 + i, w, h, 20, 4.0) for i, (w, h) in enumerate(sizes)]
    return host, [torch.from_numpy(f).to(dev) for f in host]


def _batch_oracle(host, sizes, seed0, **kw):
    return [refs.views(("batch", seed0 + i, w, h), f, synth.default_disparity(w), **kw)
            for i, (f, (w, h)) in enumerate(zip(host, sizes))]


BATCH_SIZES = [(1920, 1080), (640, 360), (1280, 720), (3840, 2160), (648, 364), (1024, 768), (2560, 1440),
               (7680, 4320)]


TUNINGS = {
    "staged": dict(mode=0, warp_lanes=256, warp_rows=1),
    "staged_wide_rows3": dict(mode=0, warp_lanes=1024, warp_rows=3),
    "staged_narrow_rows8": dict(mode=0, warp_lanes=64, warp_rows=8),
    "staged_bs16": dict(mode=0, warp_lanes=512, warp_rows=2, bs_rows=16),
    "staged_bs64": dict(mode=0, warp_lanes=256, warp_rows=4, bs_rows=64),
    "fused": dict(mode=1),
}


@pytest.mark.parametrize("tuning", list(TUNINGS))
def test_batch_matches_plain_and_oracle(ctx, oracle_mod, tuning):
    from paper_2009_09501_amd import pstereo_params_init
    from paper_2009_09501_amd.pstereo import (make_jobs, pstereo_batch_create, pstereo_batch_destroy,
                                              pstereo_batch_run, pstereo_batch_set_tuning)
    host, frames = _batch_frames(BATCH_SIZES, 700)
    outs = [[torch.zeros_like(f) for _ in range(3)] for f in frames]
    print(f"batch ({tuning}) of {len(frames)} frames: {BATCH_SIZES}", flush=True)
    b = pstereo_batch_create(ctx.handle, 16, sum(w * h for w, h in BATCH_SIZES) + 1024)
    try:
        pstereo_batch_set_tuning(b, **TUNINGS[tuning])
        p = pstereo_params_init()
        p.stream = torch.cuda.current_stream().cuda_stream
        jobs = make_jobs(frames, outs)
        pstereo_batch_run(b, jobs, len(frames), p)
        torch.cuda.synchronize()
    finally:
        pstereo_batch_destroy(b)
    ora = _batch_oracle(host, BATCH_SIZES, 700)
    for i, (f, o) in enumerate(zip(frames, outs)):
        refs.assert_views(o, ora[i], f"batch ({tuning}) frame {i} {BATCH_SIZES[i]}")
        ref = _plain(ctx, f, max_disparity=synth.default_disparity(f.shape[1]))
        for k, (got, want) in enumerate(zip(o, ref)):
            g = got.cpu().numpy()
            assert np.array_equal(g, want), f"frame {i} {BATCH_SIZES[i]} output {k}: {(g != want).any(-1).sum()} px"


@pytest.mark.parametrize("K", [2, 0])
def test_synthesize_batch_call(ctx, K):
    """pstereo_synthesize_batch (the context's own batch object, grown on
    demand) against the oracle, twice: a small batch, then a larger one that
    makes the context grow its object; K = 2 runs every frame with blocks of
    2 px (small frames: at most 32768 blocks), K = 0 the automatic size."""
    from paper_2009_09501_amd import pstereo_params_init
    from paper_2009_09501_amd.pstereo import PSTEREO_SYNC, make_jobs, pstereo_synthesize_batch
    if K == 2:
        rounds = [[(320, 240), (64, 48)], [(360, 360), (128, 96), (200, 100)]]
    else:
        rounds = [[(640, 360), (1280, 720)], [(1920, 1080), (640, 360), (3840, 2160), (2560, 1440)]]
    for r, sizes in enumerate(rounds):
        seed0 = 1500 + 20 * r + K
        host, frames = _batch_frames(sizes, seed0)
        outs = [[torch.zeros_like(f) for _ in range(3)] for f in frames]
        p = pstereo_params_init(block_size=K, flags=PSTEREO_SYNC)
        print(f"synthesize_batch K={K} round {r}: {sizes}", flush=True)
        pstereo_synthesize_batch(ctx.handle, make_jobs(frames, outs), len(frames), p)
        for i, (o, want) in enumerate(zip(outs, _batch_oracle(host, sizes, seed0, K=K))):
            refs.assert_views(o, want, f"synthesize_batch K={K} round {r} frame {i} {sizes[i]}")


@pytest.mark.parametrize("tuning", ["staged", "fused"])
def test_batch_relaunch_and_graph_replay(ctx, tuning):
    from paper_2009_09501_amd import pstereo_params_init
    from paper_2009_09501_amd.pstereo import (make_jobs, pstereo_batch_create, pstereo_batch_destroy,
                                              pstereo_batch_launch, pstereo_batch_prepare, pstereo_batch_set_tuning)
    sizes = [(1280, 720), (640, 360), (1920, 1080)]
    host, frames = _batch_frames(sizes, 900)
    outs = [[torch.zeros_like(f) for _ in range(3)] for f in frames]
    ora = _batch_oracle(host, sizes, 900)
    b = pstereo_batch_create(ctx.handle, 4, sum(w * h for w, h in sizes))
    s = torch.cuda.Stream()
    try:
        pstereo_batch_set_tuning(b, **TUNINGS[tuning])
        p = pstereo_params_init()
        p.stream = s.cuda_stream
        jobs = make_jobs(frames, outs)
        pstereo_batch_prepare(b, jobs, len(frames), p)
        for rep in range(3):
            for o in outs:
                for x in o:
                    x.zero_()
            torch.cuda.synchronize()
            pstereo_batch_launch(b, s)
            s.synchronize()
            for i, (o, r) in enumerate(zip(outs, ora)):
                refs.assert_views(o, r, f"relaunch {rep} frame {i}")
        # captured into a HIP graph (through torch's graph API) and replayed
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            pstereo_batch_launch(b, torch.cuda.current_stream())
        for rep in range(3):
            for o in outs:
                for x in o:
                    x.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for i, (o, r) in enumerate(zip(outs, ora)):
                refs.assert_views(o, r, f"graph replay {rep} frame {i}")
    finally:
        torch.cuda.synchronize()
        pstereo_batch_destroy(b)


def test_batch_autotune_picks_a_candidate_and_stays_exact(ctx):
    from paper_2009_09501_amd import pstereo_params_init
    from paper_2009_09501_amd.pstereo import (make_jobs, pstereo_batch_autotune, pstereo_batch_create,
                                              pstereo_batch_destroy, pstereo_batch_get_tuning,
                                              pstereo_batch_launch)
    sizes = [(1280, 720), (640, 360), (1920, 1080), (2560, 1440)]
    host, frames = _batch_frames(sizes, 950)
    ora = _batch_oracle(host, sizes, 950)
    outs = [[torch.zeros_like(f) for _ in range(3)] for f in frames]
    s = torch.cuda.Stream()
    b = pstereo_batch_create(ctx.handle, 4, sum(w * h for w, h in sizes))
    try:
        p = pstereo_params_init()
        p.stream = s.cuda_stream
        jobs = make_jobs(frames, outs)
        best, best_ms, trials = pstereo_batch_autotune(b, jobs, len(frames), p, reps=2)
        print(f"autotune: best {best} {best_ms:.3f} ms over {len(trials)} candidates", flush=True)
        # 12 staged candidates and the fused one, then the first pass's
        # winner with three block-statistics tile heights if it is staged
        first = min(trials[:13], key=lambda t: t["ms"])
        assert len(trials) == (16 if first["mode"] == 0 else 13)
        for t in trials[13:]:
            assert t["bs_rows"] in (16, 32, 64)
            assert (t["warp_lanes"], t["warp_rows"]) == (first["warp_lanes"], first["warp_rows"])
        assert best_ms == min(t["ms"] for t in trials)
        assert pstereo_batch_get_tuning(b) == best
        for o in outs:
            for x in o:
                x.zero_()
        torch.cuda.synchronize()
        pstereo_batch_launch(b, s)
        s.synchronize()
        for i, (o, r) in enumerate(zip(outs, ora)):
            refs.assert_views(o, r, f"autotuned batch frame {i}")
    finally:
        torch.cuda.synchronize()
        pstereo_batch_destroy(b)


def test_batch_rejects(ctx):
    from paper_2009_09501_amd.pstereo import (PSTEREO_E_ALIAS, PSTEREO_E_INVALID, PSTEREO_E_UNSUPPORTED,
                                              make_jobs, pstereo_batch_create, pstereo_batch_destroy,
                                              pstereo_batch_run)
    dev = torch.device("cuda:0")
    b = pstereo_batch_create(ctx.handle, 2, 1 << 22)
    try:
        f = torch.zeros((64, 66, 3), dtype=torch.uint8, device=dev)
        o = [torch.empty_like(f) for _ in range(3)]
        assert pstereo_batch_run(b, make_jobs([f], [o]), 1, None, check=False) == PSTEREO_E_UNSUPPORTED
        f = torch.zeros((64, 64, 3), dtype=torch.uint8, device=dev)
        o = [torch.empty_like(f) for _ in range(3)]
        assert pstereo_batch_run(b, make_jobs([f], [[o[0], o[0], o[2]]]), 1, None, check=False) == PSTEREO_E_ALIAS
        assert pstereo_batch_run(b, make_jobs([f, f, f], [o, o, o]), 3, None, check=False) == PSTEREO_E_INVALID
        big = torch.zeros((4096, 2048, 3), dtype=torch.uint8, device=dev)
        ob = [torch.empty_like(big) for _ in range(3)]
        assert pstereo_batch_run(b, make_jobs([big], [ob]), 1, None, check=False) == PSTEREO_E_INVALID
        from paper_2009_09501_amd.pstereo import pstereo_batch_set_tuning
        for bad in (dict(bs_rows=24), dict(bs_rows=128), dict(warp_rows=9), dict(warp_lanes=96)):
            assert pstereo_batch_set_tuning(b, check=False, **bad) == PSTEREO_E_INVALID, bad
    finally:
        pstereo_batch_destroy(b)
