"""GPU parity: the HIP library through its C ABI against the CPU oracle.

Every stage is integer, so every comparison is bit-exact: the three output
images, the raw and filtered depth maps and the per-block statistics, labels
and region depths.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2009_09501_amd import Context
    c = Context(0, 7680, 4320)
    yield c
    c.close()


def _run(ctx, frame, depth=None, **params):
    dev = torch.device("cuda:0")
    f = torch.from_numpy(np.ascontiguousarray(frame)).to(dev)
    h, w, _ = frame.shape
    d0 = torch.empty((h, w), dtype=torch.uint8, device=dev)
    df = torch.empty((h, w), dtype=torch.uint8, device=dev)
    dep = torch.from_numpy(np.ascontiguousarray(depth)).to(dev) if depth is not None else None
    L, R, A = ctx.synthesize(f, depth=dep, out_depth=df, out_depth_raw=d0, **params)
    torch.cuda.synchronize()
    return {"L": L.cpu().numpy(), "R": R.cpu().numpy(), "A": A.cpu().numpy(),
            "D0": d0.cpu().numpy(), "Df": df.cpu().numpy()}


def _compare(case, got, ref, blocks=None):
    for k in ("D0", "Df", "L", "R", "A"):
        g, w = got[k], getattr(ref, k)
        if not np.array_equal(g, w):
            diff = (g != w) if g.ndim == 2 else (g != w).any(-1)
            ys, xs = np.nonzero(diff)
            raise AssertionError(f"{case}: {k} differs at {diff.sum()} pixels, first (y={ys[0]}, x={xs[0]})")
    if blocks is not None:
        st, lab, db = blocks
        assert np.array_equal(st, ref.stats), f"{case}: block stats"
        assert np.array_equal(lab, ref.labels), f"{case}: labels"
        assert np.array_equal(db, ref.dblk), f"{case}: region depth"


def _check(ctx, oracle_mod, frame, B, T=150, K=0, g=24, tau=24, r=2, depth=None, case=""):
    from paper_2009_09501_amd import pstereo_debug_blocks
    print(f"case {case}: {frame.shape[1]}x{frame.shape[0]} B={B} T={T} K={K} r={r} "
          f"ext={depth is not None}", flush=True)
    got = _run(ctx, frame, depth=depth, max_disparity=B, depth_threshold=T, block_size=K,
               edge_thresh=g, link_thresh=tau, cbf_radius=r)
    ref = oracle_mod.synthesize(frame, B, T, K, g, tau, r, depth=depth)
    blocks = None if depth is not None else pstereo_debug_blocks(ctx.handle)
    _compare(case, got, ref, blocks)


def test_config0_640x360(ctx, oracle_mod):
    f = synth.gen_frame(1, 640, 360, 12, 4.0)
    _check(ctx, oracle_mod, f, 12, case="640x360 seed 1")


@pytest.mark.parametrize("w,h,seed", [(1920, 1080, 2), (3840, 2160, 3)])
def test_config1_full_frames(ctx, oracle_mod, w, h, seed):
    f = synth.gen_frame(seed, w, h, 40, 4.0)
    _check(ctx, oracle_mod, f, synth.default_disparity(w), case=f"{w}x{h} seed {seed}")


def test_8k_frame(ctx, oracle_mod):
    f = synth.gen_frame(5001, 7680, 4320, 40, 4.0)
    _check(ctx, oracle_mod, f, 154, case="8k seed 5001")


@pytest.mark.parametrize("w,h", [(333, 191), (1, 1), (5, 3), (17, 1), (1, 9), (64, 64), (130, 7),
                                 (641, 359), (1023, 17), (4097, 11)])
def test_ragged_sizes(ctx, oracle_mod, w, h):
    f = synth.gen_frame(w * 7 + h, w, h, 6, 4.0)
    _check(ctx, oracle_mod, f, min(12, 255), case=f"ragged {w}x{h}")


@pytest.mark.parametrize("K", [2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("r", [0, 1, 2, 3])
def test_block_sizes_and_radii(ctx, oracle_mod, K, r):
    w, h = 400, 240
    if (-(-w // K)) * (-(-h // K)) > 32768:
        pytest.skip("too many blocks")
    f = synth.gen_frame(K * 10 + r, w, h, 16, 4.0)
    _check(ctx, oracle_mod, f, 20, K=K, r=r, case=f"K={K} r={r}")


@pytest.mark.parametrize("B,T", [(0, 150), (1, 150), (77, 150), (255, 150), (12, -1), (12, 0), (12, 255)])
def test_disparity_parameters(ctx, oracle_mod, B, T):
    f = synth.gen_frame(B + T + 3, 320, 96, 12, 4.0)
    _check(ctx, oracle_mod, f, B, T=T, case=f"B={B} T={T}")


@pytest.mark.parametrize("g,tau", [(0, 0), (8, 80), (60, 12), (255, 765)])
def test_cue_thresholds(ctx, oracle_mod, g, tau):
    f = synth.gen_frame(g + tau, 256, 144, 20, 4.0)
    _check(ctx, oracle_mod, f, 12, g=g, tau=tau, case=f"g={g} tau={tau}")


def test_external_depth_worked_rows(ctx, oracle_mod):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "worked_rows.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        name, dep, Ls, Rs = [s.strip() for s in line.split("|")]
        dep = np.array([[int(v) for v in dep.split()]], np.uint8)
        Ls = [int(v) for v in Ls.split()]
        Rs = [int(v) for v in Rs.split()]
        w = dep.shape[1]
        f = np.zeros((1, w, 3), np.uint8)
        f[0, :, 0] = np.arange(w) * 10
        f[0, :, 1] = 255 - np.arange(w) * 10
        f[0, :, 2] = 7
        got = _run(ctx, f, depth=dep, max_disparity=12, cbf_radius=0)
        assert np.array_equal(got["L"][0], f[0, Ls]), name
        assert np.array_equal(got["R"][0], f[0, Rs]), name


@pytest.mark.parametrize("seed", [1, 2])
def test_external_random_depth(ctx, oracle_mod, seed):
    rng = np.random.default_rng(seed)
    f = synth.gen_frame(seed, 517, 203, 10, 4.0)
    dep = rng.integers(0, 256, (203, 517)).astype(np.uint8)
    _check(ctx, oracle_mod, f, 40, depth=dep, case=f"external depth seed {seed}")


@pytest.mark.parametrize("w,h", [(640, 96), (3840, 64)])
def test_black_sources_at_depth_zero(ctx, oracle_mod, w, h):
    """A black source at depth 0 has the same z-buffer key as an empty
    pixel: rows with such sources (and rows without, the zero-key tag off)
    against the oracle, with an external depth of 0 in a band and around
    black rectangles, and one row that is all black at depth 0."""
    rng = np.random.default_rng(w + h)
    f = synth.gen_frame(w * 3 + h, w, h, 12, 4.0)
    dep = np.full((h, w), 180, np.uint8)
    dep[:, : w * 2 // 5] = 0                      # a depth-0 band
    dep[h // 3: h // 2, :] = 0                    # and depth-0 rows
    f[h // 8: h // 3, w // 10: w // 4] = 0        # black inside the band
    f[h // 3: h // 2, w // 2: w // 2 + w // 8] = 0
    ys, xs = rng.integers(0, h, 400), rng.integers(0, w, 400)
    f[ys, xs] = 0                                 # scattered black pixels
    f[h - 3] = 0
    dep[h - 3] = 0                                # a black row at depth 0
    _check(ctx, oracle_mod, f, synth.default_disparity(w), depth=dep, case=f"black depth-0 {w}x{h}")


def test_zero_base_identity(ctx):
    f = synth.gen_frame(9, 640, 360, 12, 4.0)
    got = _run(ctx, f, max_disparity=0)
    for k in ("L", "R", "A"):
        assert np.array_equal(got[k], f)


@pytest.mark.parametrize("w,h,seed", [(1920, 1080, 21), (3840, 2160, 22), (7680, 4320, 23)])
def test_deterministic_repeat(ctx, w, h, seed):
    """Four runs of one frame, plain, pipelined and three-stage pipelined,
    each equal to the oracle (4K and 8K take the two warp row shapes: two and
    four quads per lane)."""
    from paper_2009_09501_amd.pstereo import PSTEREO_PIPELINE, PSTEREO_PIPELINE_DEEP
    import refs
    f = synth.gen_frame(seed, w, h, 40, 4.0)
    B = synth.default_disparity(w)
    want = refs.views(("still", seed, w, h), f, B)
    dev = torch.device("cuda:0")
    ft = torch.from_numpy(f).to(dev)
    for run, fl in enumerate((0, 0, PSTEREO_PIPELINE, PSTEREO_PIPELINE_DEEP)):
        print(f"repeat {w}x{h} run {run}", flush=True)
        L, R, A = ctx.synthesize(ft, max_disparity=B, flags=fl)
        torch.cuda.synchronize()
        refs.assert_views((L, R, A), want, f"{w}x{h} run {run}")


@pytest.mark.parametrize("variant", ["k2", "gather", "profiled", "r0", "deep-k2", "deep-gather", "deep-profiled",
                                     "deep-r0"])
def test_pipelined_variants(ctx, oracle_mod, variant):
    """PSTEREO_PIPELINE and PSTEREO_PIPELINE_DEEP with 2 px blocks, the
    Fig. 3 gather, per-kernel profiling and an unfiltered depth map (radius
    0): a run of six calls on one stream cycling three frames, every output
    equal to the oracle."""
    from paper_2009_09501_amd.pstereo import (PSTEREO_PIPELINE, PSTEREO_PIPELINE_DEEP, PSTEREO_PROFILE,
                                              PSTEREO_WARP_GATHER, pstereo_profile_collect)
    import refs
    deep = variant.startswith("deep-")
    variant = variant.removeprefix("deep-")
    w, h = (320, 200) if variant == "k2" else (1280, 720)
    B = synth.default_disparity(w)
    host = [synth.gen_frame(500 + i, w, h, 12, 4.0) for i in range(3)]
    dev = torch.device("cuda:0")
    frames = [torch.from_numpy(f).to(dev) for f in host]
    kw = {"K": 2} if variant == "k2" else {"r": 0} if variant == "r0" else {}
    params = {"block_size": 2} if variant == "k2" else {"cbf_radius": 0} if variant == "r0" else {}
    flags = (PSTEREO_PIPELINE_DEEP if deep else PSTEREO_PIPELINE) | \
        (PSTEREO_WARP_GATHER if variant == "gather" else 0) | (PSTEREO_PROFILE if variant == "profiled" else 0)
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    pstereo_profile_collect(ctx.handle)  # clear
    outs = []
    for i in range(6):
        print(f"pipelined {variant} call {i}", flush=True)
        outs.append(ctx.synthesize(frames[i % 3], stream=st, flags=flags, max_disparity=B, **params))
    st.synchronize()
    for i, o in enumerate(outs):
        f = host[i % 3]
        if variant == "gather":
            want = oracle_mod.synthesize_gather(f, B)
        else:
            want = refs.views(("pipe-variant", 500 + i % 3, w, h), f, B, **kw)
        refs.assert_views(o, want, f"{variant} call {i}")
    if variant == "profiled":
        ms, n, _ = pstereo_profile_collect(ctx.handle)
        assert n == 6 and all(m > 0 for m in ms)


def test_default_stream_ordering(oracle_mod):
    """Work on torch's default stream (the HIP null stream): the frame
    written by a torch kernel just before the call, the outputs read by
    .cpu() right after it -- no device-wide synchronisation anywhere -- and
    on a side stream with only that stream's ordering."""
    from paper_2009_09501_amd import Context
    import refs
    dev = torch.device("cuda:0")
    w, h = 1920, 1080
    frame = synth.gen_frame(41, w, h, 40, 4.0)
    want = refs.views(("still", 41, w, h), frame, 38)
    ctx = Context(0, w, h)
    try:
        src = torch.from_numpy(frame).to(dev)
        for rep in range(3):
            ft = torch.zeros_like(src)
            ft.copy_(src)  # a kernel on the default stream writes the frame
            outs = [torch.full_like(src, 7) for _ in range(3)]
            ctx.synthesize(ft, out=outs, max_disparity=38)
            refs.assert_views([o.cpu() for o in outs], want, f"default stream rep {rep}")
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            ft = torch.zeros_like(src)
            ft.copy_(src)
            outs = [torch.full_like(src, 7) for _ in range(3)]
        ctx.synthesize(ft, out=outs, stream=s, max_disparity=38)
        s.synchronize()
        refs.assert_views([o.cpu() for o in outs], want, "side stream")
    finally:
        ctx.close()


def test_pipelined_sequence(oracle_mod):
    """PSTEREO_PIPELINE over a run of frames of one and of several sizes,
    mixed with plain calls, a stream change and a block dump: every output
    equals the oracle."""
    from paper_2009_09501_amd import Context, pstereo_debug_blocks
    from paper_2009_09501_amd.pstereo import PSTEREO_PIPELINE
    import refs
    dev = torch.device("cuda:0")
    sizes = [(1920, 1080), (1920, 1080), (640, 360), (1920, 1080), (1280, 720), (333, 191), (1920, 1080),
             (1920, 1080)]
    host = [synth.gen_frame(300 + i, w, h, 40, 4.0) for i, (w, h) in enumerate(sizes)]
    frames = [torch.from_numpy(f).to(dev) for f in host]
    ctx = Context(0, 1920, 1080)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    try:
        # flags per call: pipelined except calls 3 (plain) and 6 (other stream)
        outs, streams = [], []
        for i, (f, (w, h)) in enumerate(zip(frames, sizes)):
            st = s2 if i == 6 else s1
            fl = 0 if i == 3 else PSTEREO_PIPELINE
            print(f"pipelined call {i}: {w}x{h} flags {fl}", flush=True)
            outs.append(ctx.synthesize(f, stream=st, flags=fl, max_disparity=synth.default_disparity(w)))
            streams.append(st)
            if i == 4:
                st.synchronize()
                # the block dump of call 4 (pipelined) equals the oracle's
                stt, lab, db = pstereo_debug_blocks(ctx.handle)
                ref = oracle_mod.synthesize(host[4], synth.default_disparity(1280))
                assert np.array_equal(stt, ref.stats) and np.array_equal(lab, ref.labels)
                assert np.array_equal(db, ref.dblk)
        torch.cuda.synchronize()
        for i, ((w, h), f, o) in enumerate(zip(sizes, host, outs)):
            refs.assert_views(o, refs.views(("pipe", 300 + i, w, h), f, synth.default_disparity(w)), f"call {i}")
        # a long pipelined run on one stream, outputs checked frame by frame
        ring = [frames[0], frames[1], frames[3]]
        res = []
        for i in range(24):
            res.append(ctx.synthesize(ring[i % 3], stream=s1, flags=PSTEREO_PIPELINE, max_disparity=38))
        s1.synchronize()
        for i, o in enumerate(res):
            k = [0, 1, 3][i % 3]
            refs.assert_views(o, refs.views(("pipe", 300 + k, 1920, 1080), host[k], 38), f"run frame {i}")
    finally:
        ctx.close()


def test_pipelined_deep_sequence(oracle_mod):
    """PSTEREO_PIPELINE_DEEP over a run of frames of several sizes, mixed
    with two-stage pipelined and plain calls, stream changes and a block dump
    (each restarts the pipeline), then a long three-stage run on one stream
    and one on the null stream: every output equals the oracle."""
    from paper_2009_09501_amd import Context, pstereo_debug_blocks
    from paper_2009_09501_amd.pstereo import PSTEREO_PIPELINE, PSTEREO_PIPELINE_DEEP
    import refs
    dev = torch.device("cuda:0")
    sizes = [(1920, 1080), (1920, 1080), (640, 360), (1920, 1080), (1280, 720), (333, 191), (1920, 1080),
             (1920, 1080), (1280, 720), (1920, 1080), (640, 360)]
    D, P = PSTEREO_PIPELINE_DEEP, PSTEREO_PIPELINE
    flags = [D, D, D, 0, D, D, D, P, D, D, D]
    host = [synth.gen_frame(300 + i, w, h, 40, 4.0) for i, (w, h) in enumerate(sizes)]
    frames = [torch.from_numpy(f).to(dev) for f in host]
    ctx = Context(0, 1920, 1080)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    try:
        outs = []
        for i, (f, (w, h), fl) in enumerate(zip(frames, sizes, flags)):
            st = s2 if i in (6, 7) else s1
            if i == 6:
                s2.wait_stream(s1)  # the caller orders a stream change
            if i == 8:
                s1.wait_stream(s2)
            print(f"deep pipelined call {i}: {w}x{h} flags {fl}", flush=True)
            outs.append(ctx.synthesize(f, stream=st, flags=fl, max_disparity=synth.default_disparity(w)))
            if i == 4:
                st.synchronize()
                stt, lab, db = pstereo_debug_blocks(ctx.handle)
                ref = oracle_mod.synthesize(host[4], synth.default_disparity(1280))
                assert np.array_equal(stt, ref.stats) and np.array_equal(lab, ref.labels)
                assert np.array_equal(db, ref.dblk)
        torch.cuda.synchronize()
        for i, ((w, h), f, o) in enumerate(zip(sizes, host, outs)):
            refs.assert_views(o, refs.views(("pipe", 300 + i, w, h), f, synth.default_disparity(w)), f"call {i}")
        ring = [0, 1, 3, 6]
        for name, st in (("stream", s1), ("null stream", None)):
            res = []
            for i in range(24):
                res.append(ctx.synthesize(frames[ring[i % 4]], stream=st, flags=D, max_disparity=38))
            torch.cuda.synchronize()
            for i, o in enumerate(res):
                k = ring[i % 4]
                refs.assert_views(o, refs.views(("pipe", 300 + k, 1920, 1080), host[k], 38), f"{name} frame {i}")
    finally:
        ctx.close()


def test_pipelined_streams_overlap():
    """Eight contexts made one after another in one process, half of them
    kept alive, so that their streams land on various hardware queues: on
    each, two- and three-stage pipelined 4K calls take clearly less time per
    frame than serial calls (streams sharing the caller's queue would give
    the serial time; the first pipelined call checks for that)."""
    import time
    from paper_2009_09501_amd import Context
    from paper_2009_09501_amd.pstereo import PSTEREO_PIPELINE, PSTEREO_PIPELINE_DEEP
    dev = torch.device("cuda:0")
    W, H = 3840, 2160
    frames = [torch.from_numpy(synth.gen_frame(600 + i, W, H, 40, 4.0)).to(dev) for i in range(4)]
    outs = [[torch.empty_like(frames[0]) for _ in range(3)] for _ in range(4)]
    kept = []

    def per_frame(ctx, st, fl, n=200):
        for i in range(20):
            ctx.synthesize(frames[i % 4], out=outs[i % 4], stream=st, flags=fl, max_disparity=77)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n):
            ctx.synthesize(frames[i % 4], out=outs[i % 4], stream=st, flags=fl, max_disparity=77)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    try:
        for trial in range(8):
            ctx = Context(0, W, H)
            st = torch.cuda.Stream()
            ser = per_frame(ctx, st, 0)
            p2 = per_frame(ctx, st, PSTEREO_PIPELINE)
            p3 = per_frame(ctx, st, PSTEREO_PIPELINE_DEEP)
            print(f"context {trial}: us per frame serial {ser * 1e6:.1f}, two stages {p2 * 1e6:.1f}, "
                  f"three {p3 * 1e6:.1f}", flush=True)
            assert p2 < 0.85 * ser and p3 < 0.85 * ser, trial
            if trial % 2:
                ctx.close()
            else:
                kept.append(ctx)
    finally:
        for c in kept:
            c.close()


def test_misaligned_buffers(ctx, oracle_mod):
    """Frame and outputs at odd byte offsets take the bytewise path."""
    from paper_2009_09501_amd import pstereo_params_init, pstereo_synthesize
    w, h = 320, 48
    frame = synth.gen_frame(31, w, h, 8, 4.0)
    n = w * h * 3
    dev = torch.device("cuda:0")
    big = torch.zeros(4 * n + 16, dtype=torch.uint8, device=dev)
    fsrc = big[1:1 + n]
    fsrc.copy_(torch.from_numpy(frame.reshape(-1)).to(dev))
    outs = [big[n + 3 + i * n: 2 * n + 3 + i * n] for i in range(3)]
    p = pstereo_params_init(max_disparity=12)
    p.stream = torch.cuda.current_stream().cuda_stream
    pstereo_synthesize(ctx.handle, fsrc, w, h, p, *outs)
    torch.cuda.synchronize()
    ref = oracle_mod.synthesize(frame, 12)
    for o, want in zip(outs, (ref.L, ref.R, ref.A)):
        assert np.array_equal(o.cpu().numpy().reshape(h, w, 3), want)


def test_error_codes(ctx):
    from paper_2009_09501_amd import pstereo_params_init, pstereo_synthesize
    from paper_2009_09501_amd.pstereo import (PSTEREO_E_ALIAS, PSTEREO_E_INVALID,
                                              PSTEREO_E_UNSUPPORTED)
    dev = torch.device("cuda:0")
    w, h = 64, 32
    f = torch.zeros((h, w, 3), dtype=torch.uint8, device=dev)
    o = [torch.empty_like(f) for _ in range(3)]
    hp = np.zeros((h, w, 3), np.uint8)
    p = pstereo_params_init()
    # host pointer
    assert pstereo_synthesize(ctx.handle, hp.ctypes.data, w, h, p, *o, check=False) == PSTEREO_E_INVALID
    # outputs overlapping
    assert pstereo_synthesize(ctx.handle, f, w, h, p, o[0], o[0], o[2], check=False) == PSTEREO_E_ALIAS
    assert pstereo_synthesize(ctx.handle, f, w, h, p, f, o[1], o[2], check=False) == PSTEREO_E_ALIAS
    # sizes and parameter ranges
    assert pstereo_synthesize(ctx.handle, f, 0, h, p, *o, check=False) == PSTEREO_E_INVALID
    assert pstereo_synthesize(ctx.handle, f, 8000, h, p, *o, check=False) == PSTEREO_E_INVALID
    for field, val in (("max_disparity", 256), ("depth_threshold", -2), ("cbf_radius", 4),
                       ("block_size", 12), ("edge_thresh", 300), ("link_thresh", 766)):
        q = pstereo_params_init(**{field: val})
        assert pstereo_synthesize(ctx.handle, f, w, h, q, *o, check=False) == PSTEREO_E_INVALID, field
    q = pstereo_params_init()
    q.struct_size = 4
    assert pstereo_synthesize(ctx.handle, f, w, h, q, *o, check=False) == PSTEREO_E_INVALID
    # too many blocks for explicit K
    q = pstereo_params_init(block_size=4)
    big = torch.zeros((1080, 1920, 3), dtype=torch.uint8, device=dev)
    ob = [torch.empty_like(big) for _ in range(3)]
    assert pstereo_synthesize(ctx.handle, big, 1920, 1080, q, *ob, check=False) == PSTEREO_E_INVALID
    # video replay pipelines two stages only
    from paper_2009_09501_amd.pstereo import PSTEREO_PIPELINE_DEEP, PstereoError, pstereo_video_begin
    with pytest.raises(PstereoError) as ei:
        pstereo_video_begin(ctx.handle, w, h, pstereo_params_init(flags=PSTEREO_PIPELINE_DEEP))
    assert ei.value.code == PSTEREO_E_UNSUPPORTED
    # the context still works after errors
    pstereo_synthesize(ctx.handle, f, w, h, p, *o)
    torch.cuda.synchronize()


def _block_frame(gw, gh, K, kind):
    """A frame of K x K blocks: kind[by, bx] = 0 uniform grey (100, 100, 100),
    1 uniform (150, 75, 100) -- the same luma, colour distance 75 -- and
    2 an edge block: a black/white pixel checker inside, its top row and left
    column grey, so the blocks above and to the left see no luma step into it."""
    f = np.empty((gh * K, gw * K, 3), np.uint8)
    cols = {0: (100, 100, 100), 1: (150, 75, 100)}
    yy, xx = np.mgrid[0:K, 0:K]
    checker = np.where(((yy + xx) & 1)[..., None] == 1, 255, 0).astype(np.uint8)
    for by in range(gh):
        for bx in range(gw):
            k = kind[by, bx]
            blk = f[by * K:(by + 1) * K, bx * K:(bx + 1) * K]
            if k == 2:
                blk[:] = checker
                blk[0, :] = 100
                blk[:, 0] = 100
            else:
                blk[:] = cols[k]
    return f


@pytest.mark.parametrize("w,h", [(640, 360), (1280, 720), (3840, 2160)])
def test_isoluminant_checker_many_components(ctx, oracle_mod, w, h):
    """Every block its own non-edge component (neighbours share luma, so no
    edges, but differ by 75 in colour, so no links): 3600 components at
    640x360 (strip merge), 14400 and 32400 (the merge's whole-frame grouping)."""
    K = 8 if w * h <= 1280 * 720 else 16
    gw, gh = w // K, h // K
    kind = (np.add.outer(np.arange(gh), np.arange(gw)) & 1).astype(np.int64)
    _check(ctx, oracle_mod, _block_frame(gw, gh, K, kind), synth.default_disparity(w), K=K,
           case=f"isoluminant checker {w}x{h}")


@pytest.mark.parametrize("gw,gh", [(40, 300), (240, 135), (960, 20)])
def test_serpentine_region_across_strips(ctx, oracle_mod, gw, gh):
    """One grey path winding through every block row (walls of edge blocks,
    openings alternately at the right and left end): a single component that
    crosses every strip boundary, plus enclosed grey blocks below it."""
    K = 8
    kind = np.full((gh, gw), 2, np.int64)
    for by in range(0, gh, 2):
        kind[by, :] = 0
        if by + 1 < gh:
            kind[by + 1, gw - 1 if (by // 2) % 2 == 0 else 0] = 0
    _check(ctx, oracle_mod, _block_frame(gw, gh, K, kind), 20, K=K, case=f"serpentine {gw}x{gh} blocks")


@pytest.mark.parametrize("w,h", [(640, 360), (1920, 1080), (644, 200), (333, 191), (7, 5), (1, 1)])
def test_hsbs_output(ctx, oracle_mod, w, h):
    """The fused half side-by-side epilogue equals the oracle's HSBS of the
    oracle's views (aligned widths through the u16-store path, others bytewise)."""
    dev = torch.device("cuda:0")
    frame = synth.gen_frame(31 + w, w, h, 12, 4.0)
    B = synth.default_disparity(w)
    print(f"hsbs {w}x{h} B={B}", flush=True)
    f = torch.from_numpy(frame).to(dev)
    hs = torch.zeros_like(f)
    L, R, A = ctx.synthesize(f, out_hsbs=hs, max_disparity=B)
    torch.cuda.synchronize()
    ref = oracle_mod.synthesize(frame, B)
    assert np.array_equal(L.cpu().numpy(), ref.L)
    assert np.array_equal(R.cpu().numpy(), ref.R)
    assert np.array_equal(hs.cpu().numpy(), oracle_mod.hsbs(ref.L, ref.R))


@pytest.mark.parametrize("w,h", [(640, 360), (1920, 1080), (333, 191), (7, 5)])
def test_gather_mode(ctx, oracle_mod, w, h):
    """PSTEREO_WARP_GATHER: the Fig. 3 destination-depth gather equals the
    oracle's gather of the oracle's filtered depth (with HSBS as well)."""
    from paper_2009_09501_amd.pstereo import PSTEREO_WARP_GATHER
    dev = torch.device("cuda:0")
    frame = synth.gen_frame(55 + w, w, h, 12, 4.0)
    B = synth.default_disparity(w)
    print(f"gather {w}x{h} B={B}", flush=True)
    f = torch.from_numpy(frame).to(dev)
    hs = torch.zeros_like(f)
    L, R, A = ctx.synthesize(f, out_hsbs=hs, flags=PSTEREO_WARP_GATHER, max_disparity=B)
    torch.cuda.synchronize()
    gL, gR, gA = oracle_mod.synthesize_gather(frame, B)
    assert np.array_equal(L.cpu().numpy(), gL)
    assert np.array_equal(R.cpu().numpy(), gR)
    assert np.array_equal(A.cpu().numpy(), gA)
    assert np.array_equal(hs.cpu().numpy(), oracle_mod.hsbs(gL, gR))


def test_gather_worked_rows_external_depth(ctx, oracle_mod):
    from paper_2009_09501_amd.pstereo import PSTEREO_WARP_GATHER
    dev = torch.device("cuda:0")
    rows = [[0] * 6 + [255] * 4 + [0] * 6, [0, 0, 255, 255, 255, 255] + [0] * 10, [200] * 16, [150] * 8 + [151] * 8]
    dep = np.array(rows, np.uint8)
    f = np.zeros((4, 16, 3), np.uint8)
    f[:, :, 0] = np.arange(16) * 10
    f[:, :, 1] = 255 - np.arange(16) * 10
    f[:, :, 2] = 7
    L, R, A = ctx.synthesize(torch.from_numpy(f).to(dev), depth=torch.from_numpy(dep).to(dev),
                             flags=PSTEREO_WARP_GATHER, max_disparity=12, cbf_radius=0)
    torch.cuda.synchronize()
    gL, gR, gA = oracle_mod.synthesize_gather(f, 12, depth=dep, r=0)
    assert np.array_equal(L.cpu().numpy(), gL) and np.array_equal(R.cpu().numpy(), gR)
    assert np.array_equal(A.cpu().numpy(), gA)


@pytest.mark.parametrize("w,h", [(640, 360), (333, 191), (24, 9)])
def test_inpaint_blocks_mode(ctx, oracle_mod, w, h):
    """PSTEREO_INPAINT_BLOCKS: the sweeps and composition equal the oracle's
    block-iterative inpainting of the oracle's warped views."""
    from paper_2009_09501_amd.pstereo import PSTEREO_INPAINT_BLOCKS
    dev = torch.device("cuda:0")
    frame = synth.gen_frame(77 + w, w, h, 12, 4.0)
    B = max(synth.default_disparity(w), 8)
    print(f"inpaint {w}x{h} B={B}", flush=True)
    f = torch.from_numpy(frame).to(dev)
    hs = torch.zeros_like(f)
    L, R, A = ctx.synthesize(f, out_hsbs=hs, flags=PSTEREO_INPAINT_BLOCKS, max_disparity=B)
    torch.cuda.synchronize()
    iL, iR, iA = oracle_mod.synthesize_inpaint(frame, B)
    assert np.array_equal(L.cpu().numpy(), iL)
    assert np.array_equal(R.cpu().numpy(), iR)
    assert np.array_equal(A.cpu().numpy(), iA)
    assert np.array_equal(hs.cpu().numpy(), oracle_mod.hsbs(iL, iR))
    # the plain row fill on the same frame still matches its own oracle afterwards
    L2, R2, _ = ctx.synthesize(f, max_disparity=B)
    torch.cuda.synchronize()
    ref = oracle_mod.synthesize(frame, B)
    assert np.array_equal(L2.cpu().numpy(), ref.L) and np.array_equal(R2.cpu().numpy(), ref.R)
