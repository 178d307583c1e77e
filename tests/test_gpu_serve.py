"""GPU tests of the continuous-batching server: every served frame equals the
oracle's views of that frame and the same frame run alone through the plain
call, whatever else was in flight (device and host-I/O streams); admission
follows the HBM budget; requests beyond a stream's slots wait and still
complete correctly."""
import numpy as np
import pytest

import refs
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2009_09501_amd import Context
    c = Context(0, 3840, 2160)
    yield c
    c.close()


def _alone(ctx, f):
    L, R, A = ctx.synthesize(f, max_disparity=synth.default_disparity(f.shape[1]))
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (L, R, A)]


@pytest.mark.parametrize("policy", ["batch", "plain"])
def test_served_equals_alone(ctx, policy):
    from paper_2009_09501_amd.pstereo import (PSTEREO_SERVE_BATCH, PSTEREO_SERVE_PLAIN, PSTEREO_STREAM_HOST_IO,
                                              pstereo_server_create, pstereo_server_destroy, pstereo_server_drain,
                                              pstereo_server_open_stream, pstereo_server_poll, pstereo_server_submit)
    dev = torch.device("cuda:0")
    pol = PSTEREO_SERVE_BATCH if policy == "batch" else PSTEREO_SERVE_PLAIN
    print(f"server policy {policy}: streams 1920x1080, 640x360 (device), 1280x720 (host I/O)", flush=True)
    srv = pstereo_server_create(0, 4 << 30, 8, 3, pol)
    try:
        specs = [(1920, 1080, 0, 2), (640, 360, 0, 3), (1280, 720, PSTEREO_STREAM_HOST_IO, 2)]
        sids = [pstereo_server_open_stream(srv, w, h, -1, slots, fl) for w, h, fl, slots in specs]
        jobs = []  # (sid, frame on device, frame submitted, outputs, oracle views)
        for k in range(5):
            for (w, h, fl, _), sid in zip(specs, sids):
                host = synth.VideoSpec(60 + sid, w, h, frames=20).frame(k)
                want = refs.views(("serve", 60 + sid, w, h, k), host, synth.default_disparity(w))
                fdev = torch.from_numpy(host).to(dev)
                if fl:
                    fin = torch.from_numpy(host).pin_memory()
                    outs = [torch.empty(host.shape, dtype=torch.uint8, pin_memory=True) for _ in range(3)]
                else:
                    fin = fdev
                    outs = [torch.empty_like(fdev) for _ in range(3)]
                jobs.append((sid, fdev, fin, outs, want))
        torch.cuda.synchronize()
        ids = [pstereo_server_submit(srv, sid, fin, *outs) for sid, _, fin, outs, _ in jobs]
        pstereo_server_drain(srv)
        done = pstereo_server_poll(srv, 256)
        assert sorted(c["req_id"] for c in done) == sorted(ids)
        assert all(c["status"] == 0 for c in done)
        assert all(c["t_submit"] <= c["t_launch"] <= c["t_done"] for c in done)
        for i, (sid, fdev, _, outs, want) in enumerate(jobs):
            refs.assert_views(outs, want, f"{policy} job {i} stream {sid}")
            ref = _alone(ctx, fdev)
            for v, (got, want) in enumerate(zip(outs, ref)):
                g = got.cpu().numpy()
                assert np.array_equal(g, want), f"job {i} stream {sid} output {v}: {(g != want).any(-1).sum()} px"
    finally:
        pstereo_server_destroy(srv)


def test_budget_admission_and_release():
    from paper_2009_09501_amd.pstereo import (PSTEREO_E_NOMEM, pstereo_server_close_stream, pstereo_server_create,
                                              pstereo_server_destroy, pstereo_server_info,
                                              pstereo_server_open_stream)
    srv = pstereo_server_create(0, 64 << 20, 8, 2)
    try:
        a = pstereo_server_open_stream(srv, 1920, 1080, -1, 2)       # ~5 MB of scratch
        rc, _ = pstereo_server_open_stream(srv, 3840, 2160, -1, 8, check=False)  # ~70 MB
        assert rc == PSTEREO_E_NOMEM
        used = pstereo_server_info(srv)["in_use"]
        pstereo_server_close_stream(srv, a)
        assert pstereo_server_info(srv)["in_use"] < used
        b = pstereo_server_open_stream(srv, 3840, 2160, -1, 5)
        assert b >= 0
        assert pstereo_server_info(srv)["in_use"] <= 64 << 20
    finally:
        pstereo_server_destroy(srv)


def test_requests_wait_for_slots():
    """One slot per stream and a burst of submissions: requests queue, run as
    slots free up, and every result is right."""
    from paper_2009_09501_amd import Context
    from paper_2009_09501_amd.pstereo import (pstereo_server_create, pstereo_server_destroy, pstereo_server_drain,
                                              pstereo_server_open_stream, pstereo_server_poll, pstereo_server_submit)
    dev = torch.device("cuda:0")
    spec = synth.VideoSpec(77, 960, 540, frames=16)
    host = [spec.frame(t) for t in range(12)]
    frames = [torch.from_numpy(f).to(dev) for f in host]
    outs = [[torch.empty_like(f) for _ in range(3)] for f in frames]
    srv = pstereo_server_create(0, 1 << 30, 2, 4)
    ctx = Context(0, 960, 540)
    try:
        sid = pstereo_server_open_stream(srv, 960, 540, -1, 1)
        for f, o in zip(frames, outs):
            pstereo_server_submit(srv, sid, f, *o)
        pstereo_server_drain(srv)
        done = pstereo_server_poll(srv, 64)
        assert len(done) == 12
        # one slot: the requests ran one after another, in submission order
        done.sort(key=lambda c: c["req_id"])
        for a, b in zip(done, done[1:]):
            assert a["t_done"] <= b["t_launch"] + 1e-9
        for t, (f, o) in enumerate(zip(frames, outs)):
            refs.assert_views(o, refs.views(("serve", 77, 960, 540, t), host[t], synth.default_disparity(960)),
                              f"queued request {t}")
            ref = _alone(ctx, f)
            for got, want in zip(o, ref):
                assert np.array_equal(got.cpu().numpy(), want)
    finally:
        pstereo_server_destroy(srv)
        ctx.close()


def test_served_mix_of_sizes_vs_oracle():
    """Eight streams of 1080p / 4K / 8K frames, two requests each, submitted at
    once to a batching server with four lanes: every result equals the
    oracle's (the frames run in batches of mixed sizes, overlapping on the
    lanes)."""
    from paper_2009_09501_amd.pstereo import (PSTEREO_SERVE_BATCH, pstereo_server_create, pstereo_server_destroy,
                                              pstereo_server_drain, pstereo_server_open_stream,
                                              pstereo_server_poll, pstereo_server_submit)
    dev = torch.device("cuda:0")
    sizes = [(1920, 1080), (3840, 2160), (7680, 4320), (3840, 2160), (1920, 1080), (3840, 2160), (1920, 1080),
             (7680, 4320)]
    srv = pstereo_server_create(0, 32 << 30, 8, 4, PSTEREO_SERVE_BATCH)
    try:
        sids = [pstereo_server_open_stream(srv, w, h, -1, 2) for w, h in sizes]
        jobs = []
        for k in range(2):
            for sid, (w, h) in zip(sids, sizes):
                host = synth.VideoSpec(6000 + sid, w, h, frames=300).frame(100 * k)
                jobs.append((sid, host, torch.from_numpy(host).to(dev)))
        outs = [[torch.empty_like(d) for _ in range(3)] for _, _, d in jobs]
        torch.cuda.synchronize()
        print("serving 16 requests of 8 streams (1080p/4K/8K) at once", flush=True)
        for (sid, _, d), o in zip(jobs, outs):
            pstereo_server_submit(srv, sid, d, *o)
        pstereo_server_drain(srv)
        done = pstereo_server_poll(srv, 64)
        assert len(done) == 16 and all(c["status"] == 0 for c in done)
        for i, ((sid, host, _), o) in enumerate(zip(jobs, outs)):
            w = host.shape[1]
            want = refs.views(("serve", 6000 + sid, w, host.shape[0], i // 8), host, synth.default_disparity(w))
            refs.assert_views(o, want, f"mixed serving request {i} (stream {sid}, {w}x{host.shape[0]})")
    finally:
        pstereo_server_destroy(srv)


def test_server_rejects():
    from paper_2009_09501_amd.pstereo import (PSTEREO_E_ALIAS, PSTEREO_E_INVALID, PSTEREO_E_UNSUPPORTED,
                                              pstereo_server_create, pstereo_server_destroy,
                                              pstereo_server_open_stream, pstereo_server_submit)
    dev = torch.device("cuda:0")
    srv = pstereo_server_create(0, 1 << 30, 2, 2)
    try:
        rc, _ = pstereo_server_open_stream(srv, 642, 360, -1, 2, check=False)
        assert rc == PSTEREO_E_UNSUPPORTED
        sid = pstereo_server_open_stream(srv, 640, 360, -1, 2)
        f = torch.zeros((360, 640, 3), dtype=torch.uint8, device=dev)
        o = [torch.empty_like(f) for _ in range(3)]
        host = torch.zeros((360, 640, 3), dtype=torch.uint8)
        assert pstereo_server_submit(srv, sid, host, *o, check=False)[0] == PSTEREO_E_INVALID
        assert pstereo_server_submit(srv, sid, f, o[0], o[0], o[2], check=False)[0] == PSTEREO_E_ALIAS
        assert pstereo_server_submit(srv, 1, f, *o, check=False)[0] == PSTEREO_E_INVALID
    finally:
        pstereo_server_destroy(srv)
