"""GPU test of pstereo_synthesize_noalloc (the context-free call whose scratch
is the library's static device array): its outputs equal pstereo_synthesize's
-- and the oracle's -- on two calls in a row, the second with a smaller
frame, and a frame beyond the array's size is refused."""
import numpy as np
import pytest

import refs
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _outs(like):
    return [torch.full_like(like, 3) for _ in range(3)]


def test_noalloc_equals_context_call_twice():
    from paper_2009_09501_amd import Context, pstereo_params_init, pstereo_synthesize
    from paper_2009_09501_amd.pstereo import pstereo_synthesize_noalloc
    dev = torch.device("cuda:0")
    ctx = Context(0, 3840, 2160)
    try:
        for (w, h, seed) in ((3840, 2160, 61), (1280, 720, 62)):
            host = synth.gen_frame(seed, w, h, 40, 4.0)
            B = synth.default_disparity(w)
            f = torch.from_numpy(host).to(dev)
            p = pstereo_params_init(max_disparity=B)
            print(f"noalloc {w}x{h} seed {seed}", flush=True)
            na = _outs(f)
            pstereo_synthesize_noalloc(0, f, w, h, p, *na)
            ref = _outs(f)
            pstereo_synthesize(ctx.handle, f, w, h, p, *ref)
            torch.cuda.synchronize()
            for k, (a, b) in enumerate(zip(na, ref)):
                assert torch.equal(a, b), f"{w}x{h} output {k} differs from pstereo_synthesize"
            refs.assert_views(na, refs.views(("noalloc", seed, w, h), host, B), f"noalloc {w}x{h}")
    finally:
        ctx.close()


def test_noalloc_refuses_beyond_its_scratch():
    from paper_2009_09501_amd import pstereo_last_error, pstereo_params_init
    from paper_2009_09501_amd.pstereo import (PSTEREO_E_INVALID, PSTEREO_E_UNSUPPORTED, PSTEREO_PIPELINE,
                                              PSTEREO_PIPELINE_DEEP)
    from paper_2009_09501_amd.pstereo import pstereo_synthesize_noalloc
    dev = torch.device("cuda:0")
    f = torch.zeros((2161, 3840, 3), dtype=torch.uint8, device=dev)
    o = _outs(f)
    rc = pstereo_synthesize_noalloc(0, f, 3840, 2161, pstereo_params_init(), *o, check=False)
    assert rc == PSTEREO_E_INVALID
    assert "static scratch" in pstereo_last_error(None)
    g = f[:8]
    for fl in (PSTEREO_PIPELINE, PSTEREO_PIPELINE_DEEP):
        rc = pstereo_synthesize_noalloc(0, g, 3840, 8, pstereo_params_init(flags=fl), *_outs(g), check=False)
        assert rc == PSTEREO_E_UNSUPPORTED
    torch.cuda.synchronize()
    _ = np
