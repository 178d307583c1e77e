"""ctypes binding of libpstereo.so (the C ABI declared in include/pstereo.h).

Argument marshalling only: every step of the pipeline runs in the library's
HIP kernels.  Functions carry the C names; tensors may be passed wherever the
C ABI takes a device pointer (their ``data_ptr()`` is used).  PyTorch serves
for device memory and streams.  If the library is not built this module
raises on first use; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpstereo.so")

PSTEREO_OK = 0
PSTEREO_E_INVALID = -1
PSTEREO_E_NOMEM = -2
PSTEREO_E_DEVICE = -3
PSTEREO_E_ALIAS = -4
PSTEREO_E_UNSUPPORTED = -5
PSTEREO_E_BUSY = -6

PSTEREO_DEPTH_EXTERNAL = 0x1
PSTEREO_SYNC = 0x2
PSTEREO_PROFILE = 0x4
PSTEREO_WARP_GATHER = 0x8
PSTEREO_INPAINT_BLOCKS = 0x10
PSTEREO_PIPELINE = 0x20
PSTEREO_PIPELINE_DEEP = 0x40

PSTEREO_MAX_BLOCKS = 32768

PSTEREO_BATCH_STAGED = 0
PSTEREO_BATCH_FUSED = 1

PSTEREO_SERVE_BATCH = 0
PSTEREO_SERVE_PLAIN = 1
PSTEREO_STREAM_HOST_IO = 0x1

_CODES = {0: "OK", -1: "E_INVALID", -2: "E_NOMEM", -3: "E_DEVICE", -4: "E_ALIAS",
          -5: "E_UNSUPPORTED", -6: "E_BUSY"}

# Every symbol the header declares; tests check the library exports them all.
EXPORTED = [
    "pstereo_params_init", "pstereo_create", "pstereo_synthesize", "pstereo_destroy",
    "pstereo_last_error", "pstereo_debug_blocks", "pstereo_profile_collect",
    "pstereo_video_begin", "pstereo_video_frame", "pstereo_video_end",
    "pstereo_batch_create", "pstereo_batch_prepare", "pstereo_batch_launch", "pstereo_batch_run",
    "pstereo_batch_destroy", "pstereo_batch_last_error", "pstereo_synthesize_batch",
    "pstereo_synthesize_noalloc",
    "pstereo_batch_set_tuning", "pstereo_batch_get_tuning", "pstereo_batch_autotune",
    "pstereo_server_create", "pstereo_server_open_stream", "pstereo_server_close_stream",
    "pstereo_server_submit", "pstereo_server_poll", "pstereo_server_drain", "pstereo_server_info",
    "pstereo_server_destroy", "pstereo_server_last_error",
]


class PstereoParams(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("max_disparity", ctypes.c_int32),
        ("depth_threshold", ctypes.c_int32),
        ("block_size", ctypes.c_int32),
        ("edge_thresh", ctypes.c_int32),
        ("link_thresh", ctypes.c_int32),
        ("cbf_radius", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("depth_in", ctypes.c_void_p),
        ("out_depth", ctypes.c_void_p),
        ("out_depth_raw", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
        ("out_hsbs", ctypes.c_void_p),
    ]


class PstereoJob(ctypes.Structure):
    _fields_ = [
        ("frame", ctypes.c_void_p),
        ("w", ctypes.c_int32),
        ("h", ctypes.c_int32),
        ("out_left", ctypes.c_void_p),
        ("out_right", ctypes.c_void_p),
        ("out_anaglyph", ctypes.c_void_p),
        ("max_disparity", ctypes.c_int32),
    ]


class PstereoBatchTuning(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32),
        ("warp_lanes", ctypes.c_int32),
        ("warp_rows", ctypes.c_int32),
        ("fused_grid", ctypes.c_int32),
        ("bs_rows", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PstereoBatchTrial(ctypes.Structure):
    _fields_ = [("tuning", PstereoBatchTuning), ("ms", ctypes.c_double)]


class PstereoCompletion(ctypes.Structure):
    _fields_ = [
        ("req_id", ctypes.c_uint64),
        ("stream_id", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("t_submit", ctypes.c_double),
        ("t_launch", ctypes.c_double),
        ("t_done", ctypes.c_double),
    ]


class PstereoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load_library():
    """Load libpstereo.so from the package directory; raise if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built: run __graft_entry__.build() (hipcc for gfx950) first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ci, cu = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32
    P = ctypes.POINTER(PstereoParams)
    lib.pstereo_params_init.argtypes = [P]
    lib.pstereo_params_init.restype = ci
    lib.pstereo_create.argtypes = [ctypes.POINTER(vp), ci, ci, ci]
    lib.pstereo_create.restype = ci
    lib.pstereo_synthesize.argtypes = [vp, vp, ci, ci, P, vp, vp, vp]
    lib.pstereo_synthesize.restype = ci
    lib.pstereo_synthesize_noalloc.argtypes = [ci, vp, ci, ci, P, vp, vp, vp]
    lib.pstereo_synthesize_noalloc.restype = ci
    lib.pstereo_destroy.argtypes = [vp]
    lib.pstereo_destroy.restype = ci
    lib.pstereo_last_error.argtypes = [vp]
    lib.pstereo_last_error.restype = ctypes.c_char_p
    lib.pstereo_debug_blocks.argtypes = [vp, vp, vp, vp, ci, ctypes.POINTER(ci), ctypes.POINTER(ci)]
    lib.pstereo_debug_blocks.restype = ci
    lib.pstereo_profile_collect.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ci),
                                            ctypes.POINTER(ctypes.c_double), ci]
    lib.pstereo_profile_collect.restype = ci
    lib.pstereo_video_begin.argtypes = [vp, ci, ci, P, ctypes.POINTER(vp)]
    lib.pstereo_video_begin.restype = ci
    lib.pstereo_video_frame.argtypes = [vp, vp, vp, vp, vp]
    lib.pstereo_video_frame.restype = ci
    lib.pstereo_video_end.argtypes = [vp]
    lib.pstereo_video_end.restype = ci
    J = ctypes.POINTER(PstereoJob)
    lib.pstereo_batch_create.argtypes = [vp, ci, ctypes.c_int64, ctypes.POINTER(vp)]
    lib.pstereo_batch_create.restype = ci
    lib.pstereo_batch_prepare.argtypes = [vp, J, ci, P]
    lib.pstereo_batch_prepare.restype = ci
    lib.pstereo_batch_launch.argtypes = [vp, vp]
    lib.pstereo_batch_launch.restype = ci
    lib.pstereo_batch_run.argtypes = [vp, J, ci, P]
    lib.pstereo_batch_run.restype = ci
    lib.pstereo_batch_destroy.argtypes = [vp]
    lib.pstereo_batch_destroy.restype = ci
    lib.pstereo_batch_last_error.argtypes = [vp]
    lib.pstereo_batch_last_error.restype = ctypes.c_char_p
    lib.pstereo_synthesize_batch.argtypes = [vp, J, ci, P]
    lib.pstereo_synthesize_batch.restype = ci
    T = ctypes.POINTER(PstereoBatchTuning)
    lib.pstereo_batch_set_tuning.argtypes = [vp, T]
    lib.pstereo_batch_set_tuning.restype = ci
    lib.pstereo_batch_get_tuning.argtypes = [vp, T]
    lib.pstereo_batch_get_tuning.restype = ci
    lib.pstereo_batch_autotune.argtypes = [vp, J, ci, P, ci, T, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(PstereoBatchTrial), ci, ctypes.POINTER(ci)]
    lib.pstereo_batch_autotune.restype = ci
    lib.pstereo_server_create.argtypes = [ci, ctypes.c_int64, ci, ci, ci, ctypes.POINTER(vp)]
    lib.pstereo_server_create.restype = ci
    lib.pstereo_server_open_stream.argtypes = [vp, ci, ci, ci, ci, cu, ctypes.POINTER(ci)]
    lib.pstereo_server_open_stream.restype = ci
    lib.pstereo_server_close_stream.argtypes = [vp, ci]
    lib.pstereo_server_close_stream.restype = ci
    lib.pstereo_server_submit.argtypes = [vp, ci, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_uint64)]
    lib.pstereo_server_submit.restype = ci
    lib.pstereo_server_poll.argtypes = [vp, ctypes.POINTER(PstereoCompletion), ci, ctypes.POINTER(ci), ci]
    lib.pstereo_server_poll.restype = ci
    lib.pstereo_server_drain.argtypes = [vp]
    lib.pstereo_server_drain.restype = ci
    I64 = ctypes.POINTER(ctypes.c_int64)
    U64 = ctypes.POINTER(ctypes.c_uint64)
    lib.pstereo_server_info.argtypes = [vp, I64, I64, U64, U64]
    lib.pstereo_server_info.restype = ci
    lib.pstereo_server_destroy.argtypes = [vp]
    lib.pstereo_server_destroy.restype = ci
    lib.pstereo_server_last_error.argtypes = [vp]
    lib.pstereo_server_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _check(rc: int, ctx=None):
    if rc != PSTEREO_OK:
        msg = load_library().pstereo_last_error(ctx)
        raise PstereoError(rc, msg.decode() if msg else "")
    return rc


# ----------------------------------------------------------------- C names
def pstereo_params_init(**overrides) -> PstereoParams:
    """Defaults of the C library, then keyword overrides (field names)."""
    p = PstereoParams()
    _check(load_library().pstereo_params_init(ctypes.byref(p)))
    for k, v in overrides.items():
        if k in ("depth_in", "out_depth", "out_depth_raw", "stream", "out_hsbs"):
            v = _ptr(v) if k != "stream" else v
        setattr(p, k, v)
    return p


def pstereo_create(device: int, max_w: int, max_h: int) -> int:
    h = ctypes.c_void_p()
    _check(load_library().pstereo_create(ctypes.byref(h), device, max_w, max_h), None)
    return h.value


def pstereo_synthesize(ctx: int, frame, w: int, h: int, params: Optional[PstereoParams],
                       out_left, out_right, out_anaglyph, check: bool = True) -> int:
    rc = load_library().pstereo_synthesize(
        ctx, _ptr(frame), w, h, ctypes.byref(params) if params is not None else None,
        _ptr(out_left), _ptr(out_right), _ptr(out_anaglyph))
    return _check(rc, ctx) if check else rc


def pstereo_synthesize_noalloc(device: int, frame, w: int, h: int, params: Optional[PstereoParams],
                               out_left, out_right, out_anaglyph, check: bool = True) -> int:
    """The context-free call whose scratch is the library's static device
    array (allocates nothing); errors read with pstereo_last_error(None)."""
    rc = load_library().pstereo_synthesize_noalloc(
        device, _ptr(frame), w, h, ctypes.byref(params) if params is not None else None,
        _ptr(out_left), _ptr(out_right), _ptr(out_anaglyph))
    return _check(rc, None) if check else rc


def pstereo_destroy(ctx: int) -> int:
    return load_library().pstereo_destroy(ctx)


def pstereo_last_error(ctx: Optional[int]) -> str:
    m = load_library().pstereo_last_error(ctx)
    return m.decode() if m else ""


def pstereo_debug_blocks(ctx: int, cap: int = PSTEREO_MAX_BLOCKS):
    """(stats uint32, labels int32, dblk uint8) numpy arrays shaped [gh, gw]."""
    import numpy as np
    st = np.empty(cap, np.uint32)
    lab = np.empty(cap, np.int32)
    db = np.empty(cap, np.uint8)
    gw, gh = ctypes.c_int(), ctypes.c_int()
    _check(load_library().pstereo_debug_blocks(
        ctx, st.ctypes.data, lab.ctypes.data, db.ctypes.data, cap, ctypes.byref(gw), ctypes.byref(gh)), ctx)
    n = gw.value * gh.value
    shape = (gh.value, gw.value)
    return st[:n].reshape(shape), lab[:n].reshape(shape), db[:n].reshape(shape)


def pstereo_profile_collect(ctx: int, cap: int = 4096):
    """(ms per kernel [blockstats, regions, cbf, warp] summed, number of calls,
    list of per-call durations in ms)."""
    arr = (ctypes.c_double * 4)()
    per = (ctypes.c_double * cap)()
    n = ctypes.c_int()
    _check(load_library().pstereo_profile_collect(ctx, arr, ctypes.byref(n), per, cap), ctx)
    return [arr[i] for i in range(4)], n.value, [per[i] for i in range(min(n.value, cap))]


def pstereo_video_begin(ctx: int, w: int, h: int, params: Optional[PstereoParams]) -> int:
    v = ctypes.c_void_p()
    _check(load_library().pstereo_video_begin(ctx, w, h, ctypes.byref(params) if params is not None else None,
                                              ctypes.byref(v)), ctx)
    return v.value


def pstereo_video_frame(video: int, frame, out_left, out_right, out_anaglyph, ctx: Optional[int] = None) -> int:
    rc = load_library().pstereo_video_frame(video, _ptr(frame), _ptr(out_left), _ptr(out_right), _ptr(out_anaglyph))
    return _check(rc, ctx)


def pstereo_video_end(video: int) -> int:
    return load_library().pstereo_video_end(video)


def _bcheck(rc: int, b: int):
    if rc != PSTEREO_OK:
        m = load_library().pstereo_batch_last_error(b)
        raise PstereoError(rc, m.decode() if m else "")
    return rc


def make_jobs(frames, outs, max_disparity=None):
    """ctypes array of PstereoJob from lists of frames [h, w, 3] and output
    triples (tensors or device pointers)."""
    arr = (PstereoJob * len(frames))()
    for i, (f, o) in enumerate(zip(frames, outs)):
        h, w = int(f.shape[0]), int(f.shape[1])
        arr[i] = PstereoJob(_ptr(f), w, h, _ptr(o[0]), _ptr(o[1]), _ptr(o[2]),
                            -1 if max_disparity is None else int(max_disparity[i]))
    return arr


def pstereo_batch_create(ctx: int, max_jobs: int, max_pixels: int) -> int:
    b = ctypes.c_void_p()
    _check(load_library().pstereo_batch_create(ctx, max_jobs, max_pixels, ctypes.byref(b)), None)
    return b.value


def pstereo_batch_prepare(b: int, jobs, n: int, params: Optional[PstereoParams]) -> int:
    return _bcheck(load_library().pstereo_batch_prepare(
        b, jobs, n, ctypes.byref(params) if params is not None else None), b)


def pstereo_batch_launch(b: int, stream=None, check: bool = True) -> int:
    s = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    rc = load_library().pstereo_batch_launch(b, s)
    return _bcheck(rc, b) if check else rc


def pstereo_batch_run(b: int, jobs, n: int, params: Optional[PstereoParams], check: bool = True) -> int:
    rc = load_library().pstereo_batch_run(b, jobs, n, ctypes.byref(params) if params is not None else None)
    return _bcheck(rc, b) if check else rc


def pstereo_batch_destroy(b: int) -> int:
    return load_library().pstereo_batch_destroy(b)


def pstereo_synthesize_batch(ctx: int, jobs, n: int, params: Optional[PstereoParams], check: bool = True) -> int:
    """Views of ``n`` jobs (a ``make_jobs`` array) in one batched launch with
    the context's own batch object."""
    rc = load_library().pstereo_synthesize_batch(ctx, jobs, n, ctypes.byref(params) if params is not None else None)
    return _check(rc, ctx) if check else rc


def pstereo_batch_last_error(b: int) -> str:
    m = load_library().pstereo_batch_last_error(b)
    return m.decode() if m else ""


# ------------------------------------------------------- torch convenience
def pstereo_batch_set_tuning(b: int, mode: int = PSTEREO_BATCH_STAGED, warp_lanes: int = 256,
                             warp_rows: int = 1, fused_grid: int = 0, bs_rows: int = 0, check: bool = True) -> int:
    t = PstereoBatchTuning(mode, warp_lanes, warp_rows, fused_grid, bs_rows)
    rc = load_library().pstereo_batch_set_tuning(b, ctypes.byref(t))
    return _bcheck(rc, b) if check else rc


def pstereo_batch_get_tuning(b: int) -> dict:
    t = PstereoBatchTuning()
    _bcheck(load_library().pstereo_batch_get_tuning(b, ctypes.byref(t)), b)
    return t.as_dict()


def pstereo_batch_autotune(b: int, jobs, n: int, params: Optional[PstereoParams], reps: int = 3):
    """Time every candidate tuning on these jobs; the batch is left prepared
    with the fastest.  Returns (best tuning dict, best ms, [trial dicts])."""
    best = PstereoBatchTuning()
    best_ms = ctypes.c_double()
    trials = (PstereoBatchTrial * 64)()
    nt = ctypes.c_int()
    _bcheck(load_library().pstereo_batch_autotune(b, jobs, n, ctypes.byref(params) if params is not None else None,
                                                  reps, ctypes.byref(best), ctypes.byref(best_ms), trials, 64,
                                                  ctypes.byref(nt)), b)
    tried = [dict(trials[i].tuning.as_dict(), ms=trials[i].ms) for i in range(min(nt.value, 64))]
    return best.as_dict(), best_ms.value, tried


def _scheck(rc: int, srv):
    if rc != PSTEREO_OK:
        m = load_library().pstereo_server_last_error(srv)
        raise PstereoError(rc, m.decode() if m else "")
    return rc


def pstereo_server_create(device: int, hbm_budget_bytes: int, max_streams: int, lanes: int,
                          policy: int = PSTEREO_SERVE_BATCH) -> int:
    s = ctypes.c_void_p()
    _check(load_library().pstereo_server_create(device, hbm_budget_bytes, max_streams, lanes, policy,
                                                ctypes.byref(s)))
    return s.value


def pstereo_server_open_stream(srv: int, w: int, h: int, max_disparity: int = -1, slots: int = 4,
                               flags: int = 0, check: bool = True):
    sid = ctypes.c_int()
    rc = load_library().pstereo_server_open_stream(srv, w, h, max_disparity, slots, flags, ctypes.byref(sid))
    if not check:
        return rc, sid.value
    _scheck(rc, srv)
    return sid.value


def pstereo_server_close_stream(srv: int, stream_id: int) -> int:
    return _scheck(load_library().pstereo_server_close_stream(srv, stream_id), srv)


def pstereo_server_submit(srv: int, stream_id: int, frame, out_left, out_right, out_anaglyph,
                          check: bool = True):
    """Queue one frame; returns the request id (or (rc, id) with check=False).
    ``frame`` and outputs are tensors or raw pointers (device, or host for a
    host-I/O stream)."""
    rid = ctypes.c_uint64()
    rc = load_library().pstereo_server_submit(srv, stream_id, _ptr(frame), _ptr(out_left), _ptr(out_right),
                                              _ptr(out_anaglyph), ctypes.byref(rid))
    if not check:
        return rc, rid.value
    _scheck(rc, srv)
    return rid.value


def pstereo_server_poll(srv: int, max_n: int = 256, wait_us: int = 0):
    """List of completed requests as dicts."""
    arr = (PstereoCompletion * max(max_n, 1))()
    n = ctypes.c_int()
    _scheck(load_library().pstereo_server_poll(srv, arr, max_n, ctypes.byref(n), wait_us), srv)
    return [{"req_id": c.req_id, "stream_id": c.stream_id, "status": c.status, "t_submit": c.t_submit,
             "t_launch": c.t_launch, "t_done": c.t_done} for c in arr[:n.value]]


def pstereo_server_drain(srv: int) -> int:
    return _scheck(load_library().pstereo_server_drain(srv), srv)


def pstereo_server_info(srv: int):
    b, u = ctypes.c_int64(), ctypes.c_int64()
    sub, com = ctypes.c_uint64(), ctypes.c_uint64()
    _scheck(load_library().pstereo_server_info(srv, ctypes.byref(b), ctypes.byref(u), ctypes.byref(sub),
                                               ctypes.byref(com)), srv)
    return {"budget": b.value, "in_use": u.value, "submitted": sub.value, "completed": com.value}


def pstereo_server_destroy(srv: int) -> int:
    return load_library().pstereo_server_destroy(srv)


def pstereo_server_last_error(srv: int) -> str:
    m = load_library().pstereo_server_last_error(srv)
    return m.decode() if m else ""


class Context:
    """One library context on a GPU; frames and outputs are torch uint8 CUDA
    tensors [h, w, 3].  Work goes on torch's current stream unless a stream
    is given."""

    def __init__(self, device: int = 0, max_w: int = 7680, max_h: int = 4320):
        self.device = device
        self.handle = pstereo_create(device, max_w, max_h)

    def close(self):
        if self.handle:
            pstereo_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def synthesize(self, frame, out=None, stream=None, depth=None, out_depth=None,
                   out_depth_raw=None, out_hsbs=None, flags: int = 0, **params):
        import torch
        h, w, c = frame.shape
        assert c == 3 and frame.dtype == torch.uint8 and frame.is_contiguous()
        if out is None:
            out = tuple(torch.empty_like(frame) for _ in range(3))
        if stream is None:
            stream = torch.cuda.current_stream(frame.device)
        p = pstereo_params_init(**params)
        p.flags = flags | (PSTEREO_DEPTH_EXTERNAL if depth is not None else 0)
        p.depth_in = _ptr(depth)
        p.out_depth = _ptr(out_depth)
        p.out_depth_raw = _ptr(out_depth_raw)
        p.out_hsbs = _ptr(out_hsbs)
        p.stream = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        pstereo_synthesize(self.handle, frame, w, h, p, *out)
        return out
