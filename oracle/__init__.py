"""CPU oracle of the pseudo-stereo DIBR pipeline (ctypes wrapper of oracle.c).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU
library and imports nothing from it.

Parity status per stage (what pins each function is listed beside it in the
tests): every stage is pinned by closed forms, invariants, library routines or
the pure-Python brute force in ``tests/brute.py``.  Parity against the paper's
own pictures is unpinned: the paper prints no pixel values.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

from .build import LIB_PATH, build_oracle

__all__ = ["OracleResult", "synthesize", "synthesize_views", "synthesize_views_mt", "auto_block", "disparity_lut",
           "weight_tables", "luma", "hsbs", "gather", "synthesize_gather", "inpaint_blocks",
           "synthesize_inpaint", "load", "build_oracle"]

_lib = None

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_i32p = ctypes.POINTER(ctypes.c_int32)


def load():
    """Load the oracle library, building it with gcc if it is not built yet."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build_oracle()
    lib = ctypes.CDLL(LIB_PATH)
    lib.oracle_synthesize.restype = ctypes.c_int
    lib.oracle_synthesize.argtypes = [
        _u8p, ctypes.c_int, ctypes.c_int,
        ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
        _u8p, _u8p, _u8p, _u8p,
        _u8p, _u32p, _i32p, _u8p, _u8p, _u8p,
        _i32p, _i32p, _i32p, _i32p]
    lib.oracle_synthesize_mt.restype = ctypes.c_int
    lib.oracle_synthesize_mt.argtypes = [
        _u8p, ctypes.c_int, ctypes.c_int,
        ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
        _u8p, _u8p, _u8p, ctypes.c_int]
    lib.oracle_auto_block.restype = ctypes.c_int
    lib.oracle_auto_block.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.oracle_disparity_lut.restype = None
    lib.oracle_disparity_lut.argtypes = [ctypes.c_int, ctypes.c_int, _i32p, _i32p, _i32p]
    lib.oracle_weight_tables.restype = None
    lib.oracle_weight_tables.argtypes = [_i32p, _i32p]
    lib.oracle_luma.restype = None
    lib.oracle_luma.argtypes = [_u8p, ctypes.c_int64, _u8p]
    lib.oracle_gather.restype = ctypes.c_int
    lib.oracle_gather.argtypes = [_u8p, _u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  _u8p, _u8p, _u8p]
    lib.oracle_inpaint_blocks.restype = ctypes.c_int
    lib.oracle_inpaint_blocks.argtypes = [_u8p, _i32p, ctypes.c_int, ctypes.c_int, _u8p]
    lib.oracle_hsbs.restype = ctypes.c_int
    lib.oracle_hsbs.argtypes = [_u8p, _u8p, ctypes.c_int, ctypes.c_int, _u8p]
    _lib = lib
    return lib


def _p(a: Optional[np.ndarray], t):
    if a is None:
        return ctypes.cast(None, t)
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(t)


@dataclass
class OracleResult:
    L: np.ndarray          # uint8 [h, w, 3] left view
    R: np.ndarray          # uint8 [h, w, 3] right view
    A: np.ndarray          # uint8 [h, w, 3] red-cyan anaglyph
    Y: np.ndarray          # uint8 [h, w] luma
    D0: np.ndarray         # uint8 [h, w] depth map before filtering
    Df: np.ndarray         # uint8 [h, w] filtered depth
    stats: np.ndarray      # uint32 [gh, gw] block means | edge << 24
    labels: np.ndarray     # int32 [gh, gw] region label (min block index)
    dblk: np.ndarray       # uint8 [gh, gw] region depth per block
    warpL: np.ndarray      # int32 [h, w] winning source x before filling, -1 = hole
    warpR: np.ndarray
    srcL: np.ndarray       # int32 [h, w] source x of the final colour
    srcR: np.ndarray
    K: int


def auto_block(w: int, h: int) -> int:
    return load().oracle_auto_block(w, h)


def synthesize(frame: np.ndarray, B: int, T: int = 150, K: int = 0, g: int = 24,
               tau: int = 24, r: int = 2,
               depth: Optional[np.ndarray] = None) -> OracleResult:
    """Run the whole pipeline on one RGB24 frame ``[h, w, 3]`` uint8.

    ``depth`` (uint8 [h, w]), when given, replaces the generated depth map D0;
    the cross-bilateral filter still runs (radius ``r``; r = 0 passes it
    through unchanged)."""
    lib = load()
    frame = np.ascontiguousarray(frame, dtype=np.uint8)
    h, w, c = frame.shape
    assert c == 3
    Kr = K if K else lib.oracle_auto_block(w, h)
    if Kr < 1:
        raise ValueError("no block size fits this frame")
    gw, gh = -(-w // Kr), -(-h // Kr)
    out = {n: np.empty((h, w, 3), np.uint8) for n in ("L", "R", "A")}
    Y = np.empty((h, w), np.uint8)
    D0 = np.empty((h, w), np.uint8)
    Df = np.empty((h, w), np.uint8)
    stats = np.empty((gh, gw), np.uint32)
    labels = np.empty((gh, gw), np.int32)
    dblk = np.empty((gh, gw), np.uint8)
    wl, wr_, sl, sr = (np.empty((h, w), np.int32) for _ in range(4))
    dep = None
    if depth is not None:
        dep = np.ascontiguousarray(depth, dtype=np.uint8)
        assert dep.shape == (h, w)
    rc = lib.oracle_synthesize(
        _p(frame, _u8p), w, h, B, T, Kr, g, tau, r, _p(dep, _u8p),
        _p(out["L"], _u8p), _p(out["R"], _u8p), _p(out["A"], _u8p),
        _p(Y, _u8p), _p(stats, _u32p), _p(labels, _i32p), _p(dblk, _u8p),
        _p(D0, _u8p), _p(Df, _u8p),
        _p(wl, _i32p), _p(wr_, _i32p), _p(sl, _i32p), _p(sr, _i32p))
    if rc != 0:
        raise ValueError(f"oracle_synthesize failed with code {rc}")
    return OracleResult(out["L"], out["R"], out["A"], Y, D0, Df, stats, labels,
                        dblk, wl, wr_, sl, sr, Kr)


def synthesize_views(frame: np.ndarray, B: int, **kw):
    """(L, R, A) only, with no stage dumps (the timed CPU-baseline form)."""
    lib = load()
    frame = np.ascontiguousarray(frame, dtype=np.uint8)
    h, w, _ = frame.shape
    K = kw.get("K", 0) or lib.oracle_auto_block(w, h)
    L, R, A = (np.empty((h, w, 3), np.uint8) for _ in range(3))
    rc = lib.oracle_synthesize(
        _p(frame, _u8p), w, h, B, kw.get("T", 150), K, kw.get("g", 24),
        kw.get("tau", 24), kw.get("r", 2), _p(None, _u8p),
        _p(L, _u8p), _p(R, _u8p), _p(A, _u8p),
        _p(None, _u8p), _p(None, _u32p), _p(None, _i32p), _p(None, _u8p),
        _p(None, _u8p), _p(None, _u8p),
        _p(None, _i32p), _p(None, _i32p), _p(None, _i32p), _p(None, _i32p))
    if rc != 0:
        raise ValueError(f"oracle_synthesize failed with code {rc}")
    return L, R, A


def synthesize_views_mt(frame: np.ndarray, B: int, nthreads: int, **kw):
    """(L, R, A) with the row-independent stages split over ``nthreads``
    threads (the CPU baseline's row-parallel mode); equal to
    synthesize_views for any thread count."""
    lib = load()
    frame = np.ascontiguousarray(frame, dtype=np.uint8)
    h, w, _ = frame.shape
    K = kw.get("K", 0) or lib.oracle_auto_block(w, h)
    L, R, A = (np.empty((h, w, 3), np.uint8) for _ in range(3))
    rc = lib.oracle_synthesize_mt(
        _p(frame, _u8p), w, h, B, kw.get("T", 150), K, kw.get("g", 24),
        kw.get("tau", 24), kw.get("r", 2), _p(L, _u8p), _p(R, _u8p), _p(A, _u8p), int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_synthesize_mt failed with code {rc}")
    return L, R, A


def disparity_lut(B: int, T: int = 150):
    """(P, oL, oR) int32[256]: total parallax and per-view offsets per depth."""
    P, oL, oR = (np.empty(256, np.int32) for _ in range(3))
    load().oracle_disparity_lut(B, T, _p(P, _i32p), _p(oL, _i32p), _p(oR, _i32p))
    return P, oL, oR


def weight_tables():
    """(ws[0..18], wr[0..255]) of the cross-bilateral filter."""
    ws = np.empty(19, np.int32)
    wr = np.empty(256, np.int32)
    load().oracle_weight_tables(_p(ws, _i32p), _p(wr, _i32p))
    return ws, wr


def luma(rgb: np.ndarray) -> np.ndarray:
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    n = rgb.size // 3
    out = np.empty(rgb.shape[:-1], np.uint8)
    load().oracle_luma(_p(rgb, _u8p), n, _p(out, _u8p))
    return out


def hsbs(L: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Half side-by-side frame of a stereo pair (oracle_hsbs)."""
    L = np.ascontiguousarray(L, dtype=np.uint8)
    R = np.ascontiguousarray(R, dtype=np.uint8)
    h, w, _ = L.shape
    out = np.empty_like(L)
    rc = load().oracle_hsbs(_p(L, _u8p), _p(R, _u8p), w, h, _p(out, _u8p))
    if rc != 0:
        raise ValueError(f"oracle_hsbs failed with code {rc}")
    return out


def gather(frame: np.ndarray, Df: np.ndarray, B: int, T: int = 150):
    """(L, R, A) by the Fig. 3 gather at the destination's filtered depth."""
    frame = np.ascontiguousarray(frame, dtype=np.uint8)
    Df = np.ascontiguousarray(Df, dtype=np.uint8)
    h, w, _ = frame.shape
    L, R, A = (np.empty((h, w, 3), np.uint8) for _ in range(3))
    rc = load().oracle_gather(_p(frame, _u8p), _p(Df, _u8p), w, h, B, T, _p(L, _u8p), _p(R, _u8p), _p(A, _u8p))
    if rc != 0:
        raise ValueError(f"oracle_gather failed with code {rc}")
    return L, R, A


def synthesize_gather(frame: np.ndarray, B: int, T: int = 150, K: int = 0, g: int = 24, tau: int = 24,
                      r: int = 2, depth: Optional[np.ndarray] = None):
    """The pipeline with the Fig. 3 gather in place of the z-buffered warp and
    the fill: depth stages as in synthesize, then gather(frame, Df)."""
    res = synthesize(frame, B, T, K, g, tau, r, depth=depth)
    return gather(frame, res.Df, B, T)


def inpaint_blocks(frame: np.ndarray, warp: np.ndarray):
    """(view, sweeps): block-iterative inpainting of one warped view (warp:
    winning source x per destination, -1 = hole)."""
    frame = np.ascontiguousarray(frame, dtype=np.uint8)
    warp = np.ascontiguousarray(warp, dtype=np.int32)
    h, w, _ = frame.shape
    out = np.empty_like(frame)
    rc = load().oracle_inpaint_blocks(_p(frame, _u8p), _p(warp, _i32p), w, h, _p(out, _u8p))
    if rc < 0:
        raise ValueError(f"oracle_inpaint_blocks failed with code {rc}")
    return out, rc


def synthesize_inpaint(frame: np.ndarray, B: int, T: int = 150, K: int = 0, g: int = 24, tau: int = 24,
                       r: int = 2, depth: Optional[np.ndarray] = None):
    """(L, R, A) with the block-iterative inpainting in place of the row fill:
    the same depth stages and forward warp as synthesize, then
    inpaint_blocks per view; the anaglyph from the inpainted views."""
    res = synthesize(frame, B, T, K, g, tau, r, depth=depth)
    L, _ = inpaint_blocks(frame, res.warpL)
    R, _ = inpaint_blocks(frame, res.warpR)
    A = R.copy()
    A[..., 0] = L[..., 0]
    return L, R, A
