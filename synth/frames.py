"""Seeded synthetic RGB24 frames shaped like the paper's workloads.

The paper measures 4K camera stills and a 3840x2160 60 fps demo video
(Section 5); neither is available, so these generators stand in for them with
content that exercises every stage of the method: smooth gradient backgrounds
(one large region whose depth follows the row ramp), opaque ellipses and
rectangles (object regions whose borders are edge blocks), and per-pixel
Gaussian noise.

This module holds no arithmetic of the pseudo-stereo method itself.  It is the
only code shared by the CPU oracle tests and the GPU path: both sides receive
the same uint8 arrays from here.

All randomness comes from ``numpy.random.default_rng`` (PCG64) seeded by the
caller, so a (seed, size, ...) tuple names a frame exactly.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "gen_frame",
    "gen_video_frame",
    "VideoSpec",
    "default_disparity",
    "batch_mix_sizes",
    "poisson_arrivals",
    "SIZES",
]

# Resolutions of the uneven-batch and serving workloads (width, height).
SIZES = {
    "720p": (1280, 720),
    "1080p": (1920, 1080),
    "1440p": (2560, 1440),
    "4k": (3840, 2160),
    "8k": (7680, 4320),
}


def default_disparity(width: int) -> int:
    """Maximum total disparity of 2 % of the width, rounded half up."""
    return (2 * width + 50) // 100


def _gradient(w: int, h: int, c00, c10, c01) -> np.ndarray:
    """Linear horizontal + vertical gradient, float32 [h, w, 3]."""
    c00 = np.asarray(c00, np.float32)
    c10 = np.asarray(c10, np.float32)
    c01 = np.asarray(c01, np.float32)
    fx = (np.arange(w, dtype=np.float32) / max(w - 1, 1))[None, :, None]
    fy = (np.arange(h, dtype=np.float32) / max(h - 1, 1))[:, None, None]
    return c00 + (c10 - c00) * fx + (c01 - c00) * fy


def _paint(img: np.ndarray, kind: int, cx: float, cy: float, rx: float,
           ry: float, colour) -> None:
    """Paint one opaque axis-aligned ellipse (kind 0) or rectangle (kind 1)."""
    h, w = img.shape[:2]
    x0 = max(int(math.floor(cx - rx)), 0)
    x1 = min(int(math.ceil(cx + rx)) + 1, w)
    y0 = max(int(math.floor(cy - ry)), 0)
    y1 = min(int(math.ceil(cy + ry)) + 1, h)
    if x0 >= x1 or y0 >= y1:
        return
    xs = np.arange(x0, x1, dtype=np.float32)[None, :]
    ys = np.arange(y0, y1, dtype=np.float32)[:, None]
    if kind == 0:
        m = ((xs - cx) / rx) ** 2 + ((ys - cy) / ry) ** 2 <= 1.0
    else:
        m = (np.abs(xs - cx) <= rx) & (np.abs(ys - cy) <= ry)
    img[y0:y1, x0:x1][m] = np.asarray(colour, np.float32)


def _finish(img: np.ndarray, rng: np.random.Generator, sigma: float) -> np.ndarray:
    if sigma > 0:
        img += rng.standard_normal(img.shape, dtype=np.float32) * np.float32(sigma)
    np.rint(img, out=img)
    np.clip(img, 0, 255, out=img)
    return img.astype(np.uint8)


def gen_frame(seed: int, w: int, h: int, n_shapes: int = 12,
              sigma: float = 4.0) -> np.ndarray:
    """One still frame, uint8 [h, w, 3] (RGB24, row pitch 3*w).

    Background: per-channel linear gradient between three random corner
    colours.  Then ``n_shapes`` shapes in draw order, each an ellipse or a
    rectangle with probability 1/2, centre uniform in the frame, half-axes
    uniform in [w/64, w/8) x [h/64, h/8), uniform random colour, painted
    opaque.  Finally N(0, sigma^2) noise per pixel and channel, rounded to the
    nearest integer and clipped to [0, 255].
    """
    if w < 1 or h < 1:
        raise ValueError("frame size must be positive")
    rng = np.random.default_rng(seed)
    c00, c10, c01 = (rng.integers(0, 256, 3) for _ in range(3))
    img = _gradient(w, h, c00, c10, c01)
    for _ in range(n_shapes):
        kind = 0 if rng.random() < 0.5 else 1
        cx = rng.uniform(0, w)
        cy = rng.uniform(0, h)
        rx = rng.uniform(max(w / 64, 0.5), max(w / 8, 1.0))
        ry = rng.uniform(max(h / 64, 0.5), max(h / 8, 1.0))
        colour = rng.integers(0, 256, 3)
        _paint(img, kind, cx, cy, rx, ry, colour)
    return _finish(img, rng, sigma)


class VideoSpec:
    """Moving-ellipse video: ``n`` ellipses translate 1-8 px/frame on random
    headings over a gradient whose corner colours drift linearly from one
    random set to another across ``frames`` frames; per-frame noise sigma.
    Frame ``t`` is produced on demand by :meth:`frame` (frames are independent
    given the spec, so any subset can be generated in any order)."""

    def __init__(self, seed: int, w: int, h: int, frames: int = 300,
                 n: int = 40, sigma: float = 3.0):
        self.seed, self.w, self.h, self.frames = seed, w, h, frames
        self.sigma = sigma
        rng = np.random.default_rng(seed)
        self.c_start = [rng.integers(0, 256, 3) for _ in range(3)]
        self.c_end = [rng.integers(0, 256, 3) for _ in range(3)]
        self.p0 = np.stack([rng.uniform(0, w, n), rng.uniform(0, h, n)], 1)
        speed = rng.uniform(1.0, 8.0, n)
        head = rng.uniform(0.0, 2.0 * math.pi, n)
        self.v = np.stack([speed * np.cos(head), speed * np.sin(head)], 1)
        self.rx = rng.uniform(max(w / 64, 0.5), max(w / 8, 1.0), n)
        self.ry = rng.uniform(max(h / 64, 0.5), max(h / 8, 1.0), n)
        self.colour = rng.integers(0, 256, (n, 3))

    def frame(self, t: int) -> np.ndarray:
        a = t / max(self.frames - 1, 1)
        corners = [(1 - a) * s + a * e for s, e in zip(self.c_start, self.c_end)]
        img = _gradient(self.w, self.h, *corners)
        pos = self.p0 + t * self.v
        pos[:, 0] %= self.w
        pos[:, 1] %= self.h
        for i in range(len(pos)):
            _paint(img, 0, float(pos[i, 0]), float(pos[i, 1]),
                   float(self.rx[i]), float(self.ry[i]), self.colour[i])
        rng = np.random.default_rng([self.seed, t])
        return _finish(img, rng, self.sigma)


def gen_video_frame(seed: int, w: int, h: int, t: int, frames: int = 300,
                    n: int = 40, sigma: float = 3.0) -> np.ndarray:
    """Frame ``t`` of the moving-ellipse video named by (seed, w, h, frames)."""
    return VideoSpec(seed, w, h, frames, n, sigma).frame(t)


def batch_mix_sizes(seed: int = 5, count: int = 64):
    """Resolutions of the uneven batch: ``count`` draws over
    {720p, 1080p, 1440p, 4K, 8K} with weights {.2, .3, .2, .2, .1}."""
    names = ["720p", "1080p", "1440p", "4k", "8k"]
    rng = np.random.default_rng(seed)
    idx = rng.choice(5, count, p=[0.2, 0.3, 0.2, 0.2, 0.1])
    return [SIZES[names[i]] for i in idx]


def poisson_arrivals(seed: int, fps: float, duration_s: float) -> np.ndarray:
    """Arrival times (s) of a Poisson process with rate ``fps`` on
    [0, duration_s): exponential inter-arrival gaps with mean 1/fps."""
    rng = np.random.default_rng(seed)
    n_max = int(fps * duration_s * 2 + 32)
    t = np.cumsum(rng.exponential(1.0 / fps, n_max))
    return t[t < duration_s]
