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


_BAND = 128  # rows generated at a time (keeps temporaries in cache)


def _gradient_band(w: int, h: int, y0: int, y1: int, c00, c10, c01) -> np.ndarray:
    """Rows y0..y1-1 of the linear horizontal + vertical gradient, float32."""
    c00 = np.asarray(c00, np.float32)
    c10 = np.asarray(c10, np.float32)
    c01 = np.asarray(c01, np.float32)
    fx = (np.arange(w, dtype=np.float32) / np.float32(max(w - 1, 1)))[None, :, None]
    fy = (np.arange(y0, y1, dtype=np.float32) / np.float32(max(h - 1, 1)))[:, None, None]
    return c00 + (c10 - c00) * fx + (c01 - c00) * fy


def _paint(band: np.ndarray, y0: int, kind: int, cx: float, cy: float, rx: float,
           ry: float, colour) -> None:
    """Paint the part of one opaque axis-aligned ellipse (kind 0) or rectangle
    (kind 1) that falls in the band of rows starting at image row y0."""
    hb, w = band.shape[:2]
    x0 = max(int(math.floor(cx - rx)), 0)
    x1 = min(int(math.ceil(cx + rx)) + 1, w)
    ya = max(int(math.floor(cy - ry)), y0)
    yb = min(int(math.ceil(cy + ry)) + 1, y0 + hb)
    if x0 >= x1 or ya >= yb:
        return
    xs = np.arange(x0, x1, dtype=np.float32)[None, :]
    ys = np.arange(ya, yb, dtype=np.float32)[:, None]
    if kind == 0:
        m = ((xs - np.float32(cx)) / np.float32(rx)) ** 2 + ((ys - np.float32(cy)) / np.float32(ry)) ** 2 <= 1.0
    else:
        m = (np.abs(xs - np.float32(cx)) <= rx) & (np.abs(ys - np.float32(cy)) <= ry)
    band[ya - y0:yb - y0, x0:x1][m] = np.asarray(colour, np.float32)


def _render(w: int, h: int, corners, shapes, noise_rng: np.random.Generator,
            sigma: float) -> np.ndarray:
    """Gradient, then the shapes in draw order, then N(0, sigma^2) noise per
    pixel and channel (drawn band by band in row order), rounded to the
    nearest integer and clipped to [0, 255]."""
    out = np.empty((h, w, 3), np.uint8)
    for y0 in range(0, h, _BAND):
        y1 = min(y0 + _BAND, h)
        band = _gradient_band(w, h, y0, y1, *corners)
        for sh in shapes:
            _paint(band, y0, *sh)
        if sigma > 0:
            band += noise_rng.standard_normal(band.shape, dtype=np.float32) * np.float32(sigma)
        np.rint(band, out=band)
        np.clip(band, 0, 255, out=band)
        out[y0:y1] = band
    return out


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
    corners = [rng.integers(0, 256, 3) for _ in range(3)]
    shapes = []
    for _ in range(n_shapes):
        kind = 0 if rng.random() < 0.5 else 1
        cx = rng.uniform(0, w)
        cy = rng.uniform(0, h)
        rx = rng.uniform(max(w / 64, 0.5), max(w / 8, 1.0))
        ry = rng.uniform(max(h / 64, 0.5), max(h / 8, 1.0))
        colour = rng.integers(0, 256, 3)
        shapes.append((kind, cx, cy, rx, ry, colour))
    return _render(w, h, corners, shapes, rng, sigma)


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
        pos = self.p0 + t * self.v
        pos[:, 0] %= self.w
        pos[:, 1] %= self.h
        shapes = [(0, float(pos[i, 0]), float(pos[i, 1]), float(self.rx[i]), float(self.ry[i]),
                   self.colour[i]) for i in range(len(pos))]
        return _render(self.w, self.h, corners, shapes, np.random.default_rng([self.seed, t]), self.sigma)


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
