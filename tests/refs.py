"""Oracle views for the GPU tests, computed once per input.

The row-parallel oracle (equal to the single-thread one: pinned in
test_oracle_pins) on the host's cores, cached by a caller-given key so that
several launch forms of one input compare with one oracle run."""
from __future__ import annotations

import os

import numpy as np

import oracle

_THREADS = max(1, min(16, len(os.sched_getaffinity(0))))
_cache = {}


def views(key, frame: np.ndarray, B: int, **kw):
    """(L, R, A) of the oracle for ``frame``; ``key`` names the input (for
    example its generator seed and size) and the parameters."""
    k = (key, B, tuple(sorted(kw.items())))
    if k not in _cache:
        _cache[k] = oracle.synthesize_views_mt(frame, B, _THREADS, **kw)
    return _cache[k]


def assert_views(got, want, what: str):
    """Bit-exact comparison of three output images (numpy or CPU tensors)."""
    for name, g, w in zip(("left", "right", "anaglyph"), got, want):
        g = g.cpu().numpy() if hasattr(g, "cpu") else g
        if not np.array_equal(g, w):
            diff = (g != w).any(-1)
            ys, xs = np.nonzero(diff)
            raise AssertionError(f"{what}: {name} differs from the oracle at {int(diff.sum())} px, "
                                 f"first (y={ys[0]}, x={xs[0]})")
