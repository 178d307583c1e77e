"""MI355X (gfx950) pseudo-stereo DIBR library: HIP kernels behind a C ABI
(include/pstereo.h) and a thin ctypes binding with the same names.

Importing the package loads nothing; the shared library is loaded on first
use and its absence is an error (there is no CPU fallback).
"""
from .pstereo import (PSTEREO_DEPTH_EXTERNAL, PSTEREO_PROFILE, PSTEREO_SYNC, Context,
                      PstereoError, PstereoParams, load_library, pstereo_create,
                      pstereo_debug_blocks, pstereo_destroy, pstereo_last_error,
                      pstereo_params_init, pstereo_profile_collect, pstereo_synthesize)

__all__ = [
    "Context", "PstereoError", "PstereoParams", "load_library",
    "pstereo_params_init", "pstereo_create", "pstereo_synthesize", "pstereo_destroy",
    "pstereo_last_error", "pstereo_debug_blocks", "pstereo_profile_collect",
    "PSTEREO_DEPTH_EXTERNAL", "PSTEREO_PROFILE", "PSTEREO_SYNC",
]
