"""Seeded synthetic inputs shared by the CPU oracle tests and the GPU path."""
from .frames import (SIZES, VideoSpec, batch_mix_sizes, default_disparity,
                     gen_frame, gen_video_frame, poisson_arrivals)

__all__ = ["SIZES", "VideoSpec", "batch_mix_sizes", "default_disparity",
           "gen_frame", "gen_video_frame", "poisson_arrivals"]
