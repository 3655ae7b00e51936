"""Seeded synthetic inputs (frames, pattern images, arrival schedules)."""
from .frames import (FrameSpec, make_frame, make_frames, fig6_pattern_image,
                     stream_schedule, stream_frame_spec, CONFIGS, FIG6_CASES,
                     brief_pattern)

__all__ = ["FrameSpec", "make_frame", "make_frames", "fig6_pattern_image",
           "stream_schedule", "stream_frame_spec", "CONFIGS", "FIG6_CASES",
           "brief_pattern"]
