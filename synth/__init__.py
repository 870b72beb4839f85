"""Seeded synthetic multi-camera rigs (depth, confidence, RGB) for tests and benchmarks.

This package only *generates inputs*: it ray-casts analytic scenes into depth maps and
draws confidences.  It contains none of the fusion method's arithmetic and is imported by
both the CPU oracle's tests and the GPU path's tests/bench, which is why it lives apart
from both.
"""
from .scenes import (Camera, Frame, Primitive, make_frame, make_config, ring_cameras,
                     render, CONFIGS)

__all__ = ["Camera", "Frame", "Primitive", "make_frame", "make_config", "ring_cameras",
           "render", "CONFIGS"]
