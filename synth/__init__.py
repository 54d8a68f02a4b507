"""Seeded synthetic grayscale images for the PIFS range-domain search.

This package only draws pixels. It holds none of the encoder's arithmetic
(no block sums, no isometries, no fractal dimensions, no error terms), so the
oracle and the GPU path can both take their inputs from it without sharing any
of the method.
"""
from .images import fbm, add_rectangles, piecewise_smooth, image_sha256  # noqa: F401
from .workloads import WORKLOADS, Workload, workload_images, batch_descs  # noqa: F401
