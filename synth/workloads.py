"""The named synthetic workloads: image recipe, seed, and the encode jobs
(range size B, domain step t, pool tolerance) run on each image.

A tolerance of None means exhaustive search (every domain is a candidate);
a float is the half-width of the fractal-dimension window; a negative float
asks for the adaptive window (max - min) / 3 over the image's domain values.
"""
from dataclasses import dataclass, field

import numpy as np

from .images import add_rectangles, fbm, piecewise_smooth


@dataclass(frozen=True)
class Workload:
    name: str
    description: str
    seed: int
    jobs: tuple = field(default_factory=tuple)   # ((B, t, tol), ...)
    rms: float = None    # two-level workloads: split above this RMS error (gray levels)
    color: bool = False  # interleaved RGB image (channels from color_image)


def _fbm_img(size, hurst, seed):
    return fbm(size, size, hurst, np.random.default_rng(seed))


WORKLOADS = {
    "fbm64_b8t1": Workload(
        "fbm64_b8t1",
        "64x64 fBm H=0.5; 8x8 ranges, 16x16 domains step 1; exhaustive",
        1, ((8, 1, None),)),
    "fbm512rect_b8t2": Workload(
        "fbm512rect_b8t2",
        "512x512 fBm H=0.7 + 20 rectangles; 8x8 ranges, 16x16 domains step 2; "
        "exhaustive and FD pool tol 0.05",
        2, ((8, 2, None), (8, 2, 0.05))),
    "fbm1024_b8t1": Workload(
        "fbm1024_b8t1",
        "1024x1024 fBm H=0.3; 8x8 ranges, 16x16 domains step 1; exhaustive and "
        "FD pool tol 0.02 / 0.1",
        3, ((8, 1, None), (8, 1, 0.02), (8, 1, 0.1))),
    "batch64_mixed": Workload(
        "batch64_mixed",
        "64 images, sizes U{128,256,512,1024}^2, alternating fBm H~U(0.2,0.9) and "
        "piecewise-smooth polygons with sigma=4 noise; B in {4,8} per image; step 2; "
        "FD pool tol 0.05",
        4000, ()),
    "fbm2048_twolevel": Workload(
        "fbm2048_twolevel",
        "2048x2048 fBm H=0.6; 16x16 ranges / 32x32 domains step 4 and "
        "8x8 ranges / 16x16 domains step 2; FD pool tol 0.05",
        5, ((16, 4, 0.05), (8, 2, 0.05))),
    "fbm2048_quadtree": Workload(
        "fbm2048_quadtree",
        "2048x2048 fBm H=0.6; two-level partition: 16x16 ranges / 32x32 domains step 4, "
        "ranges above 1.9 gray levels RMS split into 8x8 ranges / 16x16 domains step 2; "
        "FD pool tol 0.05 at both levels",
        5, ((16, 4, 0.05), (8, 2, 0.05)), 1.9),
    "color1024_b8t1": Workload(
        "color1024_b8t1",
        "1024x1024 RGB, channels fBm H = 0.3 / 0.5 / 0.7; 8x8 ranges, 16x16 domains step 1; "
        "FD pool tol 0.05 from the luma image",
        6, ((8, 1, 0.05),), None, True),
}


def color_image(size, seed):
    """An interleaved size x size x 3 uint8 image: three fBm channels with
    H = 0.3, 0.5, 0.7 from one generator."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(np.stack([fbm(size, size, h, rng) for h in (0.3, 0.5, 0.7)], axis=2))


def workload_images(name):
    """The single image of a one-image workload, as a C-contiguous uint8 array."""
    if name == "fbm64_b8t1":
        return _fbm_img(64, 0.5, 1)
    if name == "fbm512rect_b8t2":
        rng = np.random.default_rng(2)
        img = fbm(512, 512, 0.7, rng)
        return add_rectangles(img, 20, rng)
    if name == "fbm1024_b8t1":
        return _fbm_img(1024, 0.3, 3)
    if name in ("fbm2048_twolevel", "fbm2048_quadtree"):
        return _fbm_img(2048, 0.6, 5)
    if name == "color1024_b8t1":
        return color_image(1024, 6)
    raise KeyError(name)


def batch_descs(count=64, base_seed=4000, sizes=(128, 256, 512, 1024)):
    """The mixed batch: one (image, B, t, tol) per item.

    Each image m draws its size, range size and content from seed base+m;
    even m are fBm surfaces, odd m piecewise-smooth polygon scenes.
    """
    out = []
    for m in range(count):
        rng = np.random.default_rng(base_seed + m)
        size = int(rng.choice(sizes))
        b = int(rng.choice((4, 8)))
        if m % 2 == 0:
            img = fbm(size, size, float(rng.uniform(0.2, 0.9)), rng)
        else:
            img = piecewise_smooth(size, rng)
        out.append((img, b, 2, 0.05))
    return out
