"""Image generators: fractional Brownian surfaces, sharp-edged rectangles and
piecewise-smooth polygon scenes, all uint8 and fully determined by a seed.

The paper measures on natural photographs that are not available here; these
stand in for them with the same sizes and a controllable roughness (Hurst
exponent), plus the sharp edges and smooth gradients that natural scenes mix.
"""
import hashlib

import numpy as np


def _to_u8_round_half_up(x):
    return np.floor(x + 0.5).astype(np.uint8)


def fbm(height, width, hurst, rng):
    """Spectral synthesis of a fractional Brownian surface.

    Amplitude f^-(H+1) on the radial frequency f (power ~ f^-(2H+2)), zero at
    DC, complex Gaussian coefficients, real part of the inverse FFT, then
    min-max scaled to 0..255 with round-half-up.
    """
    fy = np.fft.fftfreq(height)[:, None]
    fx = np.fft.fftfreq(width)[None, :]
    f = np.sqrt(fx * fx + fy * fy)
    amp = np.zeros_like(f)
    nz = f > 0
    amp[nz] = f[nz] ** (-(hurst + 1.0))
    coef = amp * (rng.standard_normal((height, width))
                  + 1j * rng.standard_normal((height, width)))
    field = np.real(np.fft.ifft2(coef))
    lo, hi = field.min(), field.max()
    x = (field - lo) / (hi - lo) if hi > lo else np.zeros_like(field)
    return _to_u8_round_half_up(255.0 * x)


def add_rectangles(img, count, rng):
    """Paint `count` axis-aligned rectangles of uniform random intensity, in
    order, with corners drawn uniformly over the image."""
    out = img.copy()
    h, w = out.shape
    for _ in range(count):
        y0, y1 = np.sort(rng.integers(0, h + 1, size=2))
        x0, x1 = np.sort(rng.integers(0, w + 1, size=2))
        out[y0:y1, x0:x1] = rng.integers(0, 256)
    return out


def _even_odd_mask(verts, h, w):
    py = np.arange(h, dtype=np.float64)[:, None] + 0.5
    px = np.arange(w, dtype=np.float64)[None, :] + 0.5
    inside = np.zeros((h, w), dtype=bool)
    nv = len(verts)
    for e in range(nv):
        x1, y1 = verts[e]
        x2, y2 = verts[(e + 1) % nv]
        if y1 == y2:
            continue
        crosses = (y1 > py) != (y2 > py)
        xint = (x2 - x1) * (py - y1) / (y2 - y1) + x1
        inside ^= crosses & (px < xint)
    return inside


def piecewise_smooth(size, rng, noise_sigma=4.0):
    """Random polygons (4..12 of them, 3..7 vertices, even-odd fill), each
    filled with a linear gradient a + b*x + c*y, over a gradient background;
    then Gaussian noise, clipping and round-half-up."""
    n = size
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)

    def gradient():
        a = rng.uniform(0.0, 255.0)
        b, c = rng.uniform(-1.0, 1.0, size=2) * 255.0 / n
        return a + b * xx + c * yy

    canvas = gradient()
    for _ in range(int(rng.integers(4, 13))):
        nv = int(rng.integers(3, 8))
        verts = rng.uniform(0.0, n, size=(nv, 2))
        mask = _even_odd_mask(verts, n, n)
        canvas = np.where(mask, gradient(), canvas)
    canvas = canvas + rng.normal(0.0, noise_sigma, size=canvas.shape)
    return _to_u8_round_half_up(np.clip(canvas, 0.0, 255.0))


def image_sha256(img):
    a = np.ascontiguousarray(img, dtype=np.uint8)
    h = hashlib.sha256()
    h.update(np.asarray(a.shape, dtype=np.int64).tobytes())
    h.update(a.tobytes())
    return h.hexdigest()
