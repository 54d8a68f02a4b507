"""CPU oracle for the PIFS range-domain search.

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this; the product path never does.
It shares no code with the GPU library (``paper_1206_4880_amd``) and neither
imports the other.

The arithmetic lives in ``fic_oracle.c`` (plain loops, exact integers, fp64
fractal dimensions); this module only compiles it with gcc and marshals numpy
arrays. ``bruteforce.py`` holds the pixel-level grid search used to pin it.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fic_oracle.c")
_SO = os.path.join(_HERE, "libfic_oracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def build(force=True):
    """Compile the oracle with gcc (-O2, OpenMP). Returns the .so path."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        L.fico_num_ranges.restype = ctypes.c_int64
        L.fico_num_ranges.argtypes = [ctypes.c_int32] * 3
        L.fico_num_domains.restype = ctypes.c_int64
        L.fico_num_domains.argtypes = [ctypes.c_int32] * 4
        L.fico_iso_apply.restype = None
        L.fico_iso_apply.argtypes = [ctypes.c_int32, ctypes.c_int32, _i64p, _i64p]
        L.fico_dbc_fd.restype = ctypes.c_double
        L.fico_dbc_fd.argtypes = [_u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, _i64p]
        L.fico_fd_blocks.restype = None
        L.fico_fd_blocks.argtypes = [_u8p] + [ctypes.c_int32] * 5 + [_f64p, ctypes.c_int32]
        L.fico_resolve_tol.restype = ctypes.c_double
        L.fico_resolve_tol.argtypes = [ctypes.c_double, _f64p, ctypes.c_int64]
        L.fico_encode.restype = ctypes.c_int32
        L.fico_encode.argtypes = ([_u8p] + [ctypes.c_int32] * 5
                                  + [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                     ctypes.c_void_p, ctypes.c_int64]
                                  + [_i32p] * 5 + [_i64p, _i64p, _i64p, ctypes.c_int32])
        L.fico_pair_f.restype = ctypes.c_int64
        L.fico_pair_f.argtypes = ([_u8p] + [ctypes.c_int32] * 5
                                  + [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int32)])
        L.fico_decode.restype = ctypes.c_int32
        L.fico_decode.argtypes = ([_i32p] * 4 + [ctypes.c_int32] * 5
                                  + [ctypes.c_void_p, _u8p, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.c_int32])
        L.fico_decode_quadtree.restype = ctypes.c_int32
        L.fico_decode_quadtree.argtypes = ([_i32p] * 4 + [_u8p, ctypes.c_int32, ctypes.c_int32]
                                           + [_i32p] * 4 + [_u8p, ctypes.c_int32, ctypes.c_int32]
                                           + [ctypes.c_int32] * 3
                                           + [ctypes.c_void_p, _u8p,
                                              ctypes.POINTER(ctypes.c_int32), ctypes.c_int32])
        _lib = L
    return _lib


def _img(img):
    return np.ascontiguousarray(img, dtype=np.uint8)


def num_ranges(h, w, b):
    return int(lib().fico_num_ranges(h, w, b))


def num_domains(h, w, b, t):
    return int(lib().fico_num_domains(h, w, b, t))


def iso_apply(q, block):
    blk = np.ascontiguousarray(block, dtype=np.int64)
    b = blk.shape[0]
    out = np.empty_like(blk)
    lib().fico_iso_apply(int(q), int(b), blk, out)
    return out


def dbc_fd(block, return_counts=False):
    """Fractal dimension of one square uint8 block (side a power of two)."""
    blk = _img(block)
    m = blk.shape[0]
    counts = np.zeros(8, dtype=np.int64)
    fd = lib().fico_dbc_fd(blk, m, 0, 0, m, counts)
    if return_counts:
        return fd, counts[: int(np.log2(m))]
    return fd


def fd_blocks(img, m, step, nthreads=0):
    im = _img(img)
    h, w = im.shape
    rows, cols = (h - m) // step + 1, (w - m) // step + 1
    out = np.empty(rows * cols, dtype=np.float64)
    lib().fico_fd_blocks(im, h, w, w, m, step, out, int(nthreads))
    return out


def resolve_tol(tol, fd_dom):
    fd = np.ascontiguousarray(fd_dom, dtype=np.float64)
    return float(lib().fico_resolve_tol(float(tol), fd, fd.size))


def classify(img, b, t, nthreads=0):
    """(fd of ranges, fd of domains) in fp64."""
    return fd_blocks(img, b, b, nthreads), fd_blocks(img, 2 * b, t, nthreads)


def encode(img, b, t, tol=None, sel=None, nthreads=0, fds=None):
    """Exact codes for the selected ranges (all when sel is None).

    tol=None is exhaustive search; otherwise the fractal-dimension window with
    half-width tol (negative: the adaptive (max - min)/3).
    Returns a dict of numpy arrays: dom, iso, k, j, flags, err, f, pool, plus
    the resolved tolerance under 'tol'.
    """
    im = _img(img)
    h, w = im.shape
    if sel is None:
        n = num_ranges(h, w, b)
        selp = None
    else:
        sel = np.ascontiguousarray(sel, dtype=np.int64)
        n = sel.size
        selp = sel.ctypes.data
    out = {k: np.zeros(n, dtype=np.int32) for k in ("dom", "iso", "k", "j", "flags")}
    for k in ("err", "f", "pool"):
        out[k] = np.zeros(n, dtype=np.int64)
    fr = fdd = None
    rt = float("inf")
    if tol is not None:
        fr, fdd = fds if fds is not None else classify(im, b, t, nthreads)
        fr = np.ascontiguousarray(fr, dtype=np.float64)
        fdd = np.ascontiguousarray(fdd, dtype=np.float64)
        rt = resolve_tol(tol, fdd)
    rc = lib().fico_encode(im, h, w, w, b, t,
                           fr.ctypes.data if fr is not None else None,
                           fdd.ctypes.data if fdd is not None else None,
                           rt, selp, n,
                           out["dom"], out["iso"], out["k"], out["j"], out["flags"],
                           out["err"], out["f"], out["pool"], int(nthreads))
    if rc != 0:
        raise ValueError("oracle: invalid geometry")
    out["tol"] = rt
    return out


def pair_f(img, b, t, r, d, q):
    im = _img(img)
    h, w = im.shape
    k = ctypes.c_int32(0)
    f = lib().fico_pair_f(im, h, w, w, b, t, int(r), int(d), int(q), ctypes.byref(k))
    return int(f), int(k.value)


def decode(codes, h, w, b, t, max_iters=32, init=None, nthreads=0):
    """Decoded image and the number of sweeps run."""
    arr = [np.ascontiguousarray(codes[k], dtype=np.int32) for k in ("dom", "iso", "k", "j")]
    out = np.empty((h, w), dtype=np.uint8)
    it = ctypes.c_int32(0)
    ini = _img(init) if init is not None else None
    rc = lib().fico_decode(*arr, h, w, b, t, int(max_iters),
                           ini.ctypes.data if ini is not None else None,
                           out, ctypes.byref(it), int(nthreads))
    if rc != 0:
        raise ValueError("oracle: invalid geometry")
    return out, int(it.value)


def split_threshold(b1, rms):
    """Largest level-1 error E = 4096*n*SSE that is not split: E is split
    when its mean squared error SSE/n exceeds rms^2, i.e. E > 4096*n^2*rms^2,
    floored to an integer (E is one). fp64, in this operation order."""
    n1 = b1 * b1
    t = rms * rms * (4096.0 * n1 * n1)
    if not t < 9.0e18:
        return (1 << 63) - 1
    return int(math.floor(t))


def encode_quadtree(img, b1, t1, tol1, b2, t2, tol2, rms, nthreads=0):
    """Two-level partition (Fisher's quadtree, the paper's ref. [12], at two
    levels): every b1 x b1 range is coded; a range whose E exceeds
    split_threshold(b1, rms) is split, flagged (bit 1), and its four
    b2 x b2 sub-ranges are coded at level 2 (their own pool or exhaustive
    search over the level-2 domains); the other level-2 codes are "not
    coded": domain 0, isometry 0, k = 0, j = 0, flags bit 2, E = 0.
    Returns (level-1 codes, level-2 codes) as dicts like encode()."""
    if b1 != 2 * b2:
        raise ValueError("level-2 ranges are the quadrants of level-1 ranges")
    im = _img(img)
    h, w = im.shape
    c1 = encode(im, b1, t1, tol=tol1, nthreads=nthreads)
    split = c1["err"] > split_threshold(b1, rms)
    c1["flags"] = c1["flags"] | np.where(split, 2, 0).astype(np.int32)
    rc1, rc2 = w // b1, w // b2
    kids = []
    for r in np.flatnonzero(split):
        ry, rx = divmod(int(r), rc1)
        for a in (0, 1):
            for c in (0, 1):
                kids.append((2 * ry + a) * rc2 + 2 * rx + c)
    kids = np.array(sorted(kids), dtype=np.int64)
    n2 = num_ranges(h, w, b2)
    c2 = {k: np.zeros(n2, dtype=np.int32) for k in ("dom", "iso", "k", "j", "flags")}
    for k in ("err", "f", "pool"):
        c2[k] = np.zeros(n2, dtype=np.int64)
    c2["flags"][:] = 4
    if kids.size:
        sub = encode(im, b2, t2, tol=tol2, sel=kids, nthreads=nthreads)
        for k in ("dom", "iso", "k", "j", "flags", "err", "f", "pool"):
            c2[k][kids] = sub[k]
    return c1, c2


def decode_quadtree(c1, c2, h, w, b1, t1, b2, t2, max_iters=32, init=None, nthreads=0):
    """Decoded image of a two-level code set and the number of sweeps run."""
    a1 = [np.ascontiguousarray(c1[k], dtype=np.int32) for k in ("dom", "iso", "k", "j")]
    a2 = [np.ascontiguousarray(c2[k], dtype=np.int32) for k in ("dom", "iso", "k", "j")]
    split1 = np.ascontiguousarray((np.asarray(c1["flags"]) & 2) != 0, dtype=np.uint8)
    coded2 = np.ascontiguousarray((np.asarray(c2["flags"]) & 4) == 0, dtype=np.uint8)
    out = np.empty((h, w), dtype=np.uint8)
    it = ctypes.c_int32(0)
    ini = _img(init) if init is not None else None
    rc = lib().fico_decode_quadtree(*a1, split1, b1, t1, *a2, coded2, b2, t2, h, w,
                                    int(max_iters), ini.ctypes.data if ini is not None else None,
                                    out, ctypes.byref(it), int(nthreads))
    if rc != 0:
        raise ValueError("oracle: invalid geometry")
    return out, int(it.value)


def decode_scaled(codes, h, w, b, t, scale, max_iters=32, init=None, nthreads=0):
    """Decode at scale times the encoded size (resolution independence): the
    same maps on the lattice scaled by `scale` (ranges scale*b, domain step
    scale*t, the same domain indices), i.e. decode() with that geometry."""
    return decode(codes, h * scale, w * scale, b * scale, t * scale, max_iters, init, nthreads)


def color_planes(rgb, fd_source):
    """The three channel planes of an interleaved h x w x 3 uint8 image and
    the image the fractal dimensions are taken from: fd_source 0 = luma
    (299 R + 587 G + 114 B + 500) div 1000, 1 = channel mean
    (R + G + B + 1) div 3 (integers, so every conversion is exact)."""
    a = np.asarray(rgb, dtype=np.int64)
    planes = [np.ascontiguousarray(a[:, :, c].astype(np.uint8)) for c in range(3)]
    if fd_source == 0:
        fdimg = (299 * a[:, :, 0] + 587 * a[:, :, 1] + 114 * a[:, :, 2] + 500) // 1000
    elif fd_source == 1:
        fdimg = (a[:, :, 0] + a[:, :, 1] + a[:, :, 2] + 1) // 3
    else:
        raise ValueError("fd_source is 0 (luma) or 1 (mean)")
    return planes, np.ascontiguousarray(fdimg.astype(np.uint8))


def encode_color(rgb, b, t, tol, fd_source=0, nthreads=0):
    """Per-channel encode (Sec. 3.1 discusses colour images): the pools come
    from the dimensions of the luma (or mean) image, and each channel is
    searched over them (tol None = exhaustive). Returns three code dicts."""
    planes, fdimg = color_planes(rgb, fd_source)
    fds = classify(fdimg, b, t, nthreads) if tol is not None else None
    return [encode(p, b, t, tol=tol, fds=fds, nthreads=nthreads) for p in planes]


def code_bits(num_domains):
    """Bits of one packed code: the domain index (ceil(log2 D) bits, at least
    1), the isometry (3), the contrast index k + 16 (5) and the brightness
    index j (7) -- the fields Sec. 1 stores per range."""
    dbits = max(1, int(num_domains - 1).bit_length())
    return dbits, dbits + 15


def pack_codes(codes, num_domains):
    """The codes of all ranges, in raster order, as one little-endian bit
    string in uint32 words: range r's fields start at bit r*W, each field
    least significant bit first, in the order domain, isometry, k + 16, j."""
    dbits, W = code_bits(num_domains)
    dom, iso = np.asarray(codes["dom"]), np.asarray(codes["iso"])
    kk, jj = np.asarray(codes["k"]), np.asarray(codes["j"])
    R = dom.size
    nwords = (R * W + 31) // 32
    words = [0] * nwords
    for r in range(R):
        fields = [(int(dom[r]), dbits), (int(iso[r]), 3), (int(kk[r]) + 16, 5), (int(jj[r]), 7)]
        pos = r * W
        for value, width in fields:
            for bit in range(width):
                if (value >> bit) & 1:
                    words[(pos + bit) // 32] |= 1 << ((pos + bit) % 32)
            pos += width
    return np.array(words, dtype=np.uint32)


def unpack_codes(words, num_ranges, num_domains):
    """Inverse of pack_codes: dom, iso, k, j per range."""
    dbits, W = code_bits(num_domains)
    words = [int(x) for x in np.asarray(words, dtype=np.uint32)]
    out = {k: np.zeros(num_ranges, dtype=np.int32) for k in ("dom", "iso", "k", "j")}
    for r in range(num_ranges):
        pos = r * W
        vals = []
        for width in (dbits, 3, 5, 7):
            v = 0
            for bit in range(width):
                if (words[(pos + bit) // 32] >> ((pos + bit) % 32)) & 1:
                    v |= 1 << bit
            vals.append(v)
            pos += width
        out["dom"][r], out["iso"][r], out["k"][r], out["j"][r] = vals[0], vals[1], vals[2] - 16, vals[3]
    return out


def compression_ratio(h, w, num_ranges, num_domains):
    """8-bit pixels against the packed codes (words rounded up)."""
    _, W = code_bits(num_domains)
    return (8.0 * h * w) / (32 * ((num_ranges * W + 31) // 32))


def psnr(a, b):
    """Peak signal-to-noise ratio for 8-bit images, fp64 (inf when equal)."""
    d = a.astype(np.float64) - b.astype(np.float64)
    mse = float(np.mean(d * d))
    return float("inf") if mse == 0.0 else 10.0 * np.log10(255.0 * 255.0 / mse)


def pool_margin(fd_range, fd_dom, tol):
    """Smallest distance between any |fd_d - fd_r| and the window edge
    tol + 1e-9: how far every membership decision is from flipping."""
    edge = tol + 1e-9
    s = np.sort(np.asarray(fd_dom, dtype=np.float64))
    best = np.inf
    for sign in (-1.0, 1.0):
        target = np.asarray(fd_range, dtype=np.float64) + sign * edge
        pos = np.searchsorted(s, target)
        for off in (-1, 0):
            p = np.clip(pos + off, 0, s.size - 1)
            diff = np.abs(np.abs(s[p] - fd_range) - edge)
            best = min(best, float(diff.min()))
    return best


def pool_bounds(fd_range, fd_dom, tol):
    """Pool sizes per range by the plain membership rule (for pair counts)."""
    fr = np.asarray(fd_range, dtype=np.float64)
    fd = np.asarray(fd_dom, dtype=np.float64)
    return np.array([int(np.count_nonzero(np.abs(fd - x) <= tol + 1e-9)) for x in fr],
                    dtype=np.int64)
