"""Python binding of the C ABI in include/fic.h (ctypes).

Argument marshalling only: torch supplies device memory and the current
stream; every step of the encoder runs in the HIP library libfic.so built in
this directory. There is no fallback: if the library is missing, or there is
no device, the calls raise.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfic.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_CAPACITY, ERR_DEVICE = range(6)
KERNEL_MFMA, KERNEL_PLAIN = 0, 1
STAGES = ("classify", "pool", "range_prep", "domain_prep", "worklist", "search", "final", "decode",
          "batch")
CODE_DTYPE = np.dtype([("domain", "<u4"), ("iso", "u1"), ("s_idx", "i1"), ("o_idx", "u1"),
                       ("flags", "u1"), ("err", "<i8")])
assert CODE_DTYPE.itemsize == 16


class FicError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__("%s: %s (status %d)" % (what, status_string(status), status))


class Geom(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32), ("pitch", ctypes.c_int32),
                ("range_size", ctypes.c_int32), ("domain_step", ctypes.c_int32)]


class ImageDesc(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("geom", Geom), ("tol", ctypes.c_double),
                ("codes", ctypes.c_void_p)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("range_size", ctypes.c_int32), ("dlog2", ctypes.c_int32),
                ("bucket", ctypes.c_int32), ("images", ctypes.c_int32),
                ("chunk_log2", ctypes.c_int32), ("flush_at", ctypes.c_int32),
                ("xcd", ctypes.c_int32), ("base_chunk_log2", ctypes.c_int32),
                ("base_flush_at", ctypes.c_int32), ("base_xcd", ctypes.c_int32),
                ("base_ms", ctypes.c_float), ("tuned_ms", ctypes.c_float)]


DEBUG_REVERSE_ITEMS, DEBUG_VERIFY16, DEBUG_SEPARATE_SEARCHES = 1, 2, 4


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_st = ctypes.c_int


def lib():
    """Load libfic.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libfic.so is not built; run __graft_entry__.build() "
                           "or python paper_1206_4880_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "fic_create": (_st, [_i32, ctypes.POINTER(_vp)]),
        "fic_destroy": (_st, [_vp]),
        "fic_status_string": (ctypes.c_char_p, [_st]),
        "fic_set_counters": (_st, [_vp, _vp]),
        "fic_timing_enable": (_st, [_vp, _i32]),
        "fic_timing_read": (_st, [_vp, _vp, _vp, _i32, ctypes.POINTER(_i32)]),
        "fic_num_ranges": (ctypes.c_int64, [ctypes.POINTER(Geom)]),
        "fic_num_domains": (ctypes.c_int64, [ctypes.POINTER(Geom)]),
        "fic_fd_classify": (_st, [_vp, _vp, ctypes.POINTER(Geom), _i32, _i32, _vp, _vp, _vp]),
        "fic_pool_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int64]),
        "fic_build_domain_pool": (_st, [_vp, _vp, _i32, _vp, _i32, ctypes.c_double, _vp, _vp, _vp,
                                        _vp, ctypes.c_size_t, _vp]),
        "fic_encode_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Geom), _i32]),
        "fic_encode_pifs": (_st, [_vp, _vp, ctypes.POINTER(Geom), _vp, _vp, _vp, _i32, _vp, _vp,
                                  ctypes.c_size_t, _vp]),
        "fic_batch_workspace_bytes": (ctypes.c_size_t, [_i32, ctypes.POINTER(ImageDesc)]),
        "fic_encode_pifs_batch": (_st, [_vp, _i32, ctypes.POINTER(ImageDesc), _vp,
                                        ctypes.c_size_t, _vp]),
        "fic_set_batch_graph": (_st, [_vp, _i32]),
        "fic_quadtree_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Geom), ctypes.c_double,
                                                           ctypes.POINTER(Geom), ctypes.c_double]),
        "fic_encode_quadtree": (_st, [_vp, _vp, ctypes.POINTER(Geom), ctypes.c_double,
                                      ctypes.POINTER(Geom), ctypes.c_double, ctypes.c_double,
                                      _vp, _vp, _vp, ctypes.c_size_t, _vp]),
        "fic_decode_quadtree": (_st, [_vp, _vp, ctypes.POINTER(Geom), _vp, ctypes.POINTER(Geom),
                                      _i32, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp]),
        "fic_color_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Geom), ctypes.c_double]),
        "fic_encode_color": (_st, [_vp, _vp, ctypes.POINTER(Geom), ctypes.c_double, _i32, _vp, _vp,
                                   _vp, _vp, ctypes.c_size_t, _vp]),
        "fic_packed_words": (ctypes.c_int64, [ctypes.POINTER(Geom)]),
        "fic_pack_codes": (_st, [_vp, _vp, ctypes.POINTER(Geom), _vp, ctypes.c_int64, _vp]),
        "fic_unpack_codes": (_st, [_vp, _vp, ctypes.c_int64, ctypes.POINTER(Geom), _vp, _vp]),
        "fic_decode_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Geom)]),
        "fic_decode_pifs": (_st, [_vp, _vp, ctypes.POINTER(Geom), _i32, _vp, _vp, _vp,
                                  ctypes.c_size_t, _vp, _vp]),
        "fic_set_debug": (_st, [_vp, ctypes.c_uint32]),
        "fic_autotune_workspace_bytes": (ctypes.c_size_t, [_i32, ctypes.POINTER(ImageDesc)]),
        "fic_autotune": (_st, [_vp, _i32, ctypes.POINTER(ImageDesc), _vp, ctypes.c_size_t, _i32,
                               ctypes.POINTER(TuneEntry), _i32, ctypes.POINTER(_i32), _vp]),
        "fic_tune_save": (_st, [_vp, ctypes.c_char_p]),
        "fic_tune_load": (_st, [_vp, ctypes.c_char_p]),
        "fic_tune_reset": (_st, [_vp]),
        "fic_tune_query": (_st, [_vp, ctypes.POINTER(Geom), _i32, ctypes.c_double,
                                 ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
        "fic_kernel_hash": (ctypes.c_char_p, []),
        "fic_noalloc_scratch_bytes": (ctypes.c_size_t, []),
        "fic_encode_pifs_noalloc": (_st, [_vp, _vp, ctypes.POINTER(Geom), _vp, _vp, _vp, _i32, _vp,
                                          _vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


EXPORTED = ("fic_create", "fic_destroy", "fic_status_string", "fic_set_counters",
            "fic_timing_enable", "fic_timing_read",
            "fic_num_ranges", "fic_num_domains", "fic_fd_classify", "fic_pool_workspace_bytes",
            "fic_build_domain_pool", "fic_encode_workspace_bytes", "fic_encode_pifs",
            "fic_batch_workspace_bytes", "fic_encode_pifs_batch", "fic_set_batch_graph",
            "fic_decode_workspace_bytes", "fic_decode_pifs", "fic_quadtree_workspace_bytes",
            "fic_encode_quadtree", "fic_decode_quadtree", "fic_packed_words", "fic_pack_codes",
            "fic_unpack_codes", "fic_color_workspace_bytes", "fic_encode_color",
            "fic_set_debug", "fic_autotune_workspace_bytes", "fic_autotune", "fic_tune_save",
            "fic_tune_load", "fic_tune_reset", "fic_tune_query", "fic_kernel_hash",
            "fic_noalloc_scratch_bytes", "fic_encode_pifs_noalloc")


def status_string(status):
    try:
        return lib().fic_status_string(status).decode()
    except Exception:  # noqa: BLE001 - message only
        return "status"


def _check(status, what):
    if status != OK:
        raise FicError(status, what)


def make_geom(height, width, range_size, domain_step, pitch=None):
    return Geom(int(height), int(width), int(pitch if pitch is not None else width),
                int(range_size), int(domain_step))


class Context:
    """A library context bound to one HIP device (device=-1: host-only,
    validation only)."""

    def __init__(self, device=0):
        h = _vp()
        _check(lib().fic_create(int(device), ctypes.byref(h)), "fic_create")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib().fic_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def timing(self, enable=True):
        _check(lib().fic_timing_enable(self.handle, 1 if enable else 0), "fic_timing_enable")

    def timing_read(self):
        """[(stage, ms)] of the stages recorded since timing(True) (waits)."""
        cnt = _i32(0)
        _check(lib().fic_timing_read(self.handle, None, None, 0, ctypes.byref(cnt)),
               "fic_timing_read")
        n = cnt.value
        st = (ctypes.c_int32 * max(n, 1))()
        ms = (ctypes.c_float * max(n, 1))()
        _check(lib().fic_timing_read(self.handle, st, ms, n, ctypes.byref(cnt)), "fic_timing_read")
        return [(STAGES[st[i]], float(ms[i])) for i in range(min(n, cnt.value))]

    def set_counters(self, counters):
        ptr = counters.data_ptr() if counters is not None else None
        _check(lib().fic_set_counters(self.handle, ptr), "fic_set_counters")

    def set_batch_graph(self, enable):
        _check(lib().fic_set_batch_graph(self.handle, 1 if enable else 0), "fic_set_batch_graph")

    def set_debug(self, flags):
        _check(lib().fic_set_debug(self.handle, int(flags)), "fic_set_debug")

    def tune_save(self, path):
        _check(lib().fic_tune_save(self.handle, os.fsencode(path)), "fic_tune_save")

    def tune_load(self, path):
        """Load a tuning cache; returns the status (OK, ERR_UNSUPPORTED for a
        cache of another device or other kernels, ERR_INVALID_ARG)."""
        return int(lib().fic_tune_load(self.handle, os.fsencode(path)))

    def tune_reset(self):
        _check(lib().fic_tune_reset(self.handle), "fic_tune_reset")

    def tune_query(self, height, width, range_size, domain_step, pooled=False, pool_fraction=1.0,
                   with_xcd=False):
        """(chunk_log2, flush_at) an encode of this geometry would use, and
        the XCD-queue flag with with_xcd=True."""
        g = make_geom(height, width, range_size, domain_step)
        cl, fl, xc = _i32(0), _i32(0), _i32(0)
        _check(lib().fic_tune_query(self.handle, ctypes.byref(g), 1 if pooled else 0,
                                    float(pool_fraction), ctypes.byref(cl), ctypes.byref(fl),
                                    ctypes.byref(xc)), "fic_tune_query")
        if with_xcd:
            return int(cl.value), int(fl.value), int(xc.value)
        return int(cl.value), int(fl.value)


_contexts = {}


def context(device=None):
    import torch
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _contexts:
        _contexts[dev] = Context(dev)
    return _contexts[dev]


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need_cuda_u8(img):
    import torch
    if not (isinstance(img, torch.Tensor) and img.is_cuda and img.dtype == torch.uint8
            and img.dim() == 2 and img.stride(1) == 1):
        raise ValueError("image must be a 2-D uint8 CUDA tensor with unit column stride")


def _geom_of(img, range_size, domain_step):
    return make_geom(img.shape[0], img.shape[1], range_size, domain_step, pitch=img.stride(0))


def num_ranges(h, w, b):
    return int(lib().fic_num_ranges(ctypes.byref(make_geom(h, w, b, 1))))


def num_domains(h, w, b, t):
    return int(lib().fic_num_domains(ctypes.byref(make_geom(h, w, b, t))))


def fd_classify(img, block, step, want_fp32=True):
    """(fd64, fd32) of every block x block window at `step` (raster order)."""
    import torch
    _need_cuda_u8(img)
    h, w = img.shape
    count = ((h - block) // step + 1) * ((w - block) // step + 1)
    fd64 = torch.empty(count, dtype=torch.float64, device=img.device)
    fd32 = torch.empty(count, dtype=torch.float32, device=img.device) if want_fp32 else None
    g = make_geom(h, w, 4, 1, pitch=img.stride(0))
    _check(lib().fic_fd_classify(context(img.device.index).handle, img.data_ptr(), ctypes.byref(g),
                                 int(block), int(step), fd64.data_ptr(),
                                 fd32.data_ptr() if fd32 is not None else None, _stream()),
           "fic_fd_classify")
    return fd64, fd32


def build_domain_pool(fd_range, fd_domain, tol):
    """(perm, lo, hi) device tensors: the pool of range r is perm[lo[r]:hi[r]]."""
    import torch
    nr, nd = fd_range.numel(), fd_domain.numel()
    dev = fd_range.device
    perm = torch.empty(nd, dtype=torch.int32, device=dev)
    lo = torch.empty(nr, dtype=torch.int32, device=dev)
    hi = torch.empty(nr, dtype=torch.int32, device=dev)
    wsb = lib().fic_pool_workspace_bytes(nr, nd)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    _check(lib().fic_build_domain_pool(context(dev.index).handle, fd_range.data_ptr(), nr,
                                       fd_domain.data_ptr(), nd, float(tol), perm.data_ptr(),
                                       lo.data_ptr(), hi.data_ptr(), ws.data_ptr(), wsb, _stream()),
           "fic_build_domain_pool")
    return perm, lo, hi


class Workspace:
    """Reusable device scratch (grown on demand)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes, device):
        import torch
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
        return self.buf


_ws = Workspace()


def encode_pifs(img, range_size, domain_step, pool=None, kernel="mfma", codes=None, ws=None):
    """Codes (uint8 CUDA tensor [R, 16], fic_code layout) of one image.

    pool=None is exhaustive search; otherwise the (perm, lo, hi) triple of
    build_domain_pool."""
    import torch
    _need_cuda_u8(img)
    g = _geom_of(img, range_size, domain_step)
    nr = int(lib().fic_num_ranges(ctypes.byref(g)))
    if nr <= 0:
        raise FicError(ERR_INVALID_ARG, "geometry")
    pooled = pool is not None
    wsb = lib().fic_encode_workspace_bytes(ctypes.byref(g), int(pooled))
    buf = (ws or _ws).get(wsb, img.device)
    if codes is None:
        codes = torch.empty((nr, 16), dtype=torch.uint8, device=img.device)
    kern = KERNEL_MFMA if kernel == "mfma" else KERNEL_PLAIN if kernel == "plain" else int(kernel)
    perm, lo, hi = pool if pooled else (None, None, None)
    _check(lib().fic_encode_pifs(context(img.device.index).handle, img.data_ptr(), ctypes.byref(g),
                                 perm.data_ptr() if pooled else None,
                                 lo.data_ptr() if pooled else None,
                                 hi.data_ptr() if pooled else None,
                                 kern, codes.data_ptr(), buf.data_ptr(), wsb, _stream()),
           "fic_encode_pifs")
    return codes


def encode_pifs_noalloc(img, range_size, domain_step, pool=None, kernel="mfma", codes=None):
    """encode_pifs on the library's static device scratch (no workspace
    argument, nothing allocated by the library)."""
    import torch
    _need_cuda_u8(img)
    g = _geom_of(img, range_size, domain_step)
    nr = int(lib().fic_num_ranges(ctypes.byref(g)))
    if nr <= 0:
        raise FicError(ERR_INVALID_ARG, "geometry")
    if codes is None:
        codes = torch.empty((nr, 16), dtype=torch.uint8, device=img.device)
    kern = KERNEL_MFMA if kernel == "mfma" else KERNEL_PLAIN if kernel == "plain" else int(kernel)
    pooled = pool is not None
    perm, lo, hi = pool if pooled else (None, None, None)
    _check(lib().fic_encode_pifs_noalloc(context(img.device.index).handle, img.data_ptr(),
                                         ctypes.byref(g), perm.data_ptr() if pooled else None,
                                         lo.data_ptr() if pooled else None,
                                         hi.data_ptr() if pooled else None, kern,
                                         codes.data_ptr(), _stream()),
           "fic_encode_pifs_noalloc")
    return codes


def encode(img, range_size, domain_step, tol=None, kernel="mfma"):
    """Classify + pool (when tol is not None) + search. Returns the codes
    tensor and the pool triple (or None)."""
    pool = None
    if tol is not None and not (isinstance(tol, float) and math.isinf(tol) and tol > 0):
        fr, _ = fd_classify(img, range_size, range_size, want_fp32=False)
        fd, _ = fd_classify(img, 2 * range_size, domain_step, want_fp32=False)
        pool = build_domain_pool(fr, fd, tol)
    return encode_pifs(img, range_size, domain_step, pool=pool, kernel=kernel), pool


def batch_workspace_bytes(images, jobs):
    """fic_batch_workspace_bytes for these images and jobs [(B, t, tol)]."""
    n = len(images)
    descs = (ImageDesc * n)()
    for i, (img, (b, t, tol)) in enumerate(zip(images, jobs)):
        _need_cuda_u8(img)
        descs[i].geom = _geom_of(img, b, t)
        descs[i].tol = float("inf") if tol is None else float(tol)
    return int(lib().fic_batch_workspace_bytes(n, descs))


def encode_batch(images, jobs, codes=None, ws=None, graph=True):
    """Batch encode: images (list of uint8 CUDA tensors), jobs [(B, t, tol)].
    Returns the list of codes tensors. `codes` and `ws` (uint8 CUDA tensors)
    may be given to keep the buffers, and so a recorded graph, across calls;
    graph=False enqueues the kernels directly."""
    import torch
    n = len(images)
    descs = (ImageDesc * n)()
    outs = []
    for i, (img, (b, t, tol)) in enumerate(zip(images, jobs)):
        _need_cuda_u8(img)
        g = _geom_of(img, b, t)
        nr = int(lib().fic_num_ranges(ctypes.byref(g)))
        c = codes[i] if codes is not None else torch.empty((nr, 16), dtype=torch.uint8,
                                                            device=img.device)
        outs.append(c)
        descs[i].img = img.data_ptr()
        descs[i].geom = g
        descs[i].tol = float("inf") if tol is None else float(tol)
        descs[i].codes = c.data_ptr()
    wsb = lib().fic_batch_workspace_bytes(n, descs)
    if ws is not None:
        if ws.numel() < wsb:
            raise ValueError("batch workspace needs %d bytes" % wsb)
        buf = ws
    else:
        buf = _ws.get(wsb, images[0].device)
    ctx = context(images[0].device.index)
    ctx.set_batch_graph(graph)
    _check(lib().fic_encode_pifs_batch(ctx.handle, n, descs, buf.data_ptr(), wsb, _stream()),
           "fic_encode_pifs_batch")
    return outs


def _descs(images, jobs, codes):
    n = len(images)
    descs = (ImageDesc * n)()
    for i, (img, (b, t, tol)) in enumerate(zip(images, jobs)):
        _need_cuda_u8(img)
        descs[i].img = img.data_ptr()
        descs[i].geom = _geom_of(img, b, t)
        descs[i].tol = float("inf") if tol is None else float(tol)
        descs[i].codes = codes[i].data_ptr()
    return descs


def autotune(images, jobs, reps=2):
    """Time candidate search parameters on these images (see fic_autotune)
    and keep the winners in the device's context. Returns a list of dicts,
    one per tuning class. Blocks the host."""
    import torch
    n = len(images)
    codes = [torch.empty((num_ranges(im.shape[0], im.shape[1], b), 16), dtype=torch.uint8,
                         device=im.device) for im, (b, _, _) in zip(images, jobs)]
    descs = _descs(images, jobs, codes)
    wsb = lib().fic_autotune_workspace_bytes(n, descs)
    if wsb == 0:
        raise FicError(ERR_INVALID_ARG, "fic_autotune_workspace_bytes")
    # room for the whole batch too, so the tuner also picks its launch structure
    wsb = max(wsb, int(lib().fic_batch_workspace_bytes(n, descs)))
    buf = _ws.get(wsb, images[0].device)
    rep_ = (TuneEntry * (n + 1))()
    cnt = _i32(0)
    ctx = context(images[0].device.index)
    _check(lib().fic_autotune(ctx.handle, n, descs, buf.data_ptr(), wsb, int(reps), rep_, n + 1,
                              ctypes.byref(cnt), _stream()), "fic_autotune")
    return [{f: getattr(rep_[i], f) for f, _ in TuneEntry._fields_} for i in range(cnt.value)]


def kernel_hash():
    return lib().fic_kernel_hash().decode()


def batch_workspace_bytes(images, jobs):
    """Workspace bytes of encode_batch for these images and jobs."""
    n = len(images)
    descs = (ImageDesc * n)()
    for i, (img, (b, t, tol)) in enumerate(zip(images, jobs)):
        descs[i].geom = _geom_of(img, b, t)
        descs[i].tol = float("inf") if tol is None else float(tol)
    return int(lib().fic_batch_workspace_bytes(n, descs))


def decode_pifs(codes, height, width, range_size, domain_step, max_iters=32, init=None, scale=1):
    """(image tensor, iterations tensor) decoded from codes on the device.
    scale=2 decodes the same codes at twice the encoded height and width."""
    import torch
    if scale not in (1, 2):
        raise ValueError("scale is 1 or 2")
    height, width = height * scale, width * scale
    g = make_geom(height, width, range_size * scale, domain_step * scale)
    dev = codes.device
    out = torch.empty((height, width), dtype=torch.uint8, device=dev)
    iters = torch.zeros(1, dtype=torch.int32, device=dev)
    wsb = lib().fic_decode_workspace_bytes(ctypes.byref(g))
    scratch = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    if init is not None:
        _need_cuda_u8(init)
    _check(lib().fic_decode_pifs(context(dev.index).handle, codes.data_ptr(), ctypes.byref(g),
                                 int(max_iters), init.data_ptr() if init is not None else None,
                                 out.data_ptr(), scratch.data_ptr(), wsb, iters.data_ptr(),
                                 _stream()), "fic_decode_pifs")
    return out, iters


def encode_quadtree(img, b1, t1, tol1, b2, t2, tol2, rms, codes=None, ws=None):
    """Two-level encode (see fic_encode_quadtree): returns (codes1, codes2)
    as uint8 (R, 16) tensors. tol None = exhaustive at that level."""
    import torch
    _need_cuda_u8(img)
    g1, g2 = _geom_of(img, b1, t1), _geom_of(img, b2, t2)
    tl1 = float("inf") if tol1 is None else float(tol1)
    tl2 = float("inf") if tol2 is None else float(tol2)
    r1 = int(lib().fic_num_ranges(ctypes.byref(g1)))
    r2 = int(lib().fic_num_ranges(ctypes.byref(g2)))
    if codes is None:
        codes = (torch.empty((r1, 16), dtype=torch.uint8, device=img.device),
                 torch.empty((r2, 16), dtype=torch.uint8, device=img.device))
    wsb = lib().fic_quadtree_workspace_bytes(ctypes.byref(g1), tl1, ctypes.byref(g2), tl2)
    if wsb == 0:
        raise ValueError("invalid two-level geometry")
    buf = ws if ws is not None else _ws.get(wsb, img.device)
    _check(lib().fic_encode_quadtree(context(img.device.index).handle, img.data_ptr(),
                                     ctypes.byref(g1), tl1, ctypes.byref(g2), tl2, float(rms),
                                     codes[0].data_ptr(), codes[1].data_ptr(), buf.data_ptr(),
                                     wsb, _stream()), "fic_encode_quadtree")
    return codes


def decode_quadtree(codes1, codes2, height, width, b1, t1, b2, t2, max_iters=32, init=None):
    """(image tensor, iterations tensor) decoded from a two-level code set."""
    import torch
    g1 = make_geom(height, width, b1, t1)
    g2 = make_geom(height, width, b2, t2)
    dev = codes1.device
    out = torch.empty((height, width), dtype=torch.uint8, device=dev)
    iters = torch.zeros(1, dtype=torch.int32, device=dev)
    wsb = lib().fic_decode_workspace_bytes(ctypes.byref(g1))
    scratch = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    if init is not None:
        _need_cuda_u8(init)
    _check(lib().fic_decode_quadtree(context(dev.index).handle, codes1.data_ptr(), ctypes.byref(g1),
                                     codes2.data_ptr(), ctypes.byref(g2), int(max_iters),
                                     init.data_ptr() if init is not None else None,
                                     out.data_ptr(), scratch.data_ptr(), wsb, iters.data_ptr(),
                                     _stream()), "fic_decode_quadtree")
    return out, iters


def encode_color(rgb, range_size, domain_step, tol=None, fd_source="luma"):
    """Per-channel encode of an (H, W, 3) uint8 CUDA tensor with pools from
    the luma or mean image; returns three codes tensors (R, G, B)."""
    import torch
    if rgb.dtype != torch.uint8 or rgb.device.type != "cuda" or rgb.dim() != 3 or rgb.shape[2] != 3:
        raise ValueError("rgb must be an (H, W, 3) uint8 CUDA tensor")
    rgb = rgb.contiguous()
    H, W = int(rgb.shape[0]), int(rgb.shape[1])
    g = make_geom(H, W, range_size, domain_step, pitch=3 * W)
    src = {"luma": 0, "mean": 1}[fd_source]
    tl = float("inf") if tol is None else float(tol)
    nr = int(lib().fic_num_ranges(ctypes.byref(make_geom(H, W, range_size, domain_step))))
    codes = [torch.empty((nr, 16), dtype=torch.uint8, device=rgb.device) for _ in range(3)]
    wsb = lib().fic_color_workspace_bytes(ctypes.byref(g), tl)
    if wsb == 0:
        raise ValueError("invalid colour geometry")
    buf = _ws.get(wsb, rgb.device)
    _check(lib().fic_encode_color(context(rgb.device.index).handle, rgb.data_ptr(), ctypes.byref(g),
                                  tl, src, codes[0].data_ptr(), codes[1].data_ptr(),
                                  codes[2].data_ptr(), buf.data_ptr(), wsb, _stream()),
           "fic_encode_color")
    return codes


def pack_codes(codes, height, width, range_size, domain_step):
    """The packed bit string (uint32 CUDA tensor) of a codes tensor."""
    import torch
    g = make_geom(height, width, range_size, domain_step)
    nw = int(lib().fic_packed_words(ctypes.byref(g)))
    words = torch.empty(max(nw, 1), dtype=torch.int32, device=codes.device)
    _check(lib().fic_pack_codes(context(codes.device.index).handle, codes.data_ptr(),
                                ctypes.byref(g), words.data_ptr(), nw, _stream()),
           "fic_pack_codes")
    return words[:nw]


def unpack_bitstream(words, height, width, range_size, domain_step):
    """Codes tensor (flags and errors 0) from a packed bit string."""
    import torch
    g = make_geom(height, width, range_size, domain_step)
    nr = int(lib().fic_num_ranges(ctypes.byref(g)))
    codes = torch.empty((nr, 16), dtype=torch.uint8, device=words.device)
    _check(lib().fic_unpack_codes(context(words.device.index).handle, words.data_ptr(),
                                  words.numel(), ctypes.byref(g), codes.data_ptr(), _stream()),
           "fic_unpack_codes")
    return codes


def unpack_codes(codes):
    """numpy structured view of a codes tensor (copies to host)."""
    a = codes.detach().cpu().numpy().reshape(-1)
    return a.view(CODE_DTYPE)
