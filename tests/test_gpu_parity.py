"""GPU parity: every stage of the HIP path against the CPU oracle, through
the C ABI, on the same seeded inputs.

Bar: codes (domain, isometry, k, j, flags, E) bit-exact; fractal dimensions
within 1e-12 in fp64 and 1e-5 in fp32 of the oracle's fp64 values; pool sets
identical; decoded images bit-exact. Small cases are compared on every
range; the full-size workloads on sampled ranges (the oracle computes them
one by one) plus MFMA == plain on every range.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fic():
    import paper_1206_4880_amd as p
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    p.fic.lib()
    return p


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def dev(img):
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


def fbm(n, h, seed, w=None):
    from synth import fbm as _f
    return _f(n, w or n, h, np.random.default_rng(seed))


def assert_codes(got, ref, sel=None, what=""):
    g = got if sel is None else got[sel]
    pairs = (("domain", "dom"), ("iso", "iso"), ("s_idx", "k"), ("o_idx", "j"),
             ("flags", "flags"), ("err", "err"))
    for fg, fr in pairs:
        a = g[fg].astype(np.int64)
        b = np.asarray(ref[fr]).astype(np.int64)
        if not np.array_equal(a, b):
            bad = np.flatnonzero(a != b)[:5]
            raise AssertionError("%s: field %s differs at %s: gpu %s oracle %s"
                                 % (what, fg, bad, a[bad], b[bad]))


def gpu_encode(fic, img, b, t, tol, kernel):
    codes, pool = fic.encode(dev(img), b, t, tol=tol, kernel=kernel)
    torch.cuda.synchronize()
    return fic.unpack_codes(codes), pool


# ------------------------------------------------------------- classify
@pytest.mark.parametrize("m,step", [(4, 4), (8, 8), (16, 16), (8, 1), (8, 2), (16, 1), (16, 2),
                                    (32, 4), (32, 3)])
def test_fd_classify(fic, orc, m, step):
    imgs = [fbm(96, 0.4, 1), fbm(64, 0.8, 2, w=160),
            np.random.default_rng(3).integers(0, 256, (80, 72)).astype(np.uint8),
            np.full((64, 64), 17, np.uint8)]
    for img in imgs:
        fd64, fd32 = fic.fd_classify(dev(img), m, step)
        torch.cuda.synchronize()
        ref = orc.fd_blocks(img, m, step)
        a64, a32 = fd64.cpu().numpy(), fd32.cpu().numpy()
        assert a64.shape == ref.shape
        assert np.max(np.abs(a64 - ref)) < 1e-12
        assert np.max(np.abs(a32.astype(np.float64) - ref)) < 1e-5


def test_fd_classify_full_size(fic, orc):
    from synth import workload_images
    img = workload_images("fbm1024_b8t1")
    fd64, fd32 = fic.fd_classify(dev(img), 16, 1)
    torch.cuda.synchronize()
    ref = orc.fd_blocks(img, 16, 1)
    assert np.max(np.abs(fd64.cpu().numpy() - ref)) < 1e-12
    assert np.max(np.abs(fd32.cpu().numpy().astype(np.float64) - ref)) < 1e-5


# ------------------------------------------------------------------ pool
def check_pool(perm, lo, hi, fd_r, fd_d, tol_eff, gpu_fd_d, sel=None):
    """perm must sort the GPU's own domain values (stable); the pool sets
    must equal the oracle's window over the oracle's values."""
    perm = perm.cpu().numpy().astype(np.int64)
    lo = lo.cpu().numpy().astype(np.int64)
    hi = hi.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(perm), np.arange(fd_d.size))
    vals = gpu_fd_d[perm]
    assert np.all(np.diff(vals) >= 0)
    eq = np.diff(vals) == 0
    assert np.all(np.diff(perm)[eq] > 0)
    rows = range(fd_r.size) if sel is None else sel
    for r in rows:
        want = np.flatnonzero(np.abs(fd_d - fd_r[r]) <= tol_eff + 1e-9)
        got = np.sort(perm[lo[r]:hi[r]])
        assert np.array_equal(got, want), r


@pytest.mark.parametrize("tol", [0.0, 0.02, 0.05, 0.1, -1.0, float("inf")])
def test_pool_sets(fic, orc, tol):
    img = fbm(128, 0.5, 5)
    b, t = 4, 2
    fr_t, _ = fic.fd_classify(dev(img), b, b)
    fd_t, _ = fic.fd_classify(dev(img), 2 * b, t)
    perm, lo, hi = fic.build_domain_pool(fr_t, fd_t, tol)
    torch.cuda.synchronize()
    fr, fd = orc.classify(img, b, t)
    tol_eff = orc.resolve_tol(tol, fd)
    if math.isfinite(tol_eff):
        assert orc.pool_margin(fr, fd, tol_eff) > 1e-12
    check_pool(perm, lo, hi, fr, fd, tol_eff, fd_t.cpu().numpy())


# ---------------------------------------------------- encode, small, exact
SMALL = [
    ("fbm64 8/1 exhaustive", lambda: fbm(64, 0.5, 1), 8, 1, None),
    ("fbm 96x80 4/1", lambda: fbm(96, 0.6, 7, w=80), 4, 1, None),
    ("fbm 96x80 4/3 pool", lambda: fbm(96, 0.6, 7, w=80), 4, 3, 0.05),
    ("fbm 128 16/4", lambda: fbm(128, 0.6, 8), 16, 4, None),
    ("fbm 128 16/2 pool", lambda: fbm(128, 0.6, 8), 16, 2, 0.1),
    ("uniform 72x88 8/2", lambda: np.random.default_rng(9).integers(0, 256, (72, 88)).astype(np.uint8),
     8, 2, None),
    ("rects 128 8/1 pool", None, 8, 1, 0.05),
    ("piecewise 128 4/2 pool", None, 4, 2, 0.05),
    ("piecewise 128 8/2 adaptive", None, 8, 2, -1.0),
    ("flat 64 8/1", lambda: np.full((64, 64), 200, np.uint8), 8, 1, None),
    ("flat 64 8/1 pool", lambda: np.full((64, 64), 200, np.uint8), 8, 1, 0.05),
    ("minimal 16x16 8/1", lambda: fbm(16, 0.5, 3), 8, 1, None),
    ("tol 0: empty pools", lambda: fbm(64, 0.3, 12), 8, 2, 0.0),
    # 0/255 pixels: the largest centred operands, partial sums near 2^26 at
    # 16x16 (the one-accumulator screen rounds there), many near-ties
    ("binary 128 16/1", lambda: (np.random.default_rng(31).integers(0, 2, (128, 128)) * 255).astype(np.uint8),
     16, 1, None),
    ("binary 128 16/2 pool", lambda: (np.random.default_rng(32).integers(0, 2, (128, 128)) * 255).astype(np.uint8),
     16, 2, 0.05),
    ("binary 64 8/1", lambda: (np.random.default_rng(33).integers(0, 2, (64, 64)) * 255).astype(np.uint8),
     8, 1, None),
]


def small_image(name, make):
    from synth import add_rectangles, piecewise_smooth
    if make is not None:
        return make()
    if name.startswith("rects"):
        rng = np.random.default_rng(21)
        return add_rectangles(fbm(128, 0.7, 20), 12, rng)
    return piecewise_smooth(128, np.random.default_rng(22))


@pytest.mark.parametrize("case", SMALL, ids=[c[0] for c in SMALL])
@pytest.mark.parametrize("kernel", ["mfma", "plain"])
def test_encode_small_exact(fic, orc, case, kernel):
    name, make, b, t, tol = case
    img = small_image(name, make)
    got, _ = gpu_encode(fic, img, b, t, tol, kernel)
    ref = orc.encode(img, b, t, tol=tol)
    assert_codes(got, ref, what=name)


@pytest.mark.parametrize("b,h,w", [(4, 40, 44), (8, 64, 72), (16, 96, 80)])
def test_encode_odd_pitch_and_offset(fic, orc, b, h, w):
    """An image view whose rows start at odd addresses (odd pitch, odd start
    offset): the domain operands read the same pixels as from a packed copy,
    up to the first and last byte of the view."""
    img = fbm(h, 0.5, 40 + b, w=w)
    big = torch.zeros((h + 1, w + 5), dtype=torch.uint8, device="cuda")
    view = big[:h, 3:3 + w]                       # pitch w + 5 (odd), offset 3
    view.copy_(dev(img))
    assert view.stride(0) == w + 5 and view.data_ptr() % 4 == 3
    for tol in (None, 0.05):
        codes, _ = fic.encode(view, b, 1, tol=tol)
        torch.cuda.synchronize()
        ref = orc.encode(img, b, 1, tol=tol)
        assert_codes(fic.unpack_codes(codes), ref, what="odd pitch b=%d tol=%s" % (b, tol))


def test_encode_planted_copy(fic, orc):
    """A range planted as s=1/2 times an isometric domain copy: zero error."""
    from oracle import bruteforce as bf
    b, t = 8, 2
    img = fbm(64, 0.5, 3)
    rng = np.random.default_rng(5)
    v = 2 * rng.integers(10, 100, size=(b, b))
    v[0, 0] += (-v.sum()) % (2 * b * b)
    img[32:48, 32:48] = np.kron(v, np.ones((2, 2)))
    img[0:8, 8:16] = (bf.isometries(v)[5] - v.mean()) // 2 + 128
    for kernel in ("mfma", "plain"):
        got, _ = gpu_encode(fic, img, b, t, None, kernel)
        assert got["err"][1] == 0
        ref = orc.encode(img, b, t)
        assert_codes(got, ref, what="planted " + kernel)


# ------------------------------------------------ full-size workloads
def sampled(R, count, seed=0):
    rng = np.random.default_rng(seed)
    s = np.unique(np.concatenate([[0, R - 1], rng.choice(R, size=count, replace=False)]))
    return s.astype(np.int64)


@pytest.mark.parametrize("job", [(8, 2, None), (8, 2, 0.05)])
def test_workload_512_rects(fic, orc, job):
    from synth import workload_images
    img = workload_images("fbm512rect_b8t2")
    b, t, tol = job
    mf, _ = gpu_encode(fic, img, b, t, tol, "mfma")
    pl, _ = gpu_encode(fic, img, b, t, tol, "plain")
    for f in mf.dtype.names:
        assert np.array_equal(mf[f], pl[f]), f
    sel = sampled(mf.size, 160)
    ref = orc.encode(img, b, t, tol=tol, sel=sel)
    assert_codes(mf, ref, sel=sel, what="512 rects %s" % (job,))


@pytest.mark.parametrize("tol", [None, 0.02, 0.1])
def test_workload_1024(fic, orc, tol):
    from synth import workload_images
    img = workload_images("fbm1024_b8t1")
    mf, _ = gpu_encode(fic, img, 8, 1, tol, "mfma")
    if tol is None:
        assert np.all(mf["flags"] == 0)
    sel = sampled(mf.size, 40 if tol is None else 64, seed=1)
    sel = np.union1d(sel, np.flatnonzero(mf["flags"])[:8])   # include empty-pool ranges
    ref = orc.encode(img, 8, 1, tol=tol, sel=sel)
    assert_codes(mf, ref, sel=sel, what="1024 tol=%s" % tol)


@pytest.mark.parametrize("job", [(16, 4, 0.05), (8, 2, 0.05), (16, 4, None)])
def test_workload_2048(fic, orc, job):
    from synth import workload_images
    img = workload_images("fbm2048_twolevel")
    b, t, tol = job
    mf, _ = gpu_encode(fic, img, b, t, tol, "mfma")
    sel = sampled(mf.size, 48, seed=2)
    ref = orc.encode(img, b, t, tol=tol, sel=sel)
    assert_codes(mf, ref, sel=sel, what="2048 %s" % (job,))


@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_single(fic, orc, graph):
    from synth import batch_descs
    items = batch_descs(count=6)
    imgs = [dev(im) for (im, _, _, _) in items]
    jobs = [(b, t, tol) for (_, b, t, tol) in items]
    outs = fic.encode_batch(imgs, jobs, graph=graph)
    torch.cuda.synchronize()
    for (im, b, t, tol), c in zip(items, outs):
        got = fic.unpack_codes(c)
        single, _ = gpu_encode(fic, im, b, t, tol, "mfma")
        for f in got.dtype.names:
            assert np.array_equal(got[f], single[f]), f
        sel = sampled(got.size, 24, seed=3)
        ref = orc.encode(im, b, t, tol=tol, sel=sel)
        assert_codes(got, ref, sel=sel, what="batch %dx%d B=%d" % (im.shape + (b,)))


def _single_codes(fic, im, b, t, tol):
    c, _ = fic.encode(dev(im), b, t, tol=tol, kernel="mfma")
    torch.cuda.synchronize()
    return c.cpu().numpy()


def test_batch_mixed_sizes_and_idle_image(fic, orc):
    """Range sizes 4, 8 and 16 in one batch (one persistent search per size),
    exhaustive and pooled jobs, and a flat image whose ranges need no search
    (zero work items) between images that have items."""
    rng = np.random.default_rng(11)
    from synth import fbm as _f, piecewise_smooth
    cases = [
        (_f(128, 128, 0.5, rng), 8, 2, 0.05),
        (np.full((64, 96), 77, np.uint8), 8, 1, None),
        (piecewise_smooth(128, rng), 4, 2, None),
        (_f(128, 128, 0.7, rng), 16, 4, None),
        (_f(96, 64, 0.3, rng), 4, 1, 0.1),
        (_f(64, 64, 0.4, rng), 16, 2, 0.05),
        (_f(160, 96, 0.6, rng), 8, 3, -1.0),
    ]
    imgs = [dev(im) for (im, _, _, _) in cases]
    jobs = [(b, t, tol) for (_, b, t, tol) in cases]
    for graph in (False, True):
        outs = fic.encode_batch(imgs, jobs, graph=graph)
        torch.cuda.synchronize()
        for (im, b, t, tol), c in zip(cases, outs):
            got = fic.unpack_codes(c)
            ref = orc.encode(im, b, t, tol=tol)
            assert_codes(got, ref, what="mixed batch %dx%d B=%d t=%d tol=%s graph=%s"
                         % (im.shape + (b, t, tol, graph)))


def test_batch_graph_replays(fic):
    """A recorded batch replayed several times, with other work and host
    synchronisation between the replays, equals the eager batch every time;
    a replay after the images change encodes the new contents."""
    from synth import batch_descs
    items = batch_descs(count=5, base_seed=4100)
    imgs = [dev(im) for (im, _, _, _) in items]
    jobs = [(b, t, tol) for (_, b, t, tol) in items]
    eager = [c.cpu().numpy() for c in fic.encode_batch(imgs, jobs, graph=False)]
    torch.cuda.synchronize()
    wsb = fic.batch_workspace_bytes(imgs, jobs)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    codes = [torch.empty_like(torch.from_numpy(e)).cuda() for e in eager]
    other = dev(np.random.default_rng(5).integers(0, 256, (64, 64)).astype(np.uint8))
    for rep in range(4):
        codes_out = fic.encode_batch(imgs, jobs, codes=codes, ws=ws, graph=True)
        torch.cuda.synchronize()
        for i, (c, e) in enumerate(zip(codes_out, eager)):
            assert np.array_equal(c.cpu().numpy(), e), "replay %d image %d" % (rep, i)
        fic.encode(other, 8, 1)          # eager work between replays
        ws.fill_(0xA5)                   # replays must not depend on stale workspace
        torch.cuda.synchronize()
    # new contents under the same pointers: the replay encodes them
    new0 = np.ascontiguousarray(np.flipud(items[0][0]))
    imgs[0].copy_(torch.from_numpy(new0))
    out = fic.encode_batch(imgs, jobs, codes=codes, ws=ws, graph=True)
    torch.cuda.synchronize()
    b, t, tol = jobs[0]
    assert np.array_equal(out[0].cpu().numpy(), _single_codes(fic, new0, b, t, tol))
    for i in range(1, len(items)):
        assert np.array_equal(out[i].cpu().numpy(), eager[i])


def test_batch_full_64(fic, orc):
    """The 64-image mixed batch (sizes 128..1024, B in {4, 8}, t = 2,
    tol = 0.05) in one call: every image equals its single-image encode, and
    sampled ranges of 8 images equal the oracle."""
    from synth import batch_descs
    items = batch_descs(count=64)
    imgs = [dev(im) for (im, _, _, _) in items]
    jobs = [(b, t, tol) for (_, b, t, tol) in items]
    outs = fic.encode_batch(imgs, jobs, graph=True)
    torch.cuda.synchronize()
    for m, ((im, b, t, tol), c) in enumerate(zip(items, outs)):
        got = c.cpu().numpy()
        assert np.array_equal(got, _single_codes(fic, im, b, t, tol)), "image %d" % m
        if m % 8 == 3:
            g = fic.unpack_codes(c)
            sel = sampled(g.size, 16, seed=m)
            ref = orc.encode(im, b, t, tol=tol, sel=sel)
            assert_codes(g, ref, sel=sel, what="batch64 image %d" % m)


def test_repeat_determinism(fic):
    """The packed-key minimum does not depend on the order in which waves
    finish: repeated runs give identical codes."""
    from synth import workload_images
    img = dev(workload_images("fbm512rect_b8t2"))
    first = None
    for _ in range(3):
        c, _ = fic.encode(img, 8, 2, tol=0.05, kernel="mfma")
        torch.cuda.synchronize()
        a = c.cpu().numpy()
        if first is None:
            first = a
        assert np.array_equal(a, first)


# ----------------------------------------------------------------- decode
@pytest.mark.parametrize("case", [(64, 8, 1, None), (128, 4, 2, 0.05), (128, 16, 4, None)])
def test_decode(fic, orc, case):
    n, b, t, tol = case
    img = fbm(n, 0.6, n + b)
    codes, _ = fic.encode(dev(img), b, t, tol=tol)
    out, iters = fic.decode_pifs(codes, n, n, b, t, max_iters=32)
    torch.cuda.synchronize()
    got = fic.unpack_codes(codes)
    ref_codes = {"dom": got["domain"], "iso": got["iso"], "k": got["s_idx"], "j": got["o_idx"]}
    ref, it = orc.decode(ref_codes, n, n, b, t, max_iters=32)
    assert np.array_equal(out.cpu().numpy(), ref)
    assert int(iters.item()) == it
    assert orc.psnr(ref, img) > 20.0
    # a partial decode from a given start image
    start = np.random.default_rng(1).integers(0, 256, (n, n)).astype(np.uint8)
    out2, it2 = fic.decode_pifs(codes, n, n, b, t, max_iters=3, init=dev(start))
    torch.cuda.synchronize()
    ref2, r2 = orc.decode(ref_codes, n, n, b, t, max_iters=3, init=start)
    assert np.array_equal(out2.cpu().numpy(), ref2) and int(it2.item()) == r2


# ----------------------------------------------------------- quadtree
def _qt_compare(fic, orc, img, b1, t1, tol1, b2, t2, tol2, rms, what):
    c1, c2 = fic.encode_quadtree(dev(img), b1, t1, tol1, b2, t2, tol2, rms)
    torch.cuda.synchronize()
    g1, g2 = fic.unpack_codes(c1), fic.unpack_codes(c2)
    r1, r2 = orc.encode_quadtree(img, b1, t1, tol1, b2, t2, tol2, rms)
    assert_codes(g1, r1, what=what + " level 1")
    assert_codes(g2, r2, what=what + " level 2")
    return c1, c2, r1, r2


@pytest.mark.parametrize("case", [
    # (image kind, size, B1, t1, tol1, B2, t2, tol2, rms)
    ("fbm", 64, 8, 2, 0.05, 4, 2, 0.05, 15.3),
    ("fbm", 128, 16, 4, None, 8, 2, None, 9.0),
    ("poly", 128, 16, 2, 0.05, 8, 2, 0.1, 6.0),
    ("fbm", 96, 8, 1, -1.0, 4, 1, None, 12.0),
    ("noise", 64, 8, 2, None, 4, 2, 0.1, 0.0),
    ("fbm", 64, 16, 4, 0.05, 8, 4, 0.05, float("inf")),
])
def test_quadtree_codes(fic, orc, case):
    kind, n, b1, t1, tol1, b2, t2, tol2, rms = case
    rng = np.random.default_rng(n + b1 + int(rms if np.isfinite(rms) else 99))
    if kind == "fbm":
        img = fbm(n, 0.6, n + 7)
    elif kind == "poly":
        from synth import piecewise_smooth
        img = piecewise_smooth(n, rng)
    else:
        img = rng.integers(0, 256, (n, n)).astype(np.uint8)
    _qt_compare(fic, orc, img, b1, t1, tol1, b2, t2, tol2, rms, "quadtree %s" % (case,))


@pytest.mark.parametrize("case", [(64, 8, 2, 4, 2, 15.3), (128, 16, 4, 8, 2, 9.0)])
def test_quadtree_decode(fic, orc, case):
    n, b1, t1, b2, t2, rms = case
    img = fbm(n, 0.6, n + 7)
    c1, c2, r1, r2 = _qt_compare(fic, orc, img, b1, t1, 0.05, b2, t2, 0.05, rms,
                                 "quadtree decode %s" % (case,))
    split = (fic.unpack_codes(c1)["flags"] & 2) != 0
    assert 0 < split.sum() < split.size
    out, iters = fic.decode_quadtree(c1, c2, n, n, b1, t1, b2, t2, max_iters=32)
    torch.cuda.synchronize()
    ref, it = orc.decode_quadtree(r1, r2, n, n, b1, t1, b2, t2, max_iters=32)
    assert np.array_equal(out.cpu().numpy(), ref) and int(iters.item()) == it
    start = np.random.default_rng(3).integers(0, 256, (n, n)).astype(np.uint8)
    out2, it2 = fic.decode_quadtree(c1, c2, n, n, b1, t1, b2, t2, max_iters=2, init=dev(start))
    torch.cuda.synchronize()
    ref2, r2i = orc.decode_quadtree(r1, r2, n, n, b1, t1, b2, t2, max_iters=2, init=start)
    assert np.array_equal(out2.cpu().numpy(), ref2) and int(it2.item()) == r2i


def test_quadtree_workload_2048(fic, orc):
    """2048x2048 fBm, 16x16 ranges (step 4) over 8x8 ranges (step 2), FD pools
    0.05, split above 1.9 gray levels RMS (about a quarter of the ranges):
    split decisions on every range from the GPU's own exact E, and sampled
    codes of both levels against the oracle."""
    from synth import WORKLOADS, workload_images
    wl = WORKLOADS["fbm2048_quadtree"]
    img = workload_images("fbm2048_quadtree")
    c1, c2 = fic.encode_quadtree(dev(img), 16, 4, 0.05, 8, 2, 0.05, wl.rms)
    torch.cuda.synchronize()
    g1, g2 = fic.unpack_codes(c1), fic.unpack_codes(c2)
    emax = orc.split_threshold(16, wl.rms)
    split = (g1["flags"] & 2) != 0
    assert np.array_equal(split, g1["err"] > emax)
    assert 0 < split.sum() < split.size
    rc1, rc2 = 2048 // 16, 2048 // 8
    r2 = np.arange(g2.size)
    coded = (g2["flags"] & 4) == 0
    assert np.array_equal(coded, split[(r2 // rc2 // 2) * rc1 + (r2 % rc2) // 2])
    sel1 = sampled(g1.size, 24, seed=5)
    ref1 = orc.encode(img, 16, 4, tol=0.05, sel=sel1)
    ref1["flags"] = ref1["flags"] | np.where(ref1["err"] > emax, 2, 0)
    assert_codes(g1, ref1, sel=sel1, what="2048 quadtree level 1")
    kids = np.flatnonzero(coded)
    sel2 = np.sort(np.random.default_rng(6).choice(kids, size=24, replace=False))
    ref2 = orc.encode(img, 8, 2, tol=0.05, sel=sel2)
    assert_codes(g2, ref2, sel=sel2, what="2048 quadtree level 2")


# ----------------------------------------------------------- bitstream, 2x decode
@pytest.mark.parametrize("case", [("fbm1024_b8t1", 8, 1, None), ("fbm512rect_b8t2", 8, 2, 0.05),
                                  ("small", 4, 2, 0.1), ("small16", 16, 4, None)])
def test_pack_codes_bit_exact(fic, orc, case):
    name, b, t, tol = case
    if name == "small":
        img = fbm(128, 0.5, 61)
    elif name == "small16":
        img = fbm(128, 0.7, 62)
    else:
        from synth import workload_images
        img = workload_images(name)
    H, W = img.shape
    x = dev(img)
    codes, _ = fic.encode(x, b, t, tol=tol)
    words = fic.fic.pack_codes(codes, H, W, b, t)
    torch.cuda.synchronize()
    got = fic.unpack_codes(codes)
    ref_codes = {"dom": got["domain"], "iso": got["iso"], "k": got["s_idx"], "j": got["o_idx"]}
    D = orc.num_domains(H, W, b, t)
    ref_words = orc.pack_codes(ref_codes, D)
    assert np.array_equal(words.cpu().numpy().view(np.uint32), ref_words)
    back = fic.unpack_codes(fic.fic.unpack_bitstream(words, H, W, b, t))
    for f in ("domain", "iso", "s_idx", "o_idx"):
        assert np.array_equal(back[f], got[f]), f
    assert np.all(back["flags"] == 0) and np.all(back["err"] == 0)


@pytest.mark.parametrize("b,t,n", [(4, 2, 64), (8, 2, 128), (16, 4, 128)])
def test_decode_twice_size(fic, orc, b, t, n):
    img = fbm(n, 0.6, 40 + b)
    codes, _ = fic.encode(dev(img), b, t, tol=0.1)
    out, iters = fic.decode_pifs(codes, n, n, b, t, max_iters=32, scale=2)
    torch.cuda.synchronize()
    got = fic.unpack_codes(codes)
    ref_codes = {"dom": got["domain"], "iso": got["iso"], "k": got["s_idx"], "j": got["o_idx"]}
    ref, it = orc.decode_scaled(ref_codes, n, n, b, t, 2, max_iters=32)
    assert out.shape == (2 * n, 2 * n)
    assert np.array_equal(out.cpu().numpy(), ref) and int(iters.item()) == it


# ----------------------------------------------------------- colour
@pytest.mark.parametrize("case", [(0, 0.05, 8, 2, 128, 96), (1, 0.1, 4, 2, 64, 64),
                                  (0, None, 8, 1, 64, 64), (1, -1.0, 16, 4, 128, 128)])
def test_color_codes(fic, orc, case):
    src, tol, b, t, h, w = case
    rng = np.random.default_rng(80 + b)
    from synth import fbm as _f
    rgb = np.stack([_f(h, w, hh, rng) for hh in (0.3, 0.55, 0.8)], axis=2)
    codes = fic.encode_color(torch.from_numpy(rgb).cuda(), b, t, tol=tol,
                             fd_source=("luma", "mean")[src])
    torch.cuda.synchronize()
    ref = orc.encode_color(rgb, b, t, tol, fd_source=src)
    for c in range(3):
        assert_codes(fic.unpack_codes(codes[c]), ref[c], what="colour %s channel %d" % (case, c))


def test_color_of_gray_equals_gray(fic):
    img = fbm(128, 0.5, 90)
    rgb = np.ascontiguousarray(np.stack([img, img, img], axis=2))
    codes = fic.encode_color(torch.from_numpy(rgb).cuda(), 8, 2, tol=0.05)
    gray, _ = fic.encode(dev(img), 8, 2, tol=0.05)
    torch.cuda.synchronize()
    for c in range(3):
        assert np.array_equal(codes[c].cpu().numpy(), gray.cpu().numpy())
