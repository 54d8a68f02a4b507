"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these checks re-types the oracle's own formula: each compares it with
a value printed in the paper, a hand count, an independent derivation (numpy
rotations, the pixel-level grid brute force) or an invariant.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import bruteforce as bf

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _fbm(n, h, seed):
    from synth import fbm
    return fbm(n, n, h, np.random.default_rng(seed))


# ---------------------------------------------------------------- geometry
def test_table1_counts(oracle_lib):
    """Sec. 2, Table 1: ranges, domains and comparisons of the 8/16 lattice."""
    with open(os.path.join(GOLD, "table1_counts.json")) as f:
        tab = json.load(f)
    for row in tab["rows"]:
        n = row["image"]
        nr = oracle_lib.num_ranges(n, n, tab["range_size"])
        nd = oracle_lib.num_domains(n, n, tab["range_size"], tab["domain_step"])
        assert (nr, nd, nr * nd) == (row["ranges"], row["domains"], row["comparisons"])
    # the 1024 example of Sec. 2: about 2^34 comparisons
    assert abs(math.log2(16384 * 1018081) - 34) < 0.05


def test_lattice_matches_enumeration(oracle_lib):
    for (h, w, b, t) in [(32, 48, 4, 1), (32, 48, 4, 3), (64, 64, 8, 2), (64, 96, 16, 4)]:
        ranges, doms = bf.lattice(h, w, b, t)
        assert oracle_lib.num_ranges(h, w, b) == len(ranges)
        assert oracle_lib.num_domains(h, w, b, t) == len(doms)


# -------------------------------------------------------------- isometries
def test_isometry_table_matches_numpy_derivation(oracle_lib):
    """The C index table against numpy's rot90/flip/transpose."""
    rng = np.random.default_rng(7)
    for b in (4, 8, 16):
        blk = rng.integers(0, 1000, size=(b, b))
        ref = bf.isometries(blk)
        for q in range(8):
            assert np.array_equal(oracle_lib.iso_apply(q, blk), ref[q]), (b, q)


def test_isometry_group_laws(oracle_lib):
    """D4: rotation of order 4, rotations compose, reflections are
    involutions, reflection = rotation o mirror, all 8 distinct."""
    b = 8
    blk = np.arange(b * b, dtype=np.int64).reshape(b, b)
    T = lambda q, x: oracle_lib.iso_apply(q, x)
    r1 = lambda x: T(1, x)
    assert np.array_equal(r1(r1(r1(r1(blk)))), blk)
    assert np.array_equal(r1(r1(blk)), T(2, blk))
    assert np.array_equal(r1(r1(r1(blk))), T(3, blk))
    for q in (4, 5, 6, 7):
        assert np.array_equal(T(q, T(q, blk)), blk)
    assert np.array_equal(T(4, T(6, blk)), T(1, blk))     # mirror-LR(transpose(d)) = rot90 cw
    assert np.array_equal(T(6, T(4, blk)), T(3, blk))     # transpose(mirror-LR(d)) = rot270 cw
    assert np.array_equal(T(2, T(6, blk)), T(7, blk))     # anti-transpose = transpose o rot180
    assert len({T(q, blk).tobytes() for q in range(8)}) == 8


# ------------------------------------------------- closed form vs the grid
@pytest.mark.parametrize("b", [4, 8])
def test_pair_fit_equals_grid_bruteforce(oracle_lib, b):
    """F(k) + 4096 (sum r - 2nj)^2 with the scanned k and j equals the
    pixel-level minimum over the whole 32 x 128 (k, j) grid."""
    rng = np.random.default_rng(11 + b)
    for trial in range(40):
        kind = trial % 4
        if kind == 0:
            img = rng.integers(0, 256, size=(4 * b, 4 * b)).astype(np.uint8)
        elif kind == 1:
            img = _fbm(4 * b, 0.4, int(rng.integers(1 << 30)))
        elif kind == 2:      # a flat domain region
            img = rng.integers(0, 256, size=(4 * b, 4 * b)).astype(np.uint8)
            img[:2 * b, :2 * b] = rng.integers(0, 256)
        else:                # smooth ramp
            y, x = np.mgrid[0:4 * b, 0:4 * b]
            img = np.clip(3 * x + 2 * y + rng.integers(0, 60), 0, 255).astype(np.uint8)
        h = w = 4 * b
        t = 1
        ranges, doms = bf.lattice(h, w, b, t)
        r = int(rng.integers(len(ranges)))
        d = 0 if kind == 2 else int(rng.integers(len(doms)))
        q = int(rng.integers(8))
        f, k = oracle_lib.pair_f(img, b, t, r, d, q)
        (ry, rx), (dy, dx) = ranges[r], doms[d]
        rblk = img[ry:ry + b, rx:rx + b]
        tq = bf.isometries(bf.shrink(img, dy, dx, b))[q]
        e_ref, k_ref, j_ref = bf.brute_pair(rblk, tq)
        sr = int(rblk.astype(np.int64).sum())
        n = b * b
        j = (sr + n - 1) // (2 * n)
        assert (k, j) == (k_ref, j_ref)
        assert f + 4096 * (sr - 2 * n * j) ** 2 == e_ref


# --------------------------------------------------- whole-search brute force
@pytest.mark.parametrize("case", [
    ("uniform", 16, 4, 2), ("fbm", 16, 4, 1), ("fbm", 24, 4, 2), ("ramp", 16, 4, 2),
    ("fbm", 32, 8, 4), ("blocks", 16, 4, 2),
])
def test_search_equals_grid_bruteforce(oracle_lib, case):
    kind, size, b, t = case
    rng = np.random.default_rng(size * 31 + b)
    if kind == "uniform":
        img = rng.integers(0, 256, size=(size, size)).astype(np.uint8)
    elif kind == "fbm":
        img = _fbm(size, 0.6, size + b)
    elif kind == "ramp":
        y, x = np.mgrid[0:size, 0:size]
        img = (7 * x + 3 * y).astype(np.uint8)
    else:                     # piecewise constant: many exact ties
        img = np.kron(rng.integers(0, 4, size=(size // 4, size // 4)) * 60,
                      np.ones((4, 4))).astype(np.uint8)
    ref = bf.brute_encode(img, b, t)
    got = oracle_lib.encode(img, b, t)
    for key in ("dom", "iso", "k", "j", "err"):
        assert np.array_equal(got[key], ref[key]), key


def test_search_with_pools_equals_bruteforce(oracle_lib):
    img = _fbm(24, 0.5, 99)
    b, t, tol = 4, 2, 0.15
    fr, fd = oracle_lib.classify(img, b, t)
    pools = [np.flatnonzero(np.abs(fd - x) <= tol + 1e-9) for x in fr]
    assert min(len(p) for p in pools) < len(fd)          # the window really prunes
    ref = bf.brute_encode(img, b, t, pools=pools)
    got = oracle_lib.encode(img, b, t, tol=tol, fds=(fr, fd))
    for i, p in enumerate(pools):
        if len(p) == 0:
            assert got["flags"][i] == 1
            continue
        for key in ("dom", "iso", "k", "j", "err"):
            assert got[key][i] == ref[key][i], (i, key)
    assert np.array_equal(got["pool"], np.array([len(p) for p in pools]))


# ------------------------------------------------------------ planted cases
def test_planted_zero_error_copy(oracle_lib):
    """A range that is exactly s=1/2 times an isometric copy of a domain
    (plus an even offset) is encoded with zero error."""
    b, t = 4, 2
    rng = np.random.default_rng(5)
    img = _fbm(32, 0.5, 3)
    v = 2 * rng.integers(10, 100, size=(b, b))           # even cell values
    v[0, 0] += (-v.sum()) % (2 * b * b)                    # mean(v) even
    assert v.sum() % (2 * b * b) == 0
    dy, dx = 16, 16
    img[dy:dy + 2 * b, dx:dx + 2 * b] = np.kron(v, np.ones((2, 2)))
    q = 3
    r_blk = (bf.isometries(v)[q] - v.mean()) // 2 + 2 * 64
    ry, rx = 0, 4
    img[ry:ry + b, rx:rx + b] = r_blk
    ranges, doms = bf.lattice(32, 32, b, t)
    r = ranges.index((ry, rx))
    d = doms.index((dy, dx))
    f, k = oracle_lib.pair_f(img, b, t, r, d, q)
    assert (f, k) == (0, 8)
    got = oracle_lib.encode(img, b, t, sel=[r])
    assert got["err"][0] == 0
    assert (got["dom"][0], got["iso"][0]) <= (d, q)


def test_planted_unit_contrast_copy(oracle_lib):
    """An exact copy (s = 1) is off the grid: k = 15 and F = 16 Srr'."""
    b, t = 4, 2
    img = _fbm(32, 0.5, 8)
    rng = np.random.default_rng(1)
    cells = rng.integers(0, 64, size=(b, b))               # D = 4 * cells
    img[16:24, 8:16] = np.kron(cells, np.ones((2, 2)))
    q = 6
    r_blk = bf.isometries(cells)[q]
    img[0:4, 0:4] = r_blk
    ranges, doms = bf.lattice(32, 32, b, t)
    f, k = oracle_lib.pair_f(img, b, t, ranges.index((0, 0)), doms.index((16, 8)), q)
    n = b * b
    srr = n * int((r_blk.astype(np.int64) ** 2).sum()) - int(r_blk.sum()) ** 2
    assert k == 15 and f == 16 * srr


def test_flat_range_takes_first_pair(oracle_lib):
    img = _fbm(32, 0.5, 12)
    img[8:12, 8:12] = 77
    ranges, _ = bf.lattice(32, 32, 4, 2)
    got = oracle_lib.encode(img, 4, 2, sel=[ranges.index((8, 8))])
    assert (got["dom"][0], got["iso"][0], got["k"][0]) == (0, 0, 0)
    n = 16
    assert got["j"][0] == (77 * n + n - 1) // (2 * n)
    assert got["err"][0] == 4096 * (77 * n - 2 * n * got["j"][0]) ** 2


def test_empty_pool_gives_dc_code(oracle_lib):
    img = _fbm(32, 0.5, 4)
    fr, fd = oracle_lib.classify(img, 4, 2)
    fr_far = fr + 10.0                                      # nothing within the window
    got = oracle_lib.encode(img, 4, 2, tol=0.05, fds=(fr_far, fd))
    assert np.all(got["flags"] == 1) and np.all(got["pool"] == 0)
    assert np.all(got["dom"] == 0) and np.all(got["iso"] == 0) and np.all(got["k"] == 0)
    exh = oracle_lib.encode(img, 4, 2)
    assert np.all(got["err"] >= exh["err"])


# ------------------------------------------------------- fractal dimension
def test_dbc_golden_values(oracle_lib):
    with open(os.path.join(GOLD, "dbc_values.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        for m in c["M"]:
            if c["name"].startswith("flat"):
                blk = np.full((m, m), 93, dtype=np.uint8)
            elif c["name"].startswith("0/255"):
                blk = (((np.indices((m, m)).sum(axis=0)) % 2) * 255).astype(np.uint8)
            else:
                blk = np.zeros((m, m), dtype=np.uint8)
                blk[m // 2 + 1, 1] = int(c["name"].split()[-1])
            assert abs(oracle_lib.dbc_fd(blk) - c["fd"]) < 1e-12, (c["name"], m)


def test_dbc_invariances(oracle_lib):
    """Box counts do not change under the square isometries (cells map to
    cells) nor under g -> 255 - g (h divides 256)."""
    rng = np.random.default_rng(3)
    for m in (4, 8, 16, 32):
        for _ in range(6):
            blk = _fbm(m, float(rng.uniform(0.1, 0.9)), int(rng.integers(1 << 30)))
            fd0, c0 = oracle_lib.dbc_fd(blk, return_counts=True)
            for q in range(8):
                fdq, cq = oracle_lib.dbc_fd(bf.isometries(blk)[q].copy(), return_counts=True)
                assert np.array_equal(cq, c0) and fdq == fd0
            fdi, ci = oracle_lib.dbc_fd(255 - blk, return_counts=True)
            assert np.array_equal(ci, c0)


def test_dbc_range_and_weights(oracle_lib):
    """The least-squares slope over s = 2..M equals the hand-derived
    combination of log2 counts (M=8: log2 N_2 / 2; M=16:
    0.3 log2 N_2 + 0.1 log2 N_4 - 0.1 log2 N_8), and lies in the [2, 3]
    band the paper reports for natural content."""
    rng = np.random.default_rng(17)
    for _ in range(20):
        img = _fbm(16, float(rng.uniform(0.2, 0.9)), int(rng.integers(1 << 30)))
        fd8, c8 = oracle_lib.dbc_fd(img[:8, :8], return_counts=True)
        assert abs(fd8 - 0.5 * math.log2(c8[0])) < 1e-12
        fd16, c16 = oracle_lib.dbc_fd(img, return_counts=True)
        ref = 0.3 * math.log2(c16[0]) + 0.1 * math.log2(c16[1]) - 0.1 * math.log2(c16[2])
        assert abs(fd16 - ref) < 1e-12
        assert c16[3] == 1
    big = _fbm(256, 0.5, 1)
    fd = oracle_lib.fd_blocks(big, 16, 8)
    assert 1.8 < fd.min() and fd.max() < 3.2 and 2.0 <= np.median(fd) <= 3.0


def test_fd_blocks_layout(oracle_lib):
    img = _fbm(64, 0.4, 21)
    for (m, step) in [(8, 8), (16, 1), (16, 3)]:
        fd = oracle_lib.fd_blocks(img, m, step)
        rows = (64 - m) // step + 1
        a, c = 2, rows - 1
        assert fd[a * rows + c] == oracle_lib.dbc_fd(img[a * step:a * step + m,
                                                         c * step:c * step + m].copy())


# -------------------------------------------------------------- the window
def test_fractal_distance_closed_form(oracle_lib):
    """Sec. 3.1: D_f = (F_m - F_l) / 3 over the domain set."""
    fd = np.array([2.31, 2.02, 2.97, 2.5])
    assert oracle_lib.resolve_tol(-1.0, fd) == pytest.approx((2.97 - 2.02) / 3, abs=1e-15)
    assert oracle_lib.resolve_tol(0.05, fd) == 0.05


def test_pool_limits(oracle_lib):
    """Infinite tolerance is the exhaustive search; a wider window holds the
    narrower one's pool, and a larger pool never does worse."""
    img = _fbm(64, 0.5, 31)
    b, t = 8, 2
    fds = oracle_lib.classify(img, b, t)
    exh = oracle_lib.encode(img, b, t)
    inf = oracle_lib.encode(img, b, t, tol=float("inf"), fds=fds)
    for key in ("dom", "iso", "k", "j", "err"):
        assert np.array_equal(exh[key], inf[key])
    prev = None
    for tol in (0.02, 0.05, 0.1, 0.3):
        cur = oracle_lib.encode(img, b, t, tol=tol, fds=fds)
        assert np.all(cur["f"] >= exh["f"])
        if prev is not None:
            assert np.all(cur["pool"] >= prev["pool"])
            assert np.all(cur["f"] <= prev["f"])
        prev = cur
    adaptive = oracle_lib.encode(img, b, t, tol=-1.0, fds=fds)
    assert adaptive["tol"] == pytest.approx((fds[1].max() - fds[1].min()) / 3)


def test_sampled_encode_matches_full(oracle_lib):
    img = _fbm(64, 0.5, 2)
    full = oracle_lib.encode(img, 8, 2, tol=0.05)
    sel = np.array([0, 5, 17, 63, 40])
    part = oracle_lib.encode(img, 8, 2, tol=0.05, sel=sel)
    for key in ("dom", "iso", "k", "j", "err", "pool"):
        assert np.array_equal(part[key], full[key][sel])


# -------------------------------------------------------------- decoding
def test_decode_flat_image_is_exact(oracle_lib):
    img = np.full((32, 32), 100, dtype=np.uint8)
    codes = oracle_lib.encode(img, 4, 2)
    out, it = oracle_lib.decode(codes, 32, 32, 4, 2)
    assert np.array_equal(out, img) and it == 2
    assert oracle_lib.psnr(out, img) == float("inf")


def test_decode_sweep_matches_float_definition(oracle_lib):
    rng = np.random.default_rng(9)
    for (size, b, t) in [(32, 4, 2), (32, 8, 1), (64, 16, 4)]:
        ranges, doms = bf.lattice(size, size, b, t)
        nr = len(ranges)
        codes = {"dom": rng.integers(0, len(doms), nr), "iso": rng.integers(0, 8, nr),
                 "k": rng.integers(-16, 16, nr), "j": rng.integers(0, 128, nr)}
        start = rng.integers(0, 256, size=(size, size)).astype(np.uint8)
        cur = start
        for it in range(1, 4):
            cur = bf.decode_sweep_float(cur, codes, b, t)
            got, done = oracle_lib.decode(codes, size, size, b, t, max_iters=it, init=start)
            assert np.array_equal(got, cur) and done <= it


def test_decode_reconstructs_encoding(oracle_lib):
    img = _fbm(64, 0.7, 13)
    codes = oracle_lib.encode(img, 4, 2)
    out, it = oracle_lib.decode(codes, 64, 64, 4, 2)
    assert oracle_lib.psnr(out, img) > 28.0
    assert it <= 32


def test_window_is_closed(oracle_lib):
    """Sec. 3.1 bounds the window with <= on both sides: a domain exactly
    D_f away is in the pool, including when fp64 subtraction lands an ulp
    outside (2.1 - 2.0 = 0.10000000000000009); the 1e-9 guard keeps it."""
    img = _fbm(32, 0.5, 4)
    fr, fd = oracle_lib.classify(img, 4, 2)
    fr = np.full_like(fr, 2.0)
    fd = np.full_like(fd, 5.0)
    fd[[3, 7]] = [2.1, 1.9]                  # exactly 0.1 away in real arithmetic
    fd[11] = 2.1 + 2e-9                      # clearly outside
    got = oracle_lib.encode(img, 4, 2, tol=0.1, fds=(fr, fd))
    assert np.all(got["pool"] == 2)
    assert set(np.unique(got["dom"])) <= {3, 7}


# ----------------------------------------------------------- quadtree (ref. [12])
def _qt_image(seed, n=64):
    from synth import fbm
    return fbm(n, n, 0.6, np.random.default_rng(seed))


def test_quadtree_without_split_is_the_level1_encode(oracle_lib):
    """rms = inf: no range is split; level 1 is the plain encode and the
    two-level decode is the single-level decode."""
    import oracle
    img = _qt_image(21)
    c1, c2 = oracle.encode_quadtree(img, 8, 2, 0.1, 4, 2, 0.1, rms=float("inf"))
    ref = oracle.encode(img, 8, 2, tol=0.1)
    for k in ("dom", "iso", "k", "j", "flags", "err"):
        assert np.array_equal(c1[k], ref[k]), k
    assert np.all(c2["flags"] == 4) and np.all(c2["err"] == 0)
    a, ia = oracle.decode_quadtree(c1, c2, 64, 64, 8, 2, 4, 2, max_iters=12)
    b, ib = oracle.decode(ref, 64, 64, 8, 2, max_iters=12)
    assert np.array_equal(a, b) and ia == ib


def test_quadtree_all_split_is_the_level2_encode(oracle_lib):
    """rms = 0 on an image where every range has E > 0: every range splits;
    level 2 is the full level-2 encode and the decode is its decode."""
    import oracle
    rng = np.random.default_rng(22)
    img = rng.integers(0, 256, (64, 64)).astype(np.uint8)
    c1, c2 = oracle.encode_quadtree(img, 8, 1, None, 4, 2, None, rms=0.0)
    assert np.all(c1["err"] > 0) and np.all((c1["flags"] & 2) != 0)
    ref = oracle.encode(img, 4, 2)
    for k in ("dom", "iso", "k", "j", "flags", "err"):
        assert np.array_equal(c2[k], ref[k]), k
    a, ia = oracle.decode_quadtree(c1, c2, 64, 64, 8, 1, 4, 2, max_iters=10)
    b, ib = oracle.decode(ref, 64, 64, 4, 2, max_iters=10)
    assert np.array_equal(a, b) and ia == ib


@pytest.mark.parametrize("rms", [11.0, 13.7, 16.0])
def test_quadtree_split_rule_and_children(oracle_lib, rms):
    """A range splits exactly when its mean squared error E/(4096 n^2)
    exceeds rms^2; the coded level-2 ranges are exactly those whose parent
    (the level-1 range holding their pixels) split."""
    import oracle
    img = _qt_image(23)
    c1, c2 = oracle.encode_quadtree(img, 8, 2, 0.05, 4, 2, 0.05, rms=rms)
    mse = c1["err"].astype(np.float64) / (4096.0 * 64 * 64)
    split = (c1["flags"] & 2) != 0
    assert np.array_equal(split, mse > rms * rms)
    assert 0 < split.sum() < split.size      # a partial split exercises the geometry
    rc1, rc2 = 64 // 8, 64 // 4
    r2 = np.arange(c2["flags"].size)
    parent = (r2 // rc2 // 2) * rc1 + (r2 % rc2) // 2
    coded = (c2["flags"] & 4) == 0
    assert np.array_equal(coded, split[parent])
    assert np.all(c2["err"][~coded] == 0) and np.all(c2["dom"][~coded] == 0)


def test_quadtree_sweep_is_the_union_of_level_sweeps(oracle_lib):
    """One two-level sweep from a start image equals, pixel by pixel, one
    level-1 sweep on the unsplit ranges and one level-2 sweep on the coded
    sub-ranges, each from the same start image."""
    import oracle
    img = _qt_image(24)
    c1, c2 = oracle.encode_quadtree(img, 8, 2, 0.05, 4, 2, 0.05, rms=15.3)
    assert 0 < ((c1["flags"] & 2) != 0).sum() < 64
    start = np.random.default_rng(5).integers(0, 256, (64, 64)).astype(np.uint8)
    q, _ = oracle.decode_quadtree(c1, c2, 64, 64, 8, 2, 4, 2, max_iters=1, init=start)
    s1, _ = oracle.decode(c1, 64, 64, 8, 2, max_iters=1, init=start)
    s2, _ = oracle.decode(c2, 64, 64, 4, 2, max_iters=1, init=start)
    split = ((c1["flags"] & 2) != 0).reshape(8, 8)
    from_l2 = np.kron(split, np.ones((8, 8), dtype=bool))
    expect = np.where(from_l2, s2, s1)
    assert np.array_equal(q, expect)


# ----------------------------------------------------------- code bitstream
def test_pack_codes_hand_example():
    """Two ranges on a lattice of 5 domains (3 domain bits, 18 bits a code).
    Range 0: domain 5, isometry 3, k = -16, j = 127; range 1: domain 2,
    isometry 6, k = 15, j = 1. Worked by hand (fields least significant bit
    first): range 0 sets bits 0, 2 (domain), 3, 4 (isometry), none for
    k + 16 = 0, 11..17 (j); range 1 starts at bit 18 and sets bit 19
    (domain), 22, 23 (isometry), 24..28 (k + 16 = 31), 29 (j): word 0 =
    0x1D + 0x3F800 + 0x80000 + 0xC00000 + 0x1F000000 + 0x20000000 =
    0x3FCBF81D, word 1 = 0 (bits 32..35 hold j's zero high bits)."""
    import oracle
    codes = {"dom": [5, 2], "iso": [3, 6], "k": [-16, 15], "j": [127, 1]}
    words = oracle.pack_codes(codes, 5)
    assert words.dtype == np.uint32 and words.size == 2
    assert int(words[0]) == 0x3FCBF81D and int(words[1]) == 0


def test_pack_roundtrip_and_ratio():
    import oracle
    rng = np.random.default_rng(31)
    for D in (1, 2, 3, 1000, 1018081):
        R = 333
        codes = {"dom": rng.integers(0, D, R), "iso": rng.integers(0, 8, R),
                 "k": rng.integers(-16, 16, R), "j": rng.integers(0, 128, R)}
        back = oracle.unpack_codes(oracle.pack_codes(codes, D), R, D)
        for k in codes:
            assert np.array_equal(back[k], codes[k]), (D, k)
    # 1024x1024, 8x8 ranges, 1,018,081 domains: 20 + 15 = 35 bits a range
    assert oracle.code_bits(1018081) == (20, 35)
    assert abs(oracle.compression_ratio(1024, 1024, 16384, 1018081) - 8 * 1024 * 1024 / (16384 * 35)) < 1e-3


# ----------------------------------------------------------- decoding at 2x
def test_decode_scaled_dc_codes_are_pixel_doubled():
    """Codes with k = 0 are constant maps (value 2j): at twice the size each
    range is the same constant on a block twice as wide."""
    import oracle
    rng = np.random.default_rng(51)
    h = w = 64
    for b, t in ((4, 2), (8, 1), (16, 4)):
        R, D = oracle.num_ranges(h, w, b), oracle.num_domains(h, w, b, t)
        codes = {"dom": rng.integers(0, D, R), "iso": rng.integers(0, 8, R),
                 "k": np.zeros(R, dtype=np.int64), "j": rng.integers(0, 128, R)}
        o1, _ = oracle.decode(codes, h, w, b, t, max_iters=3)
        o2, _ = oracle.decode_scaled(codes, h, w, b, t, 2, max_iters=3)
        assert np.array_equal(o2, np.kron(o1, np.ones((2, 2), dtype=np.uint8)))


@pytest.mark.parametrize("b,t,n", [(4, 2, 64), (8, 2, 64), (16, 4, 128)])
def test_decode_scaled_attractor_matches(b, t, n):
    """Resolution independence: the attractor decoded at twice the size,
    averaged over 2x2 pixels, is the attractor at the encoded size up to
    rounding (within 45 dB)."""
    import oracle
    from synth import fbm
    img = fbm(n, n, 0.6, np.random.default_rng(40 + b))
    c = oracle.encode(img, b, t, tol=0.1)
    o1, _ = oracle.decode(c, n, n, b, t)
    o2, _ = oracle.decode_scaled(c, n, n, b, t, 2)
    down = np.round(o2.reshape(n, 2, n, 2).astype(np.float64).mean(axis=(1, 3))).astype(np.uint8)
    assert oracle.psnr(down, o1) > 45.0


# ----------------------------------------------------------- colour
@pytest.mark.parametrize("fd_source", [0, 1])
def test_color_of_gray_is_the_gray_encode(oracle_lib, fd_source):
    """A gray image in all three channels: both conversions give the gray
    value back ((299 + 587 + 114) v + 500) div 1000 = (3v + 1) div 3 = v), so
    every channel's codes are the gray encode's."""
    import oracle
    from synth import fbm
    g = fbm(64, 64, 0.5, np.random.default_rng(71))
    rgb = np.stack([g, g, g], axis=2)
    planes, fdimg = oracle.color_planes(rgb, fd_source)
    assert np.array_equal(fdimg, g)
    ref = oracle.encode(g, 8, 2, tol=0.1)
    for c in oracle.encode_color(rgb, 8, 2, 0.1, fd_source):
        for k in ("dom", "iso", "k", "j", "flags", "err"):
            assert np.array_equal(c[k], ref[k]), k


def test_color_mean_is_channel_symmetric(oracle_lib):
    """With the channel mean as the dimension image, permuting the channels
    permutes the codes."""
    import oracle
    from synth import fbm
    rng = np.random.default_rng(72)
    rgb = np.stack([fbm(64, 64, h, rng) for h in (0.3, 0.5, 0.8)], axis=2)
    a = oracle.encode_color(rgb, 8, 2, 0.05, fd_source=1)
    b = oracle.encode_color(rgb[:, :, [2, 0, 1]], 8, 2, 0.05, fd_source=1)
    for src, dst in ((2, 0), (0, 1), (1, 2)):
        for k in ("dom", "iso", "k", "j", "flags", "err"):
            assert np.array_equal(a[src][k], b[dst][k]), (src, k)
    # the luma weights are not symmetric: at least one pool differs
    c = oracle.encode_color(rgb, 8, 2, 0.05, fd_source=0)
    assert any(not np.array_equal(c[i]["pool"], a[i]["pool"]) for i in range(3))
