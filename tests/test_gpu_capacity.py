"""Searches at the capacity limit of the packed search keys.

A key packs (F, domain index, isometry) into 64 bits (Sec. 2's argmin with
its tie-breaks). F stays below 2^38 at 8x8 ranges and below 2^42 at 16x16,
which leaves 23 and 19 bits for the domain index: a 2904 x 2904 image at
domain step 1 has 8,346,321 domains for 8x8 ranges (2^23 = 8,388,608), and a
2912 x 2912 image at step 4 has 519,841 domains for 16x16 ranges
(2^19 = 524,288), so their keys use every bit. The GPU codes of sampled
ranges (the first, the last, seeded random ones and those whose best domain
has the highest indices) must equal the oracle's, exhaustively and with the
Sec. 3.1 pool; no code may fail finalize's recompute (bit 7).

The work list is planned for every range group against every chunk of the
narrowest item width; a job whose list would pass 2^26 entries at 2048
columns plans wider items instead. 4x4 ranges on a 4096 x 4096 image at
step 1 (65,536 groups, 16.7 M domains) take 16384-column items: their codes
are checked the same way.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# (image size, range size, domain step, bits left for the domain index)
LIMITS = {8: (2904, 8, 1, 23), 16: (2912, 16, 4, 19)}


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


_images = {}


def image(size):
    from synth import fbm
    if size not in _images:
        _images[size] = fbm(size, size, 0.5, np.random.default_rng(77))
    return _images[size]


def assert_codes(got, ref, what):
    pairs = (("domain", "dom"), ("iso", "iso"), ("s_idx", "k"), ("o_idx", "j"),
             ("flags", "flags"), ("err", "err"))
    for fg, fr in pairs:
        a = got[fg].astype(np.int64)
        b = np.asarray(ref[fr]).astype(np.int64)
        if not np.array_equal(a, b):
            bad = np.flatnonzero(a != b)[:5]
            raise AssertionError("%s: field %s differs at %s: gpu %s oracle %s"
                                 % (what, fg, bad, a[bad], b[bad]))


@pytest.mark.parametrize("b,tol,n_random", [(8, None, 4), (8, 0.02, 10), (16, None, 10),
                                            (16, 0.05, 10)])
def test_keys_at_the_domain_limit(fic, orc, b, tol, n_random):
    size, _, t, bits = LIMITS[b]
    img = image(size)
    R, D = orc.num_ranges(size, size, b), orc.num_domains(size, size, b, t)
    assert 2 ** (bits - 1) < D < 2 ** bits, D    # the domain field's bits all in use
    x = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    codes, _ = fic.encode(x, b, t, tol=tol)
    torch.cuda.synchronize()
    got = fic.unpack_codes(codes)
    assert got.size == R
    assert not np.any(got["flags"] & 0x80)
    coded = np.flatnonzero((got["flags"] & 1) == 0)
    top = coded[np.argsort(got["domain"][coded], kind="stable")[-2:]]
    assert got["domain"][top].max() >= 2 ** (bits - 1)   # a winner in the top half of the index range
    rnd = np.random.default_rng(5).choice(R, n_random, replace=False)
    sel = np.unique(np.concatenate([[0, R - 1], top, rnd])).astype(np.int64)
    ref = orc.encode(img, b, t, tol=tol, sel=sel)
    assert_codes(got[sel], ref, "%dx%d, %dx%d ranges, step %d, tol %s" % (size, size, b, b, t, tol))


def test_work_list_with_wider_items(fic, orc):
    import ctypes
    size, b, t = 4096, 4, 1
    img = image(size)
    g = fic.fic.make_geom(size, size, b, t)
    # 65,536 groups x 8,176 chunks of 2048 columns would be 8.6 GB of items
    assert fic.fic.lib().fic_encode_workspace_bytes(ctypes.byref(g), 1) < 3 << 30
    R = orc.num_ranges(size, size, b)
    x = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    for tol in (0.01, None):
        codes, _ = fic.encode(x, b, t, tol=tol)
        torch.cuda.synchronize()
        got = fic.unpack_codes(codes)
        assert got.size == R and not np.any(got["flags"] & 0x80)
        sel = np.unique(np.concatenate([[0, R - 1], np.random.default_rng(6).choice(R, 8, replace=False)]))
        ref = orc.encode(img, b, t, tol=tol, sel=sel.astype(np.int64))
        assert_codes(got[sel], ref, "%dx%d, 4x4 ranges, step 1, tol %s" % (size, size, tol))
