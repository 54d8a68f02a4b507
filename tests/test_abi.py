"""The C ABI on a machine without a GPU: the library loads, exports every
symbol include/fic.h declares, and validates arguments with the documented
status codes (a host-only context answers FIC_ERR_DEVICE once the
arguments are valid). No compute call is made here."""
import ctypes
import os
import re

import pytest

from paper_1206_4880_amd import fic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fic.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(fic.LIB_PATH):
        from paper_1206_4880_amd import build
        build.build()
    return fic.lib()


@pytest.fixture(scope="module")
def hctx(L):
    c = fic.Context(-1)
    yield c
    c.close()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fic_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported(L):
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(fic.EXPORTED)


def test_status_strings(L):
    for s in range(6):
        assert fic.status_string(s) not in ("", "unknown status")
    assert fic.status_string(99) == "unknown status"


def test_create_without_device(L):
    h = ctypes.c_void_p()
    assert L.fic_create(0, ctypes.byref(h)) == fic.ERR_DEVICE
    assert L.fic_create(-2, ctypes.byref(h)) == fic.ERR_INVALID_ARG
    assert L.fic_create(0, None) == fic.ERR_INVALID_ARG


def test_geometry_helpers_match_table1(L, oracle_lib):
    for n in (64, 128, 256, 512, 1024):
        g = fic.make_geom(n, n, 8, 1)
        assert L.fic_num_ranges(ctypes.byref(g)) == oracle_lib.num_ranges(n, n, 8)
        assert L.fic_num_domains(ctypes.byref(g)) == oracle_lib.num_domains(n, n, 8, 1)
    assert L.fic_num_domains(ctypes.byref(fic.make_geom(100, 64, 8, 1))) == 0  # 100 % 8


def _encode(L, ctx, g, perm=None, lo=None, hi=None, kernel=0, codes=1, ws=1, wsb=None, img=1):
    if wsb is None:
        wsb = L.fic_encode_workspace_bytes(ctypes.byref(g), int(perm is not None))
    return L.fic_encode_pifs(ctx.handle, img, ctypes.byref(g), perm, lo, hi, kernel, codes, ws,
                             wsb, None)


def test_encode_validation(L, hctx):
    good = fic.make_geom(64, 64, 8, 1)
    assert _encode(L, hctx, good) == fic.ERR_DEVICE           # valid, but no device
    bad_geoms = [fic.make_geom(64, 64, 6, 1), fic.make_geom(60, 64, 8, 1),
                 fic.make_geom(64, 8, 8, 1), fic.make_geom(64, 64, 8, 0),
                 fic.make_geom(64, 64, 8, 1, pitch=32), fic.make_geom(0, 64, 8, 1)]
    for g in bad_geoms:
        assert _encode(L, hctx, g, wsb=1 << 30) == fic.ERR_INVALID_ARG
    assert _encode(L, hctx, good, img=None) == fic.ERR_INVALID_ARG
    assert _encode(L, hctx, good, codes=None) == fic.ERR_INVALID_ARG
    assert _encode(L, hctx, good, ws=None) == fic.ERR_INVALID_ARG
    assert _encode(L, hctx, good, kernel=7) == fic.ERR_INVALID_ARG
    assert _encode(L, hctx, good, perm=1, lo=None, hi=1, wsb=1 << 30) == fic.ERR_INVALID_ARG
    need = L.fic_encode_workspace_bytes(ctypes.byref(good), 0)
    assert need > 0
    assert _encode(L, hctx, good, wsb=need - 1) == fic.ERR_WORKSPACE
    pooled = L.fic_encode_workspace_bytes(ctypes.byref(good), 1)
    assert _encode(L, hctx, good, perm=1, lo=1, hi=1, wsb=pooled) == fic.ERR_DEVICE
    assert L.fic_encode_pifs(None, 1, ctypes.byref(good), None, None, None, 0, 1, 1, need,
                             None) == fic.ERR_INVALID_ARG


def test_capacity_limit(L, hctx):
    """F needs 42 bits at 16x16 ranges; 2^19 or more domains leave fewer than
    the 64 - 42 - 3 bits an index needs. 4x4 and 8x8 searches also need their
    B operand below 2^31 bytes, and every search a work list of at most
    2^32 - 1 items."""
    ok = fic.make_geom(2048, 2048, 16, 4)         # 255,025 domains: 18 bits
    assert _encode(L, hctx, ok, wsb=1 << 40) == fic.ERR_DEVICE
    big = fic.make_geom(8192, 8192, 16, 4)        # 4,182,025 domains: 22 bits
    assert _encode(L, hctx, big, wsb=1 << 40) == fic.ERR_CAPACITY
    b8 = fic.make_geom(4096, 4096, 8, 1)          # 38 + 24 + 3 > 64
    assert _encode(L, hctx, b8, wsb=1 << 40) == fic.ERR_CAPACITY
    # 4x4: the key fits 67M domains, but the B operand (32 bytes a domain) is
    # addressed with 32-bit offsets and must stay below 2^31 bytes
    b4big = fic.make_geom(8200, 8200, 4, 1)       # 67,125,249 domains: 2^31 bytes
    assert _encode(L, hctx, b4big, wsb=1 << 40) == fic.ERR_CAPACITY
    # 66,994,225 domains fit; its work list (262,144 groups x 32,712 chunks
    # of 2048 columns) would not, so it plans wider items (at most 2^26
    # entries where possible, never more than 2^32 - 1)
    b4ok = fic.make_geom(8192, 8192, 4, 1)
    assert _encode(L, hctx, b4ok, wsb=1 << 40) == fic.ERR_DEVICE
    assert L.fic_encode_workspace_bytes(ctypes.byref(b4ok), 0) < 10 << 30


def test_classify_validation(L, hctx):
    g = fic.make_geom(64, 64, 8, 1)
    C = lambda blk, step, img=1, fd=1, gg=g: L.fic_fd_classify(hctx.handle, img, ctypes.byref(gg),
                                                                 blk, step, fd, None, None)
    assert C(16, 1) == fic.ERR_DEVICE
    assert C(12, 1) == fic.ERR_INVALID_ARG
    assert C(16, 0) == fic.ERR_INVALID_ARG
    assert C(16, 1, img=None) == fic.ERR_INVALID_ARG
    assert C(16, 1, fd=None) == fic.ERR_INVALID_ARG
    assert C(32, 1, gg=fic.make_geom(16, 64, 8, 1)) == fic.ERR_INVALID_ARG


def test_pool_validation(L, hctx):
    wsb = L.fic_pool_workspace_bytes(100, 1000)
    P = lambda tol=0.05, nr=100, nd=1000, ws=1, b=wsb, ptr=1: L.fic_build_domain_pool(
        hctx.handle, ptr, nr, ptr, nd, tol, ptr, ptr, ptr, ws, b, None)
    assert P() == fic.ERR_DEVICE
    assert P(tol=float("nan")) == fic.ERR_INVALID_ARG
    assert P(tol=float("inf")) == fic.ERR_DEVICE
    assert P(tol=-1.0) == fic.ERR_DEVICE
    assert P(nr=0) == fic.ERR_INVALID_ARG
    assert P(b=wsb - 1) == fic.ERR_WORKSPACE
    assert P(ptr=None) == fic.ERR_INVALID_ARG


def test_decode_validation(L, hctx):
    g = fic.make_geom(64, 64, 8, 1)
    wsb = L.fic_decode_workspace_bytes(ctypes.byref(g))
    D = lambda it=32, b=wsb, codes=1: L.fic_decode_pifs(hctx.handle, codes, ctypes.byref(g), it,
                                                       None, 1, 1, b, 1, None)
    assert D() == fic.ERR_DEVICE
    assert D(it=-1) == fic.ERR_INVALID_ARG
    assert D(it=100000) == fic.ERR_INVALID_ARG
    assert D(b=wsb - 1) == fic.ERR_WORKSPACE
    assert D(codes=None) == fic.ERR_INVALID_ARG


def test_batch_validation(L, hctx):
    descs = (fic.ImageDesc * 2)()
    for i in range(2):
        descs[i].img = 1
        descs[i].geom = fic.make_geom(128, 128, 4 + 4 * i, 2)
        descs[i].tol = 0.05
        descs[i].codes = 1
    wsb = L.fic_batch_workspace_bytes(2, descs)
    assert wsb > 0
    assert L.fic_encode_pifs_batch(hctx.handle, 2, descs, 1, wsb, None) == fic.ERR_DEVICE
    assert L.fic_encode_pifs_batch(hctx.handle, 2, descs, 1, wsb - 1, None) == fic.ERR_WORKSPACE
    descs[1].tol = float("nan")
    assert L.fic_encode_pifs_batch(hctx.handle, 2, descs, 1, wsb, None) == fic.ERR_INVALID_ARG
    assert L.fic_encode_pifs_batch(hctx.handle, 0, descs, 1, wsb, None) == fic.ERR_INVALID_ARG


def test_batch_workspace_is_sum_of_parts(L):
    """Every image of a batch keeps its own workspace part (all are prepared
    before the shared searches), so the batch needs more than its largest
    image alone, and adding an image adds its part."""
    def descs_of(geoms):
        d = (fic.ImageDesc * len(geoms))()
        for i, g in enumerate(geoms):
            d[i].img = 1
            d[i].geom = g
            d[i].tol = 0.05
            d[i].codes = 1
        return d
    g1, g2 = fic.make_geom(256, 256, 8, 2), fic.make_geom(128, 128, 4, 2)
    one = L.fic_batch_workspace_bytes(1, descs_of([g1]))
    two = L.fic_batch_workspace_bytes(2, descs_of([g1, g2]))
    assert one > L.fic_encode_workspace_bytes(ctypes.byref(g1), 1)
    assert two > one + L.fic_encode_workspace_bytes(ctypes.byref(g2), 1)


def test_batch_graph_switch(L, hctx):
    assert L.fic_set_batch_graph(None, 1) == fic.ERR_INVALID_ARG
    assert L.fic_set_batch_graph(hctx.handle, 0) == fic.OK
    assert L.fic_set_batch_graph(hctx.handle, 1) == fic.OK


def test_workspace_sizes_grow(L):
    a = L.fic_encode_workspace_bytes(ctypes.byref(fic.make_geom(256, 256, 8, 1)), 0)
    b = L.fic_encode_workspace_bytes(ctypes.byref(fic.make_geom(512, 512, 8, 1)), 0)
    assert 0 < a < b
    assert L.fic_encode_workspace_bytes(ctypes.byref(fic.make_geom(30, 30, 8, 1)), 0) == 0


def test_quadtree_validation(L, hctx):
    g1, g2 = fic.make_geom(128, 128, 16, 4), fic.make_geom(128, 128, 8, 2)
    ws = L.fic_quadtree_workspace_bytes(ctypes.byref(g1), 0.05, ctypes.byref(g2), 0.05)
    assert ws > (L.fic_encode_workspace_bytes(ctypes.byref(g1), 1)
                 + L.fic_encode_workspace_bytes(ctypes.byref(g2), 1))

    def E(a=g1, b=g2, rms=8.0, wsb=ws, tol1=0.05, img=1):
        return L.fic_encode_quadtree(hctx.handle, img, ctypes.byref(a), tol1, ctypes.byref(b),
                                     0.05, rms, 1, 1, 1, wsb, None)
    assert E() == fic.ERR_DEVICE
    assert E(rms=float("inf")) == fic.ERR_DEVICE
    assert E(rms=0.0) == fic.ERR_DEVICE
    assert E(rms=-1.0) == fic.ERR_INVALID_ARG
    assert E(rms=float("nan")) == fic.ERR_INVALID_ARG
    assert E(tol1=float("nan")) == fic.ERR_INVALID_ARG
    assert E(wsb=ws - 1) == fic.ERR_WORKSPACE
    assert E(img=None) == fic.ERR_INVALID_ARG
    # level 2 must be the quadrants of level 1 on the same image
    assert E(b=fic.make_geom(128, 128, 4, 2)) == fic.ERR_INVALID_ARG
    assert E(b=fic.make_geom(128, 64, 8, 2)) == fic.ERR_INVALID_ARG
    assert E(a=fic.make_geom(128, 128, 8, 2), b=fic.make_geom(128, 128, 4, 1),
             wsb=1 << 40) == fic.ERR_DEVICE
    assert L.fic_quadtree_workspace_bytes(ctypes.byref(g1), 0.05,
                                          ctypes.byref(fic.make_geom(128, 128, 4, 2)), 0.05) == 0
    dws = L.fic_decode_workspace_bytes(ctypes.byref(g1))

    def D(it=32, wsb=dws, b=g2):
        return L.fic_decode_quadtree(hctx.handle, 1, ctypes.byref(g1), 1, ctypes.byref(b), it,
                                     None, 1, 1, wsb, 1, None)
    assert D() == fic.ERR_DEVICE
    assert D(it=-1) == fic.ERR_INVALID_ARG
    assert D(wsb=dws - 1) == fic.ERR_WORKSPACE
    assert D(b=fic.make_geom(128, 128, 16, 4)) == fic.ERR_INVALID_ARG


def test_pack_validation_and_sizes(L, hctx, oracle_lib):
    import oracle
    g = fic.make_geom(1024, 1024, 8, 1)
    nw = L.fic_packed_words(ctypes.byref(g))
    R, D = oracle.num_ranges(1024, 1024, 8), oracle.num_domains(1024, 1024, 8, 1)
    assert nw == (R * oracle.code_bits(D)[1] + 31) // 32 == (16384 * 35 + 31) // 32
    assert L.fic_pack_codes(hctx.handle, 1, ctypes.byref(g), 1, nw, None) == fic.ERR_DEVICE
    assert L.fic_pack_codes(hctx.handle, 1, ctypes.byref(g), 1, nw - 1, None) == fic.ERR_WORKSPACE
    assert L.fic_pack_codes(hctx.handle, None, ctypes.byref(g), 1, nw, None) == fic.ERR_INVALID_ARG
    assert L.fic_unpack_codes(hctx.handle, 1, nw, ctypes.byref(g), 1, None) == fic.ERR_DEVICE
    assert L.fic_unpack_codes(hctx.handle, 1, nw - 1, ctypes.byref(g), 1, None) == fic.ERR_INVALID_ARG
    assert L.fic_packed_words(ctypes.byref(fic.make_geom(30, 30, 8, 1))) == 0


def test_decode_accepts_twice_size_geometry(L, hctx):
    """16x16 codes decode at twice the size with 32x32 ranges; the encoder
    does not take 32x32 ranges."""
    g32 = fic.make_geom(256, 256, 32, 8)
    ws = L.fic_decode_workspace_bytes(ctypes.byref(g32))
    assert ws > 0
    assert L.fic_decode_pifs(hctx.handle, 1, ctypes.byref(g32), 8, None, 1, 1, ws, 1,
                             None) == fic.ERR_DEVICE
    assert L.fic_encode_workspace_bytes(ctypes.byref(g32), 0) == 0
    assert L.fic_decode_workspace_bytes(ctypes.byref(fic.make_geom(32, 32, 32, 8))) == 0


def test_color_validation(L, hctx):
    g = fic.make_geom(128, 96, 8, 2, pitch=3 * 96)
    ws = L.fic_color_workspace_bytes(ctypes.byref(g), 0.05)
    assert ws > 0

    def C(gg=g, src=0, wsb=ws, tol=0.05):
        return L.fic_encode_color(hctx.handle, 1, ctypes.byref(gg), tol, src, 1, 1, 1, 1, wsb, None)
    assert C() == fic.ERR_DEVICE
    assert C(src=1) == fic.ERR_DEVICE
    assert C(src=2) == fic.ERR_INVALID_ARG
    assert C(wsb=ws - 1) == fic.ERR_WORKSPACE
    assert C(tol=float("nan")) == fic.ERR_INVALID_ARG
    assert C(gg=fic.make_geom(128, 96, 8, 2, pitch=96)) == fic.ERR_INVALID_ARG   # not 3 bytes a pixel
    assert L.fic_color_workspace_bytes(ctypes.byref(fic.make_geom(128, 96, 8, 2, pitch=200)), 0.05) == 0


def test_debug_switch_validation(L, hctx):
    assert L.fic_set_debug(hctx.handle, 0) == fic.OK
    assert L.fic_set_debug(hctx.handle, fic.DEBUG_REVERSE_ITEMS | fic.DEBUG_VERIFY16) == fic.OK
    assert L.fic_set_debug(hctx.handle, fic.DEBUG_SEPARATE_SEARCHES) == fic.OK
    assert L.fic_set_debug(hctx.handle, 8) == fic.ERR_INVALID_ARG
    assert L.fic_set_debug(None, 0) == fic.ERR_INVALID_ARG
    assert L.fic_set_debug(hctx.handle, 0) == fic.OK


def _tune_file(path, arch, khash, rows, xcd=None, batch_separate=None):
    import json
    doc = {"format": "fic-tune-1", "arch": arch, "kernel_hash": khash,
           "rows": [dict({"range_size": b, "dlog2": dl, "chunk_log2": cl, "flush_at": fl},
                         **({"xcd": xcd} if xcd is not None else {}))
                    for b, dl, cl, fl in rows]}
    if batch_separate is not None:
        doc["batch_separate"] = batch_separate
    with open(path, "w") as f:
        json.dump(doc, f)


def test_tune_defaults_and_bucket_rule(L, tmp_path):
    """Defaults: exhaustive items 2^14 columns, pooled 2^12, early flush 64
    at 8x8 only. A loaded row is used per pool-fraction bucket: 0 for
    exhaustive, 1 for f >= 1/2, 2 for [1/4, 1/2), ... 5 below 1/16."""
    c = fic.Context(-1)
    try:
        assert c.tune_query(1024, 1024, 8, 1) == (14, 64)
        assert c.tune_query(1024, 1024, 8, 1, pooled=True, pool_fraction=0.3) == (12, 64)
        assert c.tune_query(512, 512, 4, 2, pooled=True, pool_fraction=0.3) == (12, 0)
        assert c.tune_query(2048, 2048, 16, 4) == (14, 0)
        g = fic.make_geom(1024, 1024, 8, 1)
        dl = int(L.fic_num_domains(ctypes.byref(g))).bit_length() - 1     # floor(log2 D)
        p = str(tmp_path / "t.json")
        _tune_file(p, "none", fic.kernel_hash(),
                   [(8, dl, [11, 12, 13, 14, 15, 16], [0, 32, 64, 128, 192, 256])])
        assert c.tune_load(p) == fic.OK
        q = lambda f: c.tune_query(1024, 1024, 8, 1, pooled=True, pool_fraction=f)
        assert c.tune_query(1024, 1024, 8, 1) == (11, 0)
        assert q(1.0) == (12, 32) and q(0.5) == (12, 32)
        assert q(0.4999) == (13, 64) and q(0.25) == (13, 64)
        assert q(0.2499) == (14, 128) and q(0.125) == (14, 128)
        assert q(0.1249) == (15, 192) and q(0.0625) == (15, 192)
        assert q(0.0624) == (16, 256) and q(0.0) == (16, 256)
        # another lattice class keeps the defaults
        assert c.tune_query(512, 512, 8, 1) == (14, 64)
        assert c.tune_query(1024, 1024, 8, 1, with_xcd=True) == (11, 0, 0)   # no "xcd": 0
        _tune_file(p, "none", fic.kernel_hash(),
                   [(8, dl, [11, 12, 13, 14, 15, 16], [0, 32, 64, 128, 192, 256])],
                   xcd=[1, 0, 1, 0, 1, 0])
        assert c.tune_load(p) == fic.OK
        assert c.tune_query(1024, 1024, 8, 1, with_xcd=True) == (11, 0, 1)
        assert c.tune_query(1024, 1024, 8, 1, pooled=True, pool_fraction=0.3,
                            with_xcd=True) == (13, 64, 1)
        # save -> reset -> load round trip
        p2 = str(tmp_path / "t2.json")
        c.tune_save(p2)
        c.tune_reset()
        assert c.tune_query(1024, 1024, 8, 1) == (14, 64)
        assert c.tune_load(p2) == fic.OK
        assert q(0.3) == (13, 64)
    finally:
        c.close()


def test_tune_cache_rejections(L, tmp_path):
    c = fic.Context(-1)
    try:
        row = [(8, 20, [12] * 6, [64] * 6)]
        p = str(tmp_path / "a.json")
        _tune_file(p, "gfx942", fic.kernel_hash(), row)
        assert c.tune_load(p) == fic.ERR_UNSUPPORTED              # another architecture
        _tune_file(p, "none", "0000000000000000", row)
        assert c.tune_load(p) == fic.ERR_UNSUPPORTED              # other kernels
        _tune_file(p, "none", fic.kernel_hash(), [(8, 20, [10] * 6, [64] * 6)])
        assert c.tune_load(p) == fic.ERR_INVALID_ARG              # item width out of range
        _tune_file(p, "none", fic.kernel_hash(), [(6, 20, [12] * 6, [64] * 6)])
        assert c.tune_load(p) == fic.ERR_INVALID_ARG              # range size
        _tune_file(p, "none", fic.kernel_hash(), [(8, 20, [12] * 6, [64] * 6)], xcd=[2] * 6)
        assert c.tune_load(p) == fic.ERR_INVALID_ARG              # xcd is 0 or 1
        _tune_file(p, "none", fic.kernel_hash(), row, batch_separate=2)
        assert c.tune_load(p) == fic.ERR_INVALID_ARG              # batch_separate is 0 or 1
        with open(p, "w") as f:
            f.write("not json")
        assert c.tune_load(p) == fic.ERR_INVALID_ARG
        assert c.tune_load(str(tmp_path / "missing.json")) == fic.ERR_INVALID_ARG
        assert c.tune_query(1024, 1024, 8, 1) == (14, 64)          # unchanged
    finally:
        c.close()


def test_tune_cache_keeps_the_batch_launch_choice(L, tmp_path):
    """The batch launch structure (one combined search or one per range
    size) is saved with the rows and restored by a load; absent means
    combined."""
    import json
    c = fic.Context(-1)
    try:
        p, q = str(tmp_path / "in.json"), str(tmp_path / "out.json")
        row = [(8, 20, [12] * 6, [64] * 6)]
        c.tune_save(q)
        assert json.load(open(q))["batch_separate"] == 0          # default
        _tune_file(p, "none", fic.kernel_hash(), row, batch_separate=1)
        assert c.tune_load(p) == fic.OK
        c.tune_save(q)
        doc = json.load(open(q))
        assert doc["batch_separate"] == 1 and doc["rows"][0]["chunk_log2"] == [12] * 6
        _tune_file(p, "none", fic.kernel_hash(), row)               # absent: combined
        assert c.tune_load(p) == fic.OK
        c.tune_save(q)
        assert json.load(open(q))["batch_separate"] == 0
        _tune_file(p, "none", fic.kernel_hash(), row, batch_separate=1)
        assert c.tune_load(p) == fic.OK
        c.tune_reset()
        c.tune_save(q)
        assert json.load(open(q))["batch_separate"] == 0
    finally:
        c.close()


def test_autotune_validation(L, hctx):
    descs = (fic.ImageDesc * 2)()
    for i in range(2):
        descs[i].img = 1
        descs[i].geom = fic.make_geom(128, 128, 4 + 4 * i, 2)
        descs[i].tol = 0.05
        descs[i].codes = 1
    wsb = L.fic_autotune_workspace_bytes(2, descs)
    assert 0 < wsb < L.fic_batch_workspace_bytes(2, descs)
    cnt = ctypes.c_int32(-1)
    rep = (fic.TuneEntry * 2)()
    A = lambda n=2, ws=wsb, reps=2, r=rep, cap=2: L.fic_autotune(
        hctx.handle, n, descs, 1, ws, reps, r, cap, ctypes.byref(cnt), None)
    assert A() == fic.ERR_DEVICE
    assert A(ws=wsb - 1) == fic.ERR_WORKSPACE
    assert A(reps=0) == fic.ERR_INVALID_ARG
    assert A(n=0) == fic.ERR_INVALID_ARG
    assert A(r=None, cap=2) == fic.ERR_INVALID_ARG
    assert A(r=None, cap=0) == fic.ERR_DEVICE
    descs[0].tol = float("nan")
    assert A() == fic.ERR_INVALID_ARG


def test_noalloc_validation(L, hctx):
    """The no-allocation encode validates like fic_encode_pifs and rejects
    geometries whose workspace exceeds its static scratch."""
    lim = L.fic_noalloc_scratch_bytes()
    assert lim == 64 << 20
    N = lambda g, perm=None, lo=None, hi=None, kernel=0, img=1, codes=1: L.fic_encode_pifs_noalloc(
        hctx.handle, img, ctypes.byref(g), perm, lo, hi, kernel, codes, None)
    small = fic.make_geom(512, 512, 8, 1)
    big = fic.make_geom(1024, 1024, 8, 1)
    assert L.fic_encode_workspace_bytes(ctypes.byref(small), 1) <= lim
    assert L.fic_encode_workspace_bytes(ctypes.byref(big), 0) > lim
    assert N(small) == fic.ERR_DEVICE                        # valid, no device
    assert N(small, perm=1, lo=1, hi=1) == fic.ERR_DEVICE
    assert N(big) == fic.ERR_WORKSPACE
    assert N(small, perm=1) == fic.ERR_INVALID_ARG
    assert N(small, kernel=3) == fic.ERR_INVALID_ARG
    assert N(small, img=None) == fic.ERR_INVALID_ARG
    assert N(fic.make_geom(60, 64, 8, 1)) == fic.ERR_INVALID_ARG
    assert N(fic.make_geom(8192, 8192, 16, 4)) == fic.ERR_CAPACITY
