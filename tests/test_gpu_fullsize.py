"""GPU parity on EVERY range of the full-size workloads.

The oracle's codes for these jobs take hours of CPU time, so they are stored
as SHA-256 digests per block of 1024 ranges in tests/golden/config_digests.json
(written by tests/golden/make_digests.py, which calls only the oracle and the
seeded image generators). Each test encodes the job on the GPU through the C
ABI and compares every block digest; on a mismatch it names the block and
compares that block range by range with the oracle.

Also here: both kernels (MFMA and plain) on every job; the work list consumed
in reverse order (the packed-key minimum must not depend on it); the pool
sets of every range against the oracle's window (Sec. 3.1); the rounding
bound of the 16x16 one-accumulator screen checked on the matrix cores; the
two-level 2048^2 encode against the digest-checked single-level codes.
"""
import hashlib
import importlib.util
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
DIGESTS = os.path.join(HERE, "golden", "config_digests.json")


def _maker():
    spec = importlib.util.spec_from_file_location("make_digests",
                                                  os.path.join(HERE, "golden", "make_digests.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


MK = _maker()


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


@pytest.fixture(scope="module")
def golden():
    with open(DIGESTS) as f:
        doc = json.load(f)
    with open(os.path.join(os.path.dirname(HERE), "oracle", "fic_oracle.c"), "rb") as f:
        assert doc["oracle_sha256"] == hashlib.sha256(f.read()).hexdigest(), \
            "digests were written by another oracle source: rerun tests/golden/make_digests.py"
    return doc


def dev(img):
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


def fields(codes_np):
    """The digest fields of a GPU code array (structured, fic_code layout)."""
    return {"dom": codes_np["domain"], "iso": codes_np["iso"], "k": codes_np["s_idx"],
            "j": codes_np["o_idx"], "flags": codes_np["flags"], "err": codes_np["err"]}


def check_digests(orc, rec, img, got, what):
    """Every finished block of the job record against the GPU codes; the
    number of ranges checked."""
    from synth import image_sha256
    assert rec["image_sha256"] == image_sha256(img), what + ": image differs from the digests'"
    R = rec["ranges"]
    assert got.size == R
    assert not np.any(got["flags"] & 0x80), what + ": a code failed its internal check (bit 7)"
    f = fields(got)
    for blk, want in enumerate(rec["blocks"]):
        a, b = blk * MK.BLOCK, min(R, (blk + 1) * MK.BLOCK)
        part = {k: v[a:b] for k, v in f.items()}
        if MK.block_digest(part) == want:
            continue
        sel = np.arange(a, b, dtype=np.int64)
        ref = orc.encode(img, rec["b"], rec["t"], tol=rec["tol"], sel=sel)
        for k in MK.FIELDS:
            x = np.asarray(part[k]).astype(np.int64)
            y = np.asarray(ref[k]).astype(np.int64)
            bad = np.flatnonzero(x != y)
            if bad.size:
                raise AssertionError("%s: block %d (ranges %d..%d), field %s differs at ranges %s: "
                                     "gpu %s oracle %s" % (what, blk, a, b - 1, k, a + bad[:5],
                                                           x[bad[:5]], y[bad[:5]]))
        raise AssertionError("%s: block %d digest differs but no field does" % (what, blk))
    return min(R, len(rec["blocks"]) * MK.BLOCK)


def job_record(golden, jid):
    """The job's digest record; the committed file covers every range of
    every full-size job."""
    rec = golden["jobs"].get(jid)
    assert rec is not None and rec.get("complete"), "no complete oracle digests for " + jid
    return rec


SINGLE = [("fbm512rect_b8t2", 8, 2, None), ("fbm512rect_b8t2", 8, 2, 0.05),
          ("fbm1024_b8t1", 8, 1, None), ("fbm1024_b8t1", 8, 1, 0.02),
          ("fbm1024_b8t1", 8, 1, 0.1), ("fbm2048_twolevel", 16, 4, 0.05),
          ("fbm2048_twolevel", 8, 2, 0.05), ("fbm2048_twolevel", 16, 4, None)]


def jid_of(name, b, t, tol):
    return "%s/%d_%d_%s" % (name, b, t, MK._tol_name(tol))


def gpu_codes(fic, img, b, t, tol, kernel="mfma"):
    c, _ = fic.encode(dev(img), b, t, tol=tol, kernel=kernel)
    torch.cuda.synchronize()
    return fic.unpack_codes(c)


@pytest.mark.parametrize("job", SINGLE, ids=[jid_of(*j) for j in SINGLE])
@pytest.mark.parametrize("kernel", ["mfma", "plain"])
def test_every_range_against_oracle(fic, orc, golden, job, kernel):
    from synth import workload_images
    name, b, t, tol = job
    rec = job_record(golden, jid_of(*job))
    img = workload_images(name)
    got = gpu_codes(fic, img, b, t, tol, kernel)
    n = check_digests(orc, rec, img, got, "%s %s" % (jid_of(*job), kernel))
    print("%s %s: %d of %d ranges bit-exact" % (jid_of(*job), kernel, n, rec["ranges"]))


@pytest.mark.parametrize("job", [("fbm1024_b8t1", 8, 1, 0.02), ("fbm1024_b8t1", 8, 1, None),
                                 ("fbm2048_twolevel", 8, 2, 0.05),
                                 ("fbm2048_twolevel", 16, 4, 0.05)],
                         ids=lambda j: jid_of(*j))
def test_reverse_item_order(fic, orc, golden, job):
    """The persistent search taking its work items last to first gives the
    same codes (order independence of the packed-key minimum)."""
    from synth import workload_images
    name, b, t, tol = job
    img = workload_images(name)
    fwd = gpu_codes(fic, img, b, t, tol)
    ctx = fic.fic.context()
    ctx.set_debug(fic.fic.DEBUG_REVERSE_ITEMS)
    try:
        rev = gpu_codes(fic, img, b, t, tol)
    finally:
        ctx.set_debug(0)
    for f in fwd.dtype.names:
        assert np.array_equal(fwd[f], rev[f]), f
    check_digests(orc, job_record(golden, jid_of(*job)), img, rev, jid_of(*job) + " reversed")


@pytest.mark.parametrize("chunk_log2", [13, 16])
def test_xcd_queues_every_range(fic, orc, golden, tmp_path, chunk_log2):
    """Single-image searches taking their items from one queue per XCD (with
    stealing), at two item widths, on the 1024^2 jobs and the 2048^2 8x8
    job: every range equals the oracle digests."""
    from synth import workload_images
    ctx = fic.fic.context()
    arch = torch.cuda.get_device_properties(0).gcnArchName
    path = str(tmp_path / "xcd.json")
    rows = [{"range_size": b, "dlog2": dl, "chunk_log2": [chunk_log2] * 6, "flush_at": [64] * 6,
             "xcd": [1] * 6} for b in (4, 8, 16) for dl in range(0, 31)]
    with open(path, "w") as f:
        json.dump({"format": "fic-tune-1", "arch": arch, "kernel_hash": fic.fic.kernel_hash(),
                   "rows": rows}, f)
    assert ctx.tune_load(path) == fic.fic.OK
    try:
        for job in [("fbm1024_b8t1", 8, 1, None), ("fbm1024_b8t1", 8, 1, 0.02),
                    ("fbm1024_b8t1", 8, 1, 0.1), ("fbm2048_twolevel", 8, 2, 0.05),
                    ("fbm2048_twolevel", 16, 4, 0.05)]:
            rec = job_record(golden, jid_of(*job))
            img = workload_images(job[0])
            got = gpu_codes(fic, img, *job[1:])
            check_digests(orc, rec, img, got, jid_of(*job) + " xcd queues")
    finally:
        ctx.tune_reset()


def test_batch64_every_range(fic, orc, golden):
    """The 64-image mixed batch in one call (graph): every image's codes
    against its oracle digests; then the same batch with the work items
    reversed gives the same codes."""
    from synth import batch_descs
    items = batch_descs(count=64)
    imgs = [dev(im) for (im, _, _, _) in items]
    jobs = [(b, t, tol) for (_, b, t, tol) in items]
    outs = fic.encode_batch(imgs, jobs, graph=True)
    torch.cuda.synchronize()
    got = [fic.unpack_codes(c) for c in outs]
    checked = 0
    total = 0
    for m, ((im, b, t, tol), g) in enumerate(zip(items, got)):
        jid = "batch64_mixed/%02d_%d_%d_%s" % (m, b, t, MK._tol_name(tol))
        total += g.size
        assert not np.any(g["flags"] & 0x80)
        checked += check_digests(orc, job_record(golden, jid), im, g, jid)
    print("batch64: %d of %d ranges checked against the oracle digests" % (checked, total))
    # the committed digests cover every range of every image
    assert checked == total, "the digests cover %d of %d ranges" % (checked, total)
    ctx = fic.fic.context()
    ctx.set_debug(fic.fic.DEBUG_REVERSE_ITEMS)
    try:
        rev = fic.encode_batch(imgs, jobs, graph=True)
        torch.cuda.synchronize()
    finally:
        ctx.set_debug(0)
    for m, (a, c) in enumerate(zip(got, rev)):
        assert np.array_equal(a, fic.unpack_codes(c)), "image %d reversed" % m


def test_quadtree_2048_every_range(fic, golden, orc):
    """The two-level 2048^2 encode equals the digest-checked single-level
    codes: level 1 is the 16/4 job with split flags from its own E, every
    coded level-2 range is the 8/2 job's code for that range."""
    from synth import WORKLOADS, workload_images
    wl = WORKLOADS["fbm2048_quadtree"]
    img = workload_images("fbm2048_quadtree")
    j1, j2 = ("fbm2048_twolevel", 16, 4, 0.05), ("fbm2048_twolevel", 8, 2, 0.05)
    r1, r2 = job_record(golden, jid_of(*j1)), job_record(golden, jid_of(*j2))
    s1, s2 = gpu_codes(fic, img, 16, 4, 0.05), gpu_codes(fic, img, 8, 2, 0.05)
    check_digests(orc, r1, img, s1, "quadtree level-1 reference")
    check_digests(orc, r2, img, s2, "quadtree level-2 reference")
    c1, c2 = fic.encode_quadtree(dev(img), 16, 4, 0.05, 8, 2, 0.05, wl.rms)
    torch.cuda.synchronize()
    g1, g2 = fic.unpack_codes(c1), fic.unpack_codes(c2)
    split = s1["err"] > orc.split_threshold(16, wl.rms)
    assert np.array_equal((g1["flags"] & 2) != 0, split)
    for f in ("domain", "iso", "s_idx", "o_idx", "err"):
        assert np.array_equal(g1[f], s1[f]), f
    assert np.array_equal(g1["flags"] & np.uint8(0xFD), s1["flags"])
    coded = (g2["flags"] & 4) == 0
    rc1, rc2 = 2048 // 16, 2048 // 8
    r = np.arange(g2.size)
    assert np.array_equal(coded, split[(r // rc2 // 2) * rc1 + (r % rc2) // 2])
    for f in ("domain", "iso", "s_idx", "o_idx", "err", "flags"):
        assert np.array_equal(g2[f][coded], s2[f][coded]), f


# ------------------------------------------------------------ pool sets
def window_bounds(sorted_vals, fd_r, edge):
    """Per range, [lo, hi) of the sorted values v with |v - fd_r| <= edge,
    found by bisection on that predicate itself (fp64, the oracle's
    rule): the set is contiguous because fp64 subtraction is monotone."""
    n = sorted_vals.size
    R = fd_r.size

    def first(pred):
        lo = np.zeros(R, dtype=np.int64)
        hi = np.full(R, n, dtype=np.int64)
        while np.any(lo < hi):
            mid = (lo + hi) // 2
            ok = pred(sorted_vals[np.minimum(mid, n - 1)]) & (lo < hi)
            hi = np.where(ok, mid, hi)
            lo = np.where(~ok & (lo < hi), mid + 1, lo)
        return lo
    # left end: first v with v >= fd_r - ... i.e. not (v < fd_r and fd_r - v > edge)
    a = first(lambda v: ~((v < fd_r) & (np.abs(v - fd_r) > edge)))
    b = first(lambda v: (v > fd_r) & (np.abs(v - fd_r) > edge))
    return a, b


def check_pool_all(perm, lo, hi, fd_r, fd_d, tol_eff, gpu_fd_d):
    """perm sorts the GPU's own values stably, and for EVERY range the set
    perm[lo:hi] equals {d : |fd_d - fd_r| <= tol + 1e-9} over the oracle's
    values. Sets are compared by their sizes and by sums of random 64-bit
    weights of their members (prefix sums along each order, wrapping)."""
    perm = perm.cpu().numpy().astype(np.int64)
    lo = lo.cpu().numpy().astype(np.int64)
    hi = hi.cpu().numpy().astype(np.int64)
    D = fd_d.size
    assert np.array_equal(np.sort(perm), np.arange(D))
    vals = gpu_fd_d[perm]
    assert np.all(np.diff(vals) >= 0)
    eq = np.diff(vals) == 0
    assert np.all(np.diff(perm)[eq] > 0)
    order = np.argsort(fd_d, kind="stable")
    a, b = window_bounds(fd_d[order], fd_r, tol_eff + 1e-9)
    assert np.array_equal(hi - lo, b - a), "pool sizes differ"
    w = np.random.default_rng(7).integers(0, 2**63, size=D, dtype=np.int64).astype(np.uint64)
    with np.errstate(over="ignore"):
        pg = np.concatenate([[np.uint64(0)], np.cumsum(w[perm], dtype=np.uint64)])
        po = np.concatenate([[np.uint64(0)], np.cumsum(w[order], dtype=np.uint64)])
        hg = pg[hi] - pg[lo]
        ho = po[b] - po[a]
    bad = np.flatnonzero(hg != ho)
    if bad.size:
        r = int(bad[0])
        want = np.flatnonzero(np.abs(fd_d - fd_r[r]) <= tol_eff + 1e-9)
        raise AssertionError("pool of range %d differs: gpu %d members, oracle %d"
                             % (r, hi[r] - lo[r], want.size))
    return int((hi - lo).sum())


@pytest.mark.parametrize("job", [("fbm512rect_b8t2", 8, 2, 0.05), ("fbm1024_b8t1", 8, 1, 0.02),
                                 ("fbm1024_b8t1", 8, 1, 0.1), ("fbm2048_twolevel", 16, 4, 0.05),
                                 ("fbm2048_twolevel", 8, 2, 0.05)],
                         ids=lambda j: jid_of(*j))
def test_pool_sets_every_range(fic, orc, job):
    from synth import workload_images
    name, b, t, tol = job
    img = workload_images(name)
    x = dev(img)
    fr_t, _ = fic.fd_classify(x, b, b, want_fp32=False)
    fd_t, _ = fic.fd_classify(x, 2 * b, t, want_fp32=False)
    perm, lo, hi = fic.build_domain_pool(fr_t, fd_t, tol)
    torch.cuda.synchronize()
    fr, fd = orc.classify(img, b, t)
    assert np.max(np.abs(fd_t.cpu().numpy() - fd)) < 1e-12
    tol_eff = orc.resolve_tol(tol, fd)
    assert orc.pool_margin(fr, fd, tol_eff) > 1e-11
    members = check_pool_all(perm, lo, hi, fr, fd, tol_eff, fd_t.cpu().numpy())
    print("%s: %d ranges, %d pool members, sets equal" % (jid_of(*job), fr.size, members))


# ------------------------------------------------ 16x16 rounding bound
@pytest.mark.parametrize("case", [
    ("binary 128 16/1", None, 16, 1, None),
    ("binary 128 16/2 pool", None, 16, 2, 0.05),
    ("fbm2048 16/4", "fbm2048_twolevel", 16, 4, None),
    ("fbm2048 16/4 pool", "fbm2048_twolevel", 16, 4, 0.05)], ids=lambda c: c[0])
def test_verify16_rounding_bound(fic, case):
    """With the verify switch the 16x16 search recomputes every screened
    block's exact chunk sums and checks the error of its one-accumulator
    FP32 sums against the bound the screen threshold is lowered by: no sum
    may exceed it. Codes do not change."""
    name, wl, b, t, tol = case
    if wl is None:
        seed = 31 if t == 1 else 32
        img = (np.random.default_rng(seed).integers(0, 2, (128, 128)) * 255).astype(np.uint8)
    else:
        from synth import workload_images
        img = workload_images(wl)
    plain = gpu_codes(fic, img, b, t, tol)
    ctx = fic.fic.context()
    cnt = torch.zeros(8, dtype=torch.int64, device="cuda")
    ctx.set_counters(cnt)
    ctx.set_debug(fic.fic.DEBUG_VERIFY16)
    try:
        ver = gpu_codes(fic, img, b, t, tol)
    finally:
        ctx.set_debug(0)
        ctx.set_counters(None)
    c = cnt.cpu().numpy()
    print("%s: %d sums checked, %d over the bound, largest error/bound %.3g"
          % (name, c[5], c[4], c[6] / 2.0**20))
    assert c[5] > 0
    assert c[4] == 0
    for f in plain.dtype.names:
        assert np.array_equal(plain[f], ver[f]), f
