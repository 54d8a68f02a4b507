"""GPU tests of the autotuned search parameters and the combined batch launch.

Every (columns per work item, early flush trigger) candidate the autotuner
may pick must give the same codes (only the schedule changes); the
autotuner's choices are stored, saved and loaded; a batch's single combined
4x4 + 8x8 launch equals one launch per range size.
"""
import json

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


def dev(img):
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


def _cases():
    from synth import workload_images
    from test_gpu_parity import SMALL, small_image
    out = [(name, small_image(name, make), b, t, tol) for name, make, b, t, tol in SMALL]
    img = workload_images("fbm512rect_b8t2")
    out += [("fbm512rect 8/2 exhaustive", img, 8, 2, None), ("fbm512rect 8/2 pool", img, 8, 2, 0.05)]
    return out


def _codes(fic, cases):
    out = []
    for _, img, b, t, tol in cases:
        c, _ = fic.encode(dev(img), b, t, tol=tol)
        out.append(c.cpu().numpy())
    torch.cuda.synchronize()
    return out


def _write_rows(path, chunk_log2, flush_at, xcd=0):
    arch = torch.cuda.get_device_properties(0).gcnArchName
    import paper_1206_4880_amd as p
    rows = [{"range_size": b, "dlog2": dl, "chunk_log2": [chunk_log2] * 6,
             "flush_at": [flush_at] * 6, "xcd": [xcd] * 6}
            for b in (4, 8, 16) for dl in range(0, 31)]
    with open(path, "w") as f:
        json.dump({"format": "fic-tune-1", "arch": arch, "kernel_hash": p.fic.kernel_hash(),
                   "rows": rows}, f)


def test_codes_identical_under_every_candidate(fic, tmp_path):
    cases = _cases()
    ctx = fic.fic.context()
    ctx.tune_reset()
    ref = _codes(fic, cases)
    path = str(tmp_path / "cand.json")
    try:
        for cl in range(11, 17):
            for fl in (0, 16, 32, 128):
                for xc in (0, 1):
                    _write_rows(path, cl, fl, xc)
                    assert ctx.tune_load(path) == fic.fic.OK
                    assert ctx.tune_query(512, 512, 8, 2, with_xcd=True) == (cl, fl, xc)
                    got = _codes(fic, cases)
                    for (name, *_), a, b in zip(cases, ref, got):
                        assert np.array_equal(a, b), "%s, chunk 2^%d, flush %d, xcd %d" % (
                            name, cl, fl, xc)
    finally:
        ctx.tune_reset()


def test_autotune_then_cache_round_trip(fic, tmp_path):
    from synth import batch_descs, workload_images
    img = workload_images("fbm512rect_b8t2")
    items = batch_descs(count=4, base_seed=4200)
    images = [dev(img), dev(img)] + [dev(im) for (im, _, _, _) in items]
    jobs = [(8, 2, None), (8, 2, 0.05)] + [(b, t, tol) for (_, b, t, tol) in items]
    ctx = fic.fic.context()
    ctx.tune_reset()
    before = []
    for x, (b, t, tol) in zip(images, jobs):
        c, _ = fic.encode(x, b, t, tol=tol)
        before.append(c.cpu().numpy())
    try:
        rep = fic.fic.autotune(images, jobs, reps=1)
        assert rep, "no tuning classes"
        launch = [r for r in rep if r["range_size"] == 0]
        rep = [r for r in rep if r["range_size"] != 0]
        if {b for b, _, _ in jobs} >= {4, 8}:
            assert len(launch) == 1 and launch[0]["flush_at"] in (0, 1)
            assert launch[0]["tuned_ms"] <= launch[0]["base_ms"]
        for r in rep:
            assert 11 <= r["chunk_log2"] <= 16 and r["flush_at"] in (0, 16, 32, 64, 128)
            assert r["xcd"] in (0, 1)
            assert r["tuned_ms"] <= r["base_ms"]
            print("B=%d log2 D=%d bucket %d (%d images): chunk 2^%d flush %d, %.3f -> %.3f ms"
                  % (r["range_size"], r["dlog2"], r["bucket"], r["images"], r["chunk_log2"],
                     r["flush_at"], r["base_ms"], r["tuned_ms"]))
        for x, (b, t, tol), want in zip(images, jobs, before):
            c, _ = fic.encode(x, b, t, tol=tol)
            assert np.array_equal(c.cpu().numpy(), want)
        # the batch, with whatever launch structure was kept, equals them too
        outs = fic.encode_batch(images, jobs, graph=True)
        for c, want in zip(outs, before):
            assert np.array_equal(c.cpu().numpy(), want)
        # the exhaustive class answers with its chosen row; save, reset, load
        q = ctx.tune_query(512, 512, 8, 2)
        path = str(tmp_path / "tuned.json")
        ctx.tune_save(path)
        ctx.tune_reset()
        assert ctx.tune_query(512, 512, 8, 2) == (14, 64)
        assert ctx.tune_load(path) == fic.fic.OK
        assert ctx.tune_query(512, 512, 8, 2) == q
        doc = json.load(open(path))
        assert doc["kernel_hash"] == fic.fic.kernel_hash()
    finally:
        ctx.tune_reset()


def test_batch_combined_launch_equals_separate(fic):
    """The 64-image batch: one combined 4x4 + 8x8 launch and one launch per
    range size give the same codes."""
    from synth import batch_descs
    items = batch_descs(count=64)
    imgs = [dev(im) for (im, _, _, _) in items]
    jobs = [(b, t, tol) for (_, b, t, tol) in items]
    assert {b for b, _, _ in jobs} == {4, 8}
    comb = [c.cpu().numpy() for c in fic.encode_batch(imgs, jobs, graph=False)]
    ctx = fic.fic.context()
    ctx.set_debug(fic.fic.DEBUG_SEPARATE_SEARCHES)
    try:
        sep = [c.cpu().numpy() for c in fic.encode_batch(imgs, jobs, graph=False)]
    finally:
        ctx.set_debug(0)
    for m, (a, b) in enumerate(zip(comb, sep)):
        assert np.array_equal(a, b), "image %d" % m
