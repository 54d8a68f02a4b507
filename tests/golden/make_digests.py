"""Write tests/golden/config_digests.json: SHA-256 digests of the oracle's
codes for EVERY range of the full-size workloads, in blocks of 1024 ranges
(ranges in raster order), so that the GPU tests can check whole jobs code for
code without running the oracle themselves (it takes hours at these sizes).

Calls only ``oracle`` (the CPU oracle) and ``synth`` (the seeded images); it
never loads the GPU library. Per job it also records the image's SHA-256, the
resolved tolerance, the pair evaluations (sum of pool sizes times 8), and for
pooled jobs the smallest distance of any |fd_d - fd_r| from the window edge
tol + 1e-9 (oracle.pool_margin): how far the closest membership decision of
the Sec. 3.1 window is from flipping.

Resumable: the file is rewritten after every block, and a job whose image,
parameters and oracle source are unchanged continues after its last finished
block. cfg-sized oracle runs take hours on a few cores; run it in the
background:

    nice -n 19 python tests/golden/make_digests.py [--only REGEX] [--threads N]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "config_digests.json")
BLOCK = 1024
FIELDS = ("dom", "iso", "k", "j", "flags", "err")


def block_digest(fields):
    """SHA-256 of one block's codes: each field of FIELDS in turn, as
    little-endian int64 values, ranges in raster order."""
    h = hashlib.sha256()
    for f in FIELDS:
        h.update(np.ascontiguousarray(np.asarray(fields[f]).astype("<i8")).tobytes())
    return h.hexdigest()


def oracle_sha256():
    with open(os.path.join(ROOT, "oracle", "fic_oracle.c"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _tol_name(tol):
    return "exhaustive" if tol is None else ("adaptive" if tol < 0 else "pool_%g" % tol)


def job_list():
    """(job id, image loader, B, t, tol) of every full-size job: the 512^2,
    1024^2 and 2048^2 workloads and each image of the 64-image batch, roughly
    cheapest first (the batch's 8x8 images before its 4x4 ones)."""
    from synth import batch_descs, workload_images
    batch = {}

    def batch_img(m):
        if not batch:
            for i, item in enumerate(batch_descs(count=64)):
                batch[i] = item
        return batch[m][0]

    def single(name, b, t, tol):
        return ("%s/%d_%d_%s" % (name, b, t, _tol_name(tol)),
                (lambda n=name: workload_images(n)), b, t, tol)

    jobs = [single("fbm512rect_b8t2", 8, 2, None), single("fbm512rect_b8t2", 8, 2, 0.05),
            single("fbm1024_b8t1", 8, 1, 0.02), single("fbm2048_twolevel", 16, 4, 0.05),
            single("fbm1024_b8t1", 8, 1, 0.1), single("fbm1024_b8t1", 8, 1, None),
            single("fbm2048_twolevel", 16, 4, None), single("fbm2048_twolevel", 8, 2, 0.05)]
    descs = [(m, b, t, tol, img.shape[0]) for m, (img, b, t, tol) in enumerate(batch_descs(count=64))]
    for m, b, t, tol, size in sorted(descs, key=lambda x: (-x[1], x[4], x[0])):
        jobs.append(("batch64_mixed/%02d_%d_%d_%s" % (m, b, t, _tol_name(tol)),
                     (lambda m=m: batch_img(m)), b, t, tol))
    return jobs


def load():
    try:
        with open(OUT) as f:
            return json.load(f)
    except (OSError, ValueError):
        return None


def save(doc):
    tmp = OUT + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, OUT)


def run(only=None, threads=0):
    import oracle
    from synth import image_sha256
    oracle.build(force=False)
    osha = oracle_sha256()
    doc = load()
    if not doc or doc.get("oracle_sha256") != osha or doc.get("block") != BLOCK:
        doc = {"oracle_sha256": osha, "block": BLOCK, "fields": list(FIELDS), "jobs": {}}
    for jid, loader, b, t, tol in job_list():
        if only and not re.search(only, jid):
            continue
        img = loader()
        h, w = img.shape
        sha = image_sha256(img)
        rec = doc["jobs"].get(jid)
        same = (rec and rec.get("image_sha256") == sha and rec.get("b") == b and rec.get("t") == t
                and rec.get("tol") == tol)
        if same and rec.get("complete"):
            continue
        R = oracle.num_ranges(h, w, b)
        if not same:
            rec = {"image_sha256": sha, "shape": [h, w], "b": b, "t": t, "tol": tol,
                   "ranges": R, "domains": oracle.num_domains(h, w, b, t), "blocks": [],
                   "block_pairs": [], "seconds": 0.0, "complete": False}
        fds = None
        if tol is not None:
            fds = oracle.classify(img, b, t, threads)
            rec["tol_resolved"] = oracle.resolve_tol(tol, fds[1])
            rec["pool_margin"] = oracle.pool_margin(fds[0], fds[1], rec["tol_resolved"])
        nblk = (R + BLOCK - 1) // BLOCK
        for blk in range(len(rec["blocks"]), nblk):
            sel = np.arange(blk * BLOCK, min(R, (blk + 1) * BLOCK), dtype=np.int64)
            t0 = time.time()
            out = oracle.encode(img, b, t, tol=tol, sel=sel, nthreads=threads, fds=fds)
            dt = time.time() - t0
            rec["blocks"].append(block_digest(out))
            rec["block_pairs"].append(int(np.sum(out["pool"])) * 8)
            rec["seconds"] = round(rec["seconds"] + dt, 2)
            rec["complete"] = len(rec["blocks"]) == nblk
            if rec["complete"]:
                rec["pairs"] = int(sum(rec["block_pairs"]))
            doc["jobs"][jid] = rec
            save(doc)
            print("%s block %d/%d: %.1f s" % (jid, blk + 1, nblk, dt), flush=True)
        doc["jobs"][jid] = rec
        save(doc)
    return doc


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=None, help="regex over job ids")
    ap.add_argument("--threads", type=int, default=0, help="oracle threads (0 = all)")
    a = ap.parse_args()
    run(a.only, a.threads)
