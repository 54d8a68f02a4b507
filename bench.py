"""Benchmark of the range-domain matching search on one MI355X.

Single-image workloads (default: 1024x1024 fBm, 8x8 ranges, step 1,
exhaustive + FD pools 0.02 / 0.1): one step is one pass of the whole hot
path over the image -- fractal dimension of all ranges and domains
(differential box counting) per pooled geometry, the dynamic pool for each
tolerance (sort + window bounds), and for every job range prep, domain prep,
the persistent MFMA search and finalize.
The 64-image mixed workload (--workload batch64_mixed): one step is one
batch call (classify, pool and prep of every image, one persistent search per
range size, finalize), replayed as a HIP graph.
Inputs are resident in HBM before the timed region. The JSON line reports
pair evaluations per second over the whole step (value), encode seconds per
image, a roofline of the dominant kernel (the longest MFMA search launch,
timed by HIP events the library records on its own stream), the plain
one-thread-per-pair kernel on the exhaustive search, and the CPU oracle timed
on a bounded sample of ranges on the host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "range-domain pair evals/s + encode s/image, 1024² uint8; MFMA vs plain GPU"
PEAK_FP16_TFLOPS = 2500.0    # MI355X dense FP16 MFMA
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "search_mfma_fbm1024_traffic.json")


def kernel_source_hash():
    """Hash of the search kernels' code with comments and layout removed, so
    that the traffic record stays valid across comment-only edits."""
    import re
    h = hashlib.sha256()
    for f in ("encode.hip", "fic_internal.h"):
        with open(os.path.join(ROOT, "paper_1206_4880_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per exhaustive search launch from the committed rocprofv3
    counter runs, or None when they were taken on other kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    from synth import WORKLOADS
    ap.add_argument("--workload", default="fbm1024_b8t1",
                    choices=sorted(WORKLOADS) + ["adaptive_window"],
                    help="the synthetic job set a step runs (default fbm1024_b8t1: the 1024x1024 "
                         "exhaustive, pool 0.02 and pool 0.1 searches)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-kernel comparison")
    ap.add_argument("--counters", action="store_true",
                    help="one extra untimed step with survivor counters (the default for "
                         "single-image workloads)")
    ap.add_argument("--no-counters", action="store_true",
                    help="skip the untimed survivor-counter step")
    ap.add_argument("--only", default=None,
                    help="run only this job per step (e.g. 'exhaustive'), for profiling")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a device copy of this many MiB (counter calibration)")
    ap.add_argument("--no-tune", action="store_true",
                    help="time the built-in search parameters (skip the autotuner)")
    ap.add_argument("--tune-reps", type=int, default=2,
                    help="encodes per candidate in the autotuner (best of)")
    ap.add_argument("--tune-file", default=None,
                    help="load these search parameters (fic_tune_load) instead of autotuning")
    ap.add_argument("--tune-save", default=None,
                    help="after autotuning, save the parameters (fic_tune_save) to this file")
    ap.add_argument("--separate-searches", action="store_true",
                    help="batch: one search launch per range size instead of the combined one")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the search shards by ranges with no exchange "
              "beyond gathering codes, and the library drives one device per process "
              "(got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1206_4880_amd as fic
    from synth import WORKLOADS, workload_images

    if args.copy_mib:
        nbytes = args.copy_mib << 20
        src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes}))
        return

    wl = WORKLOADS.get(args.workload)
    if args.workload == "adaptive_window":
        out = bench_adaptive(args, fic)
    elif wl.name == "batch64_mixed":
        out = bench_batch(args, fic, wl)
    elif wl.rms is not None:
        out = bench_quadtree(args, fic, wl, workload_images(args.workload))
    elif wl.color:
        out = bench_color(args, fic, wl, workload_images(args.workload))
    else:
        out = bench_image(args, fic, wl, workload_images(args.workload))
    print(json.dumps(out))


def job_label(b, t, tol, multi):
    base = "exhaustive" if tol is None else "pool_%g" % tol
    return ("b%dt%d_" % (b, t) + base) if multi else base


def stage_sums(recs, steps):
    out = {}
    for (name, ms) in recs:
        out[name] = out.get(name, 0.0) + ms / steps
    return out


def progress(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def oracle_rate(img_np, b, t, tol, pool_sizes, D, seconds, what):
    """The oracle (as it stands) on an evenly spaced sample of ranges of about
    `seconds` of host work. The sample grows geometrically (at most 8x per
    run) until one run takes half the budget, so its fixed set-up cost can
    not make the sample explode; the last run is the reported one."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    R = len(pool_sizes)
    count = min(R, 8)
    while True:
        sel = np.linspace(0, R - 1, count).astype(np.int64)
        t0 = time.perf_counter()
        oracle.encode(img_np, b, t, tol=tol, sel=sel, nthreads=threads)
        cpu_s = time.perf_counter() - t0
        progress("oracle sample of %d ranges: %.2f s" % (count, cpu_s))
        if cpu_s >= 0.5 * seconds or count >= R:
            break
        grow = min(8.0, max(2.0, seconds / max(cpu_s, 1e-3)))
        count = min(R, int(count * grow))
    cpu_pairs = int(np.asarray(pool_sizes)[sel].sum()) * 8
    return {"value": round(cpu_pairs / cpu_s, 1), "unit": "pair evals/s", "cores": threads,
            "kind": "oracle",
            "sample": "%s: %d of %d ranges (%d pair evaluations, %.1f s)"
                      % (what, count, R, cpu_pairs, cpu_s)}


def oracle_single_thread():
    """The oracle on one host thread: the whole 64x64 exhaustive encode
    (8x8 ranges, step 1: 64 ranges x 2401 domains x 8), pairs/s per core."""
    import oracle
    from synth import workload_images
    oracle.build(force=False)
    img = workload_images("fbm64_b8t1")
    pairs = 64 * 2401 * 8
    best = None
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.encode(img, 8, 1, tol=None, nthreads=1)
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    return {"value": round(pairs / best, 1), "unit": "pair evals/s per core", "cores": 1,
            "sample": "fbm64_b8t1 exhaustive, all 64 ranges (%d pair evaluations, best of 3: "
                      "%.3f s)" % (pairs, best)}


def pool_margin(fr_t, fd_t, tol):
    """Smallest distance of any |fd_d - fd_r| from the window edge tol + 1e-9
    over the GPU's own fp64 dimensions (tol < 0: (max - min) / 3 of the
    domain values): how far the closest pool decision is from flipping."""
    import numpy as np
    fr = fr_t.cpu().numpy()
    fd = np.sort(fd_t.cpu().numpy())
    te = tol if tol >= 0 else (float(fd[-1]) - float(fd[0])) / 3.0
    edge = te + 1e-9
    best = np.inf
    for sign in (-1.0, 1.0):
        pos = np.searchsorted(fd, fr + sign * edge)
        for off in (-1, 0):
            p = np.clip(pos + off, 0, fd.size - 1)
            best = min(best, float(np.abs(np.abs(fd[p] - fr) - edge).min()))
    return best


def run_autotune(args, fic, images, jobs):
    """The library's autotuner on the workload's own images (untimed); the
    timed steps then run with its choices. Returns the report."""
    if args.tune_file:
        st = fic.fic.context(images[0].device.index).tune_load(args.tune_file)
        if st != fic.fic.OK:
            raise SystemExit("tune file %s not loaded (status %d)" % (args.tune_file, st))
        return {"tuned": "file", "file": os.path.basename(args.tune_file)}
    if args.no_tune:
        return {"tuned": False}
    t0 = time.perf_counter()
    rep = fic.fic.autotune(images, jobs, reps=max(1, args.tune_reps))
    dt = time.perf_counter() - t0
    if args.tune_save:
        fic.fic.context(images[0].device.index).tune_save(args.tune_save)
    launch = [r for r in rep if r["range_size"] == 0]
    rep = [r for r in rep if r["range_size"] != 0]
    for r in rep:
        progress("autotune B=%d log2D=%d bucket %d (%d images): chunk 2^%d -> 2^%d, flush %d -> %d, "
                 "xcd %d -> %d, %.3f -> %.3f ms"
                 % (r["range_size"], r["dlog2"], r["bucket"], r["images"], r["base_chunk_log2"],
                    r["chunk_log2"], r["base_flush_at"], r["flush_at"], r["base_xcd"], r["xcd"],
                    r["base_ms"], r["tuned_ms"]))
    out = {"tuned": True, "seconds": round(dt, 2)}
    if launch:
        r = launch[0]
        out["batch_search_launches"] = {
            "chosen": "one per range size" if r["flush_at"] else "one combined 4x4 + 8x8",
            "combined_ms": round(r["base_ms"], 4), "chosen_ms": round(r["tuned_ms"], 4)}
        progress("autotune batch launches: %s (combined %.3f ms, chosen %.3f ms)"
                 % (out["batch_search_launches"]["chosen"], r["base_ms"], r["tuned_ms"]))
    return dict(out, **{
            "classes": [{"range_size": r["range_size"], "log2_domains": r["dlog2"],
                         "pool_bucket": r["bucket"], "images": r["images"],
                         "chunk_log2": r["chunk_log2"], "flush_at": r["flush_at"],
                         "xcd_queues": r["xcd"],
                         "default_chunk_log2": r["base_chunk_log2"],
                         "default_flush_at": r["base_flush_at"],
                         "default_search_ms": round(r["base_ms"], 4),
                         "tuned_search_ms": round(r["tuned_ms"], 4)}
                        for r in rep]})


def searched_sizes(img_np, b, sizes):
    """Pool sizes with those of flat ranges set to 0. A range whose pixels
    are all equal (Srr' = 0) is coded without a search: every domain fits it
    exactly at k = 0, so the lowest pool domain under isometry 0 wins, and
    the search kernels skip it. Its pairs are not evaluated and are not
    counted. Ranges in raster order, as the pools."""
    import numpy as np
    h, w = img_np.shape
    blk = np.asarray(img_np)[:h // b * b, :w // b * b].reshape(h // b, b, w // b, b)
    flat = (blk.max(axis=(1, 3)) == blk.min(axis=(1, 3))).ravel()
    return np.where(flat, 0, np.asarray(sizes))


def search_kernel_name(b):
    """Name of the matrix-core search kernel the library runs for B x B ranges."""
    return {4: "k_search_mfma32<4>", 16: "k_search_lds16<16>"}.get(b, "k_search_mfma<%d>" % b)


def roofline_of(kernel, flops, t_s):
    achieved = flops / t_s / 1e12
    return {"kernel": kernel, "bound": "mfma", "achieved": round(achieved, 2),
            "peak": PEAK_FP16_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP16_TFLOPS, 4), "traffic": None,
            "avg_launch_ms": round(t_s * 1e3, 4), "flop_per_launch": int(flops)}


def bench_image(args, fic, wl, img_np):
    import numpy as np
    import torch

    dev = torch.device("cuda:0")
    img = torch.from_numpy(img_np).to(dev)
    H, W = img_np.shape
    jobs = list(wl.jobs)
    multi = len(set((b, t) for (b, t, _) in jobs)) > 1
    if args.only:
        jobs = [j for j in jobs if job_label(*j, multi) == args.only]
        if not jobs:
            raise SystemExit("no job named %s in %s" % (args.only, wl.name))
    geos = []
    for (b, t, tol) in jobs:
        if tol is not None and (b, t) not in geos:
            geos.append((b, t))
    ctx = fic.fic.context(0)
    R = {b: fic.fic.num_ranges(H, W, b) for (b, _, _) in jobs}
    D = {(b, t): fic.fic.num_domains(H, W, b, t) for (b, t, _) in jobs}
    codes = [torch.empty((R[b], 16), dtype=torch.uint8, device=dev) for (b, _, _) in jobs]

    def step(kernel="mfma"):
        fds = {}
        for (b, t) in geos:
            fr, _ = fic.fd_classify(img, b, b, want_fp32=False)
            fd, _ = fic.fd_classify(img, 2 * b, t, want_fp32=False)
            fds[(b, t)] = (fr, fd)
        pools = {}
        for (b, t, tol) in jobs:
            if tol is not None:
                pools[(b, t, tol)] = fic.build_domain_pool(*fds[(b, t)], tol)
        for i, (b, t, tol) in enumerate(jobs):
            fic.encode_pifs(img, b, t, pool=pools.get((b, t, tol)), kernel=kernel,
                            codes=codes[i])
        return pools

    # the autotuner on this image's jobs, before anything is timed
    tune = run_autotune(args, fic, [img] * len(jobs), jobs)

    # pair counts and pool sizes per job (from one untimed step)
    pools = step()
    torch.cuda.synchronize()
    margins = {}
    for (b, t, tol) in jobs:
        if tol is not None:
            fr, _ = fic.fd_classify(img, b, b, want_fp32=False)
            fd, _ = fic.fd_classify(img, 2 * b, t, want_fp32=False)
            margins[job_label(b, t, tol, multi)] = pool_margin(fr, fd, tol)
    pairs, sizes = [], []
    for (b, t, tol) in jobs:
        if tol is None:
            sizes.append(np.full(R[b], D[(b, t)], dtype=np.int64))
        else:
            _, lo, hi = pools[(b, t, tol)]
            sizes.append((hi.long() - lo.long()).cpu().numpy())
        pairs.append(int(searched_sizes(img_np, b, sizes[-1]).sum()) * 8)
    pairs_step = sum(pairs)
    progress("%s: %d jobs, %d pair evaluations per step" % (wl.name, len(jobs), pairs_step))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    recs = ctx.timing_read()
    ctx.timing(False)
    ms_step = (t_end - t_start) * 1e3 / args.steps
    progress("timed %d steps: %.3f ms per step" % (args.steps, ms_step))

    # records per step: classify x2 per classified geometry, one pool per
    # pooled job, then per job range_prep .. final
    per_step = len(recs) // args.steps
    stage_ms = stage_sums(recs, args.steps)
    n_cls, n_pool = 2 * len(geos), sum(1 for j in jobs if j[2] is not None)
    cls_ms = {g: 0.0 for g in geos}
    pool_ms = {}
    job_ms = [dict() for _ in jobs]
    search_ms = [[] for _ in jobs]
    enc_steps = [[] for _ in jobs]        # per step: the job's whole encode, ms
    pooled_jobs = [j for j in jobs if j[2] is not None]
    for s in range(args.steps):
        chunk = recs[s * per_step:(s + 1) * per_step]
        cls_s, pool_s = {}, {}
        for k in range(n_cls):
            cls_ms[geos[k // 2]] += chunk[k][1] / args.steps
            cls_s[geos[k // 2]] = cls_s.get(geos[k // 2], 0.0) + chunk[k][1]
        for k in range(n_pool):
            pool_ms[pooled_jobs[k]] = pool_ms.get(pooled_jobs[k], 0.0) + \
                chunk[n_cls + k][1] / args.steps
            pool_s[pooled_jobs[k]] = chunk[n_cls + k][1]
        ji = -1
        job_s = [0.0 for _ in jobs]
        for (name, ms) in chunk[n_cls + n_pool:]:
            if name == "range_prep":
                ji += 1
            job_ms[ji][name] = job_ms[ji].get(name, 0.0) + ms / args.steps
            job_s[ji] += ms
            if name == "search":
                search_ms[ji].append(ms)
        for i, (b, t, tol) in enumerate(jobs):
            # a pooled job also needs its classification and its pool
            extra = cls_s[(b, t)] + pool_s[(b, t, tol)] if tol is not None else 0.0
            enc_steps[i].append(job_s[i] + extra)

    # encode s/image and search rate: medians over the timed steps
    encode_s, job_rate = {}, {}
    for i, (b, t, tol) in enumerate(jobs):
        lab = job_label(b, t, tol, multi)
        encode_s[lab] = round(float(np.median(enc_steps[i])) / 1e3, 6)
        job_rate[lab] = pairs[i] / (float(np.median(search_ms[i])) / 1e3)

    # roofline of the dominant kernel: the search launch that takes longest
    dom = max(range(len(jobs)), key=lambda i: np.mean(search_ms[i]))
    bd, td, told = jobs[dom]
    t_search = float(np.mean(search_ms[dom])) / 1e3
    roofline = roofline_of("%s (%s)" % (search_kernel_name(bd), job_label(bd, td, told, multi)),
                           pairs[dom] * 2 * bd * bd, t_search)
    if wl.name == "fbm1024_b8t1" and dom == 0:
        roofline["traffic"] = measured_traffic()

    # HBM fraction of the classify and domain-prep stages
    hbm = {}
    if geos:
        cbytes = sum(2 * H * W + 8 * (R[b] + D[(b, t)]) for (b, t) in geos)
        gbs = cbytes / (sum(cls_ms.values()) / 1e3) / 1e9
        hbm["classify"] = {"GB/s": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4),
                           "bytes": cbytes}
    dbytes = H * W + D[(bd, td)] * (2 * bd * bd + 4 + 4 + 8 + 4)
    dms = job_ms[dom].get("domain_prep", 0.0)
    if dms:
        gbs = dbytes / (dms / 1e3) / 1e9
        hbm["domain_prep"] = {"GB/s": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4),
                              "bytes": dbytes}

    out = {
        "metric": METRIC,
        "value": round(pairs_step / (ms_step / 1e3), 1),
        "unit": "pair evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16", "data": "synthetic",
        "config": {"workload": wl.name, "description": wl.description,
                   "image": "%dx%d" % (H, W),
                   "jobs": [job_label(b, t, tol, multi) for (b, t, tol) in jobs],
                   "pairs_per_step": pairs_step, "pairs_per_job": pairs},
        "encode_s_per_image": encode_s,
        "search_pairs_per_s": {k: round(v, 1) for k, v in job_rate.items()},
        "stage_ms_per_step": {k: round(v, 4) for k, v in stage_ms.items()},
        "roofline": roofline,
        "hbm_stages": hbm,
        "autotune": tune,
        "pool_margin": {k: float("%.3g" % v) for k, v in margins.items()},
        "bitstream": {"%dx%d_b%dt%d" % (H, W, b, t): {
            "bits_per_range": int(fic.fic.lib().fic_packed_words(
                fic.fic.make_geom(H, W, b, t)) * 32 // R[b]),
            "packed_bytes": int(fic.fic.lib().fic_packed_words(fic.fic.make_geom(H, W, b, t))) * 4,
            "compression_ratio": round(8.0 * H * W / (32 * int(fic.fic.lib().fic_packed_words(
                fic.fic.make_geom(H, W, b, t)))), 3)} for (b, t) in sorted(set((b, t) for (b, t, _) in jobs))},
    }

    if args.counters or not args.no_counters:
        cnt = torch.zeros(4, dtype=torch.int64, device=dev)
        ctx.set_counters(cnt)
        step()
        torch.cuda.synchronize()
        ctx.set_counters(None)
        c = cnt.cpu().numpy()
        out["screen"] = {"pairs_screened": int(c[0]), "exact_evaluations": int(c[1]),
                         "work_items": int(c[2]), "seed_evaluations": int(c[3]),
                         "exact_fraction": float(c[1]) / pairs_step}

    # every code of every job: no internal-check failure (flag bit 7)
    torch.cuda.synchronize()
    mfma_codes = [c.cpu().numpy() for c in codes]
    out["codes_flag7"] = int(sum(int(np.count_nonzero(fic.unpack_codes(c)["flags"] & 0x80))
                                 for c in codes))
    if not args.no_plain:
        ex = [i for i, j in enumerate(jobs) if j[2] is None]
        if ex:
            i = ex[0]
            b, t, _ = jobs[i]
            fic.encode_pifs(img, b, t, pool=None, kernel="plain", codes=codes[i])   # warm
            torch.cuda.synchronize()
            ctx.timing(True)
            fic.encode_pifs(img, b, t, pool=None, kernel="plain", codes=codes[i])
            torch.cuda.synchronize()
            prec = ctx.timing_read()
            ctx.timing(False)
            p_search = sum(ms for (nme, ms) in prec if nme == "search") / 1e3
            p_total = sum(ms for (nme, ms) in prec) / 1e3
            lab = job_label(b, t, None, multi)
            out["plain"] = {"exhaustive_search_pairs_per_s": round(pairs[i] / p_search, 1),
                            "exhaustive_encode_s": round(p_total, 6),
                            "mfma_search_speedup": round(job_rate[lab] / (pairs[i] / p_search),
                                                         3),
                            "codes_equal_mfma": bool(np.array_equal(codes[i].cpu().numpy(),
                                                                    mfma_codes[i]))}

    if not args.no_cpu:
        out["cpu_baseline"] = oracle_rate(
            img_np, bd, td, told, sizes[dom], D[(bd, td)], args.cpu_seconds,
            "%s, %s" % (wl.name, job_label(bd, td, told, multi)))
        out["cpu_baseline"]["single_thread"] = oracle_single_thread()
    return out


def bench_quadtree(args, fic, wl, img_np):
    """One step = one two-level encode (fic_encode_quadtree): classify, pool
    and search the 16x16 ranges, split, classify, pool and search the
    quadrants of the split ranges. Pair evaluations count level 1 in full and
    level 2 only for the coded quadrants."""
    import numpy as np
    import torch

    dev = torch.device("cuda:0")
    img = torch.from_numpy(img_np).to(dev)
    H, W = img_np.shape
    (b1, t1, tol1), (b2, t2, tol2) = wl.jobs
    ctx = fic.fic.context(0)
    # the autotuner on the two levels' jobs over the whole image: its rows are
    # per (range size, domain count), so the two-level encode uses them
    tune = run_autotune(args, fic, [img, img], list(wl.jobs))
    c1, c2 = fic.encode_quadtree(img, b1, t1, tol1, b2, t2, tol2, wl.rms)

    def step():
        fic.encode_quadtree(img, b1, t1, tol1, b2, t2, tol2, wl.rms, codes=(c1, c2))

    torch.cuda.synchronize()
    sizes = []
    for (b, t, tol) in wl.jobs:
        fr, _ = fic.fd_classify(img, b, b, want_fp32=False)
        fd, _ = fic.fd_classify(img, 2 * b, t, want_fp32=False)
        _, lo, hi = fic.build_domain_pool(fr, fd, tol)
        sizes.append((hi.long() - lo.long()).cpu().numpy())
    coded = (fic.unpack_codes(c2)["flags"] & 4) == 0
    split = int(((fic.unpack_codes(c1)["flags"] & 2) != 0).sum())
    s1 = searched_sizes(img_np, b1, sizes[0])
    s2 = searched_sizes(img_np, b2, sizes[1])
    pairs = [int(s1.sum()) * 8, int(s2[coded].sum()) * 8]
    pairs_step = sum(pairs)
    progress("%s: %d of %d ranges split, %d pair evaluations per step"
             % (wl.name, split, sizes[0].size, pairs_step))
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t_start) * 1e3 / args.steps
    recs = ctx.timing_read()
    ctx.timing(False)
    progress("timed %d steps: %.3f ms per step" % (args.steps, ms_step))
    stage_ms = stage_sums(recs, args.steps)
    searches = [ms for (name, ms) in recs if name == "search"]
    lv_ms = [float(np.mean(searches[0::2])), float(np.mean(searches[1::2]))]
    dom = 0 if lv_ms[0] >= lv_ms[1] else 1
    bd = wl.jobs[dom][0]
    roofline = roofline_of("%s (level %d)" % (search_kernel_name(bd), dom + 1),
                           pairs[dom] * 2 * bd * bd, lv_ms[dom] / 1e3)
    out = {
        "metric": METRIC,
        "value": round(pairs_step / (ms_step / 1e3), 1),
        "unit": "pair evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16", "data": "synthetic",
        "config": {"workload": wl.name, "description": wl.description,
                   "image": "%dx%d" % (H, W), "rms_split": wl.rms,
                   "split_ranges": split, "level1_ranges": int(sizes[0].size),
                   "pairs_per_step": pairs_step, "pairs_per_level": pairs},
        "encode_s_per_image": round(ms_step / 1e3, 6),
        "search_ms_per_level": [round(v, 4) for v in lv_ms],
        "search_pairs_per_s_per_level": [round(p / (m / 1e3), 1) for p, m in zip(pairs, lv_ms)],
        "stage_ms_per_step": {k: round(v, 4) for k, v in stage_ms.items()},
        "roofline": roofline,
        "autotune": tune,
        # codes whose key disagreed with finalize's recompute from pixels
        "codes_flag7": int(sum(int(np.count_nonzero(fic.unpack_codes(c)["flags"] & 0x80))
                               for c in (c1, c2))),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = oracle_rate(img_np, b1, t1, tol1, sizes[0], None, args.cpu_seconds,
                                          "%s, level 1 (b%dt%d pool %g)" % (wl.name, b1, t1, tol1))
    return out


def bench_color(args, fic, wl, rgb_np):
    """One step = one colour encode (fic_encode_color): channel planes and the
    luma image, its classification and pool, the three channel searches."""
    import numpy as np
    import torch

    dev = torch.device("cuda:0")
    rgb = torch.from_numpy(rgb_np).to(dev)
    H, W = rgb_np.shape[:2]
    (b, t, tol), = wl.jobs
    ctx = fic.fic.context(0)
    a = rgb_np.astype(np.int64)
    luma = ((299 * a[:, :, 0] + 587 * a[:, :, 1] + 114 * a[:, :, 2] + 500) // 1000).astype(np.uint8)
    lx = torch.from_numpy(luma).to(dev)
    fr, _ = fic.fd_classify(lx, b, b, want_fp32=False)
    fd, _ = fic.fd_classify(lx, 2 * b, t, want_fp32=False)
    _, lo, hi = fic.build_domain_pool(fr, fd, tol)
    sz = (hi.long() - lo.long()).cpu().numpy()
    pairs_step = sum(int(searched_sizes(rgb_np[:, :, c], b, sz).sum()) * 8 for c in range(3))
    progress("%s: %d pair evaluations per step" % (wl.name, pairs_step))
    for _ in range(args.warmup):
        fic.encode_color(rgb, b, t, tol=tol)
    torch.cuda.synchronize()
    ctx.timing(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    out = None
    for _ in range(args.steps):
        out = fic.encode_color(rgb, b, t, tol=tol)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t_start) * 1e3 / args.steps
    recs = ctx.timing_read()
    ctx.timing(False)
    if out is None:
        out = fic.encode_color(rgb, b, t, tol=tol)
    progress("timed %d steps: %.3f ms per step" % (args.steps, ms_step))
    searches = [ms for (name, ms) in recs if name == "search"]
    t_s = float(np.mean(searches)) / 1e3
    roofline = roofline_of("%s (one channel)" % search_kernel_name(b), pairs_step / 3 * 2 * b * b, t_s)
    return {
        "metric": METRIC, "value": round(pairs_step / (ms_step / 1e3), 1), "unit": "pair evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f16",
        "data": "synthetic",
        "config": {"workload": wl.name, "description": wl.description, "image": "%dx%dx3" % (H, W),
                   "pairs_per_step": pairs_step},
        "encode_s_per_image": round(ms_step / 1e3, 6),
        "stage_ms_per_step": {k: round(v, 4) for k, v in stage_sums(recs, args.steps).items()},
        "roofline": roofline,
        # codes whose key disagreed with finalize's recompute from pixels
        "codes_flag7": int(sum(int(np.count_nonzero(fic.unpack_codes(c)["flags"] & 0x80))
                               for c in out)),
    }


def bench_adaptive(args, fic):
    """The paper's own window, D_f = (F_max - F_min)/3 over the image's domain
    dimensions (Sec. 3.1), against exhaustive search on the same images:
    pool fraction, PSNR of the decoded image (32 sweeps from gray), and the
    search rate. value = pair evaluations per second of the adaptive encodes."""
    import numpy as np
    import torch
    from synth import batch_descs, workload_images

    dev = torch.device("cuda:0")
    cases = [("fbm512rect_b8t2", workload_images("fbm512rect_b8t2"), 8, 2),
             ("fbm1024_b8t1", workload_images("fbm1024_b8t1"), 8, 1),
             ("fbm2048_twolevel", workload_images("fbm2048_twolevel"), 16, 4),
             ("fbm2048_twolevel", workload_images("fbm2048_twolevel"), 8, 2)]
    for m, (im, b, t, _) in enumerate(batch_descs(count=8)):
        cases.append(("batch64_mixed image %d" % m, im, b, t))

    def psnr(a, ref):
        d = a.astype(np.float64) - ref.astype(np.float64)
        mse = float(np.mean(d * d))
        return float("inf") if mse == 0 else 10.0 * np.log10(255.0 ** 2 / mse)

    def timed_encode(x, b, t, tol):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(max(1, args.steps)):
            codes, pool = fic.encode(x, b, t, tol=tol)
        torch.cuda.synchronize()
        return codes, pool, (time.perf_counter() - t0) * 1e3 / max(1, args.steps)

    def timed_graph(x, b, t, tol, ref):
        """The same encode as a one-image batch call replayed as a HIP graph
        (recorded by the first call): ms per call, and whether its codes
        equal the single-image call's."""
        job = [(b, t, tol)]
        ws = torch.empty(fic.batch_workspace_bytes([x], job), dtype=torch.uint8, device=dev)
        out = fic.encode_batch([x], job, ws=ws, graph=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(max(1, args.steps)):
            fic.encode_batch([x], job, codes=out, ws=ws, graph=True)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / max(1, args.steps)
        return ms, bool(torch.equal(out[0], ref))

    rows, tot_pairs, tot_ms = [], 0, 0.0
    for (name, im, b, t) in cases:
        x = torch.from_numpy(np.ascontiguousarray(im)).to(dev)
        H, W = im.shape
        R, D = fic.fic.num_ranges(H, W, b), fic.fic.num_domains(H, W, b, t)
        for _ in range(args.warmup):
            fic.encode(x, b, t, tol=-1.0)
        ce, _, ms_e = timed_encode(x, b, t, None)
        cd, pool, ms_d = timed_encode(x, b, t, -1.0)
        graph = {}
        if H * W <= 256 * 256:
            # small images: is the time host launch overhead or the GPU's kernel chain?
            ge, eq_e = timed_graph(x, b, t, None, ce)
            gd, eq_d = timed_graph(x, b, t, -1.0, cd)
            graph = {"encode_ms_exhaustive_graph": round(ge, 3),
                     "encode_ms_adaptive_graph": round(gd, 3),
                     "graph_codes_equal": eq_e and eq_d}
        _, lo, hi = pool
        sizes = (hi.long() - lo.long()).cpu().numpy()
        frac = float(sizes.mean()) / D
        oe, _ = fic.decode_pifs(ce, H, W, b, t, max_iters=32)
        od, _ = fic.decode_pifs(cd, H, W, b, t, max_iters=32)
        fr, _ = fic.fd_classify(x, b, b, want_fp32=False)
        fd, _ = fic.fd_classify(x, 2 * b, t, want_fp32=False)
        fdn = fd.cpu().numpy()
        pe, pd = psnr(oe.cpu().numpy(), im), psnr(od.cpu().numpy(), im)
        pairs = int(searched_sizes(im, b, sizes).sum()) * 8
        tot_pairs += pairs
        tot_ms += ms_d
        rows.append({"workload": name, "image": "%dx%d" % (H, W), "range_size": b,
                     "domain_step": t, "D_f": round((float(fdn.max()) - float(fdn.min())) / 3.0, 6),
                     "pool_fraction": round(frac, 4),
                     "empty_pool_ranges": int((sizes == 0).sum()),
                     "psnr_exhaustive_db": round(pe, 3), "psnr_adaptive_db": round(pd, 3),
                     "encode_ms_exhaustive": round(ms_e, 3), "encode_ms_adaptive": round(ms_d, 3),
                     **graph})
        progress("%s B=%d t=%d: pool %.3f, PSNR %.2f / %.2f dB, %.2f / %.2f ms"
                 % (name, b, t, frac, pe, pd, ms_e, ms_d))
    return {
        "metric": METRIC, "value": round(tot_pairs / (tot_ms / 1e3), 1), "unit": "pair evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(tot_ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f16", "data": "synthetic",
        "config": {"workload": "adaptive_window",
                   "description": "the adaptive D_f window on the 512, 1024, 2048 (both range "
                                  "sizes) images and 8 batch images, against exhaustive search"},
        "quality": rows,
    }


def bench_batch(args, fic, wl):
    """One step = one fic_encode_pifs_batch of the 64-image mixed workload
    (replayed as a HIP graph): classify, pool, prep of every image, one
    persistent search per range size, finalize."""
    import numpy as np
    import torch
    from synth import batch_descs

    items = batch_descs(count=64, base_seed=wl.seed)
    dev = torch.device("cuda:0")
    imgs = [torch.from_numpy(np.ascontiguousarray(im)).to(dev) for (im, _, _, _) in items]
    jobs = [(b, t, tol) for (_, b, t, tol) in items]
    ctx = fic.fic.context(0)
    if args.separate_searches:
        ctx.set_debug(fic.fic.DEBUG_SEPARATE_SEARCHES)
    ws = torch.empty(fic.batch_workspace_bytes(imgs, jobs), dtype=torch.uint8, device=dev)
    codes = [torch.empty(((im.shape[0] // b) * (im.shape[1] // b), 16), dtype=torch.uint8,
                         device=dev) for (im, b, _, _) in items]
    tune = run_autotune(args, fic, imgs, jobs)
    # pair counts: the same classification and pool kernels, image by image
    sizes, pairs_b, margin = [], {}, float("inf")
    for x, (b, t, tol) in zip(imgs, jobs):
        fr, _ = fic.fd_classify(x, b, b, want_fp32=False)
        fd, _ = fic.fd_classify(x, 2 * b, t, want_fp32=False)
        _, lo, hi = fic.build_domain_pool(fr, fd, tol)
        sz = (hi.long() - lo.long()).cpu().numpy()
        sizes.append(sz)
        pairs_b[b] = pairs_b.get(b, 0) + int(searched_sizes(x.cpu().numpy(), b, sz).sum()) * 8
        margin = min(margin, pool_margin(fr, fd, tol))
    pairs_step = sum(pairs_b.values())
    progress("%s: %d images, %d pair evaluations per step" % (wl.name, len(items), pairs_step))

    def step(graph=True):
        fic.encode_batch(imgs, jobs, codes=codes, ws=ws, graph=graph)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t_start) * 1e3 / args.steps
    progress("timed %d steps: %.3f ms per step" % (args.steps, ms_step))

    # stage breakdown from one eager (ungraphed) batch with the library's events
    ctx.timing(True)
    step(graph=False)
    torch.cuda.synchronize()
    recs = ctx.timing_read()
    ctx.timing(False)
    stage_ms = stage_sums(recs, 1)
    searches = [ms for (name, ms) in recs if name == "search"]
    flops = {b: pairs_b[b] * 2 * b * b for b in pairs_b}
    if 4 in pairs_b and 8 in pairs_b and len(searches) < len(pairs_b):
        # one combined launch over the 4x4 and 8x8 images (then 16x16 alone)
        launches = {"4+8": searches[0]}
        lflops = {"4+8": flops[4] + flops[8]}
        names = {"4+8": "k_search_mixed (batch, all 4x4 and 8x8 images)"}
        rest = [b for b in sorted(pairs_b) if b not in (4, 8)]
        searches = searches[1:]
    else:
        launches, lflops, names = {}, {}, {}
        rest = sorted(pairs_b)              # one search launch per range size, ascending B
    for b, ms in zip(rest, searches):
        launches[str(b)] = ms
        lflops[str(b)] = flops[b]
        names[str(b)] = "%s (batch, all B=%d images)" % (search_kernel_name(b), b)
    bd = max(launches, key=lambda k: launches[k])
    roofline = roofline_of(names[bd], lflops[bd], launches[bd] / 1e3)
    out = {
        "metric": METRIC,
        "value": round(pairs_step / (ms_step / 1e3), 1),
        "unit": "pair evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16", "data": "synthetic",
        "config": {"workload": wl.name, "description": wl.description, "images": len(items),
                   "pairs_per_step": pairs_step,
                   "pairs_per_range_size": {str(b): v for b, v in pairs_b.items()}},
        "encode_s_per_image": round(ms_step / 1e3 / len(items), 6),
        "search_ms_per_launch": {k: round(v, 4) for k, v in launches.items()},
        "eager_stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "roofline": roofline,
        "autotune": tune,
        "pool_margin_min": float("%.3g" % margin),
        # codes whose key disagreed with finalize's recompute from pixels
        "codes_flag7": int(sum(int(np.count_nonzero(fic.unpack_codes(c)["flags"] & 0x80))
                               for c in codes)),
    }
    if not args.no_cpu:
        big = max(range(len(items)), key=lambda i: int(sizes[i].sum()))
        im, b, t, tol = items[big]
        out["cpu_baseline"] = oracle_rate(im, b, t, tol, sizes[big], None, args.cpu_seconds,
                                          "batch image %d (%dx%d, B=%d, t=%d, tol %g)"
                                          % ((big,) + im.shape + (b, t, tol)))
    return out


if __name__ == "__main__":
    main()
