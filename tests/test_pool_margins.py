"""Robustness of every pool of the workloads (CPU, oracle only).

A range's pool is the Sec. 3.1 window |fd_d - fd_r| <= tol (evaluated as
<= tol + 1e-9 in fp64). The GPU's fp64 dimensions agree with the oracle's to
about 1e-12, not bit for bit (different log routines), so the GPU and oracle
pools are the same sets only if no |fd_d - fd_r| lies within that distance of
the window edge. This checks the smallest such distance over all pooled jobs
of the workloads, the 64 batch images and the adaptive-window jobs, against
1e-11 (the GPU tests check the dimensions to 1e-12 and the sets exactly).
"""
import numpy as np
import pytest

MARGIN = 1e-11


def _jobs():
    from synth import batch_descs, workload_images
    from synth.workloads import color_image
    out = []
    for name, b, t, tol in (("fbm512rect_b8t2", 8, 2, 0.05), ("fbm1024_b8t1", 8, 1, 0.02),
                            ("fbm1024_b8t1", 8, 1, 0.1), ("fbm2048_twolevel", 16, 4, 0.05),
                            ("fbm2048_twolevel", 8, 2, 0.05)):
        out.append(("%s %d/%d tol %g" % (name, b, t, tol), (lambda n=name: workload_images(n)),
                    b, t, tol))
    for name, b, t in (("fbm512rect_b8t2", 8, 2), ("fbm1024_b8t1", 8, 1),
                       ("fbm2048_twolevel", 16, 4), ("fbm2048_twolevel", 8, 2)):
        out.append(("%s %d/%d adaptive" % (name, b, t), (lambda n=name: workload_images(n)),
                    b, t, -1.0))

    def luma():
        import oracle
        return oracle.color_planes(color_image(1024, 6), 0)[1]
    out.append(("color1024 luma 8/1 tol 0.05", luma, 8, 1, 0.05))
    for m, (im, b, t, tol) in enumerate(batch_descs(count=64)):
        out.append(("batch64 image %d %d/%d tol %g" % (m, b, t, tol), (lambda im=im: im), b, t, tol))
        if m < 8:
            out.append(("batch64 image %d %d/%d adaptive" % (m, b, t), (lambda im=im: im), b, t, -1.0))
    return out


@pytest.mark.slow
def test_pool_margins_of_all_workloads(oracle_lib):
    orc = oracle_lib
    worst = (np.inf, "")
    for what, load, b, t, tol in _jobs():
        img = load()
        fr, fd = orc.classify(img, b, t)
        te = orc.resolve_tol(tol, fd)
        m = orc.pool_margin(fr, fd, te)
        assert m > MARGIN, "%s: a pool decision is %.3g from the window edge" % (what, m)
        worst = min(worst, (m, what))
    print("smallest margin %.3g (%s)" % worst)
