"""The flush-time fit of the matrix-core search, restated on the CPU.

The queue flushes pick each pair's contrast index from three candidates,
round(v') - 1, round(v'), round(v') + 1 (v' an fp32 approximation of the
parabola's vertex 64 Srd'/Sdd', clamped into [-16, 15]), and compare their F
exactly. These tests check that rule against the minimum over all 32 values
of k (ties to the smaller |k|), including exact half-way vertices, clamped
vertices and the largest 16x16 magnitudes, and that every F is an integer
below 2^53 (so the fp64 fmas are exact).
"""
import numpy as np

KS = np.arange(-16, 16)


def f_of(k, srr, srd, sdd):
    return 4096 * srr - 128 * k * srd + k * k * sdd


def brute(srr, srd, sdd):
    fs = [f_of(int(k), srr, srd, sdd) for k in KS]
    best = min(fs)
    ks = [int(k) for k, f in zip(KS, fs) if f == best]
    return best, min(ks, key=abs)


def three(srr, srd, sdd):
    if sdd <= 0:
        return 4096 * srr, 0
    inv = np.float32(1.0) / np.float32(sdd)            # an fp32 reciprocal
    v = np.float32(64.0) * np.float32(srd) * inv
    kr = int(np.rint(min(max(float(v), -17.0), 16.0)))
    kr = -15 if kr < -15 else (14 if kr > 14 else kr)
    best, bk = None, None
    for k in (kr - 1, kr, kr + 1):
        f = f_of(k, srr, srd, sdd)
        if best is None or f < best or (f == best and abs(k) < abs(bk)):
            best, bk = f, k
    return best, bk


def cases(rng, n):
    out = []
    for _ in range(3000):
        r = rng.integers(0, 256, n)
        d = rng.integers(0, 1021, n) if rng.random() < 0.7 else \
            np.where(rng.random(n) < 0.5, 0, 1020)
        srr = n * int((r * r).sum()) - int(r.sum()) ** 2
        sdd = n * int((d * d).sum()) - int(d.sum()) ** 2
        perm = rng.permutation(n)
        srd = n * int((r * d[perm]).sum()) - int(r.sum()) * int(d.sum())
        out.append((srr, srd, sdd))
    # exact half-way vertices and clamps: Srd' = (k + 1/2) Sdd' / 64
    for k in range(-20, 20):
        sdd = 128 * 1000003
        out.append((10 ** 6, (2 * k + 1) * sdd // 128, sdd))
    out.append((0, 0, 0))
    return out


def test_three_candidates_equal_brute_force():
    rng = np.random.default_rng(11)
    for n in (16, 64, 256):
        for srr, srd, sdd in cases(rng, n):
            assert three(srr, srd, sdd) == brute(srr, srd, sdd), (n, srr, srd, sdd)


def test_terms_below_2_53():
    n = 256
    srr = n * n * 255 * 255 // 4
    sdd = n * n * 1020 * 1020 // 4
    srd = int(np.sqrt(srr * sdd))
    assert 4096 * srr + 128 * 16 * srd + 256 * sdd < 2 ** 53
