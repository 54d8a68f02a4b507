"""The rounding bound behind the one-accumulator screen of 16x16 ranges.

The matrix-core search of 16x16 ranges sums all n = 256 products of a
(range, isometry, domain) pair in one FP32 accumulator and lowers the range's
threshold T by e = (n + KS) 2^-23 sqrt(n) ||A|| with ||A||^2 <= Srr'/n + n/4,
claiming that the FP32 sum is within (n + KS) 2^-23 ||A|| ||B|| of the exact
cross term and that ||B|| <= sqrt(n) (u + 1/2), u = sqrt(Sdd')/n. These CPU
tests check the three inequalities on centred integer operands of the
search's ranges (|A| <= 255, |B| <= 1020), with the worst accumulation model
(every product added to the running FP32 sum on its own, 8 blocks of 32).
"""
import numpy as np

N, KS = 256, 8


def centred(x):
    """x - round(mean(x)) with the kernels' integer level (sum + n/2) // n."""
    n = x.size
    lvl = (int(x.sum()) + n // 2) // n
    return x - lvl


def fp32_sequential(a, b, order):
    acc = np.float32(0.0)
    for i in order:
        acc = np.float32(acc + np.float32(float(a[i]) * float(b[i])))
    return float(acc)


def operands(rng, kind):
    if kind == "uniform":
        r = rng.integers(0, 256, N)
        d = rng.integers(0, 1021, N)
    elif kind == "extreme":           # two-level blocks: largest |A|, |B|
        r = np.where(rng.random(N) < 0.5, 0, 255)
        d = np.where(rng.random(N) < 0.5, 0, 1020)
        d = np.where(r > 0, 1020, 0) if rng.random() < 0.5 else d
    else:                               # low contrast around a level
        r = 128 + rng.integers(-2, 3, N)
        d = 512 + rng.integers(-6, 7, N)
    return r.astype(np.int64), d.astype(np.int64)


def test_one_accumulator_sum_within_bound():
    rng = np.random.default_rng(7)
    worst = 0.0
    for t in range(300):
        r, d = operands(rng, ("uniform", "extreme", "low")[t % 3])
        a, b = centred(r), centred(d)
        exact = int((a * b).sum())
        na, nb = float(np.sqrt((a * a).sum())), float(np.sqrt((b * b).sum()))
        bound = (N + KS) * 2.0 ** -23 * na * nb
        order = np.argsort(a * b) if t % 2 else rng.permutation(N)   # sorted: largest partial sums
        err = abs(fp32_sequential(a, b, order) - exact)
        assert err <= bound, (t, err, bound)
        worst = max(worst, err / max(bound, 1e-30))
    assert worst < 1.0


def test_norm_bounds_from_range_and_domain_sums():
    rng = np.random.default_rng(8)
    for t in range(300):
        r, d = operands(rng, ("uniform", "extreme", "low")[t % 3])
        a, b = centred(r), centred(d)
        srr = N * int((r * r).sum()) - int(r.sum()) ** 2
        sdd = N * int((d * d).sum()) - int(d.sum()) ** 2
        assert float((a * a).sum()) <= srr / N + N / 4 + 1e-9
        u = np.sqrt(sdd) / N
        assert np.sqrt(float((b * b).sum())) <= np.sqrt(N) * (u + 0.5) + 1e-9


def test_threshold_reduction_is_small():
    """The part of the error not proportional to u is at most e/2 <= 1.1,
    inside the screen's fixed allowance of 64."""
    na = 255.0 * np.sqrt(N)           # every |A| <= 255
    e = (N + KS) * 2.0 ** -23 * np.sqrt(N) * na
    assert e / 2 <= 1.1


# ---------------------------------------------------- clamped-contrast screen
def _f32(x):
    return np.float32(x)


def clamp_threshold(t, u, n):
    """The kernels' clamp_threshold in FP32 (fma emulated by one rounding of
    the fp64 value)."""
    t, u = _f32(t), _f32(u)
    if not t > _f32(_f32(n * 0.25) * u):
        return _f32(0.0)
    a = _f32(t * _f32(1.0 / n))
    b = _f32(_f32(_f32(n * 0.125) * u) * u)
    g = _f32(np.float64(_f32(2.0) * t) * np.float64(a) + np.float64(b))
    return _f32(g * _f32(1.0 - 2.0 ** -20))


def kernel_screen(c, t, u, n):
    """Both tests a queued cell goes through: max |C'''| >= T u - n/4 (one
    rounding) and, when the contrast is clamped, >= clamp_threshold - n/4."""
    slack = _f32(n / 4.0)
    c = _f32(abs(c))
    plain = _f32(np.float64(c) - np.float64(_f32(t)) * np.float64(_f32(u))) >= -slack
    return bool(plain and c >= _f32(clamp_threshold(t, u, n) - slack))


def best_f(srr, srd, sdd):
    return min(4096 * srr - 128 * k * srd + k * k * sdd for k in range(-16, 16))


def test_clamped_screen_never_rejects_a_pair_that_reaches_the_best():
    """For every pair and every F_best the pair reaches (its exact best F over
    k in [-16, 15] is <= F_best), the clamped-contrast screen lets it pass,
    with the kernels' rounding of T and u; and it rejects pairs the plain
    screen lets through (high-contrast ranges against flat domains)."""
    rng = np.random.default_rng(11)
    stricter = 0
    for b in (4, 8):
        n = b * b
        for trial in range(3000):
            kind = trial % 3
            if kind == 0:
                r = rng.integers(0, 256, n)
                d = rng.integers(0, 1021, n)
            elif kind == 1:                      # contrasty range, flat-ish domain
                r = np.where(rng.random(n) < 0.5, rng.integers(0, 40, n), rng.integers(200, 256, n))
                d = 500 + rng.integers(-30, 31, n)
            else:                                # domain similar to the range, any scale
                r = rng.integers(0, 256, n)
                s = rng.choice([0.25, 0.5, 1.0, 2.0, 4.0])
                d = np.clip(np.round(4 * (r - r.mean()) * s + 510 + rng.integers(-20, 21, n)), 0, 1020)
            r, d = r.astype(np.int64), d.astype(np.int64)
            rh = (int(r.sum()) + n // 2) // n            # the kernels' centring levels
            dh = (int(d.sum()) + n // 2) // n
            c = int(((r - rh) * (d - dh)).sum())         # C''', exact
            srr = n * int((r * r).sum()) - int(r.sum()) ** 2
            sdd = n * int((d * d).sum()) - int(d.sum()) ** 2
            srd = n * int((r * d).sum()) - int(r.sum()) * int(d.sum())
            if srr == 0 or sdd == 0:
                continue
            fx = best_f(srr, srd, sdd)
            u = np.sqrt(sdd) / n * (1.0 - 2.0 ** -20)
            for fb in (fx, fx + 1, fx + int(rng.integers(0, 4096 * 64)), 4096 * srr):
                if fb > 4096 * srr:
                    continue
                theta = srr - fb / 4096.0
                t = np.sqrt(theta) * (1.0 - 2.0 ** -20) if theta > 0 else 0.0
                assert kernel_screen(c, t, u, n), (b, trial, fb, fx)
            # a best key between the unclamped optimum and what the clamped
            # contrast reaches: the plain screen passes, the clamped one need not
            fcont = 4096 * srr - 4096.0 * srd * srd / sdd
            fb = int((fcont + fx) / 2)
            theta = srr - fb / 4096.0
            if theta > 0:
                t = np.sqrt(theta) * (1.0 - 2.0 ** -20)
                plain = _f32(np.float64(abs(c)) - np.float64(_f32(t)) * np.float64(_f32(u))) >= -n / 4
                if plain and not kernel_screen(c, t, u, n):
                    stricter += 1
    assert stricter > 0


def quant_threshold(u, n):
    return _f32(_f32(_f32(n * (1.0 / 128.0)) * _f32(u)) * _f32(u) * _f32(1.0 - 2.0 ** -20))


def test_quantised_contrast_screen_keeps_every_pair_that_beats_the_dc_code():
    """A pair can replace a range's key only with F < 4096 Srr' (the key
    starts at the DC code, the smallest (domain, isometry) of the pool), and
    then it passes max |C'''| >= n u^2/128 - n/4 with the kernels' rounding;
    pairs whose best k is 0 are mostly rejected."""
    rng = np.random.default_rng(12)
    rejected = 0
    for b in (4, 8, 16):
        n = b * b
        for trial in range(2000):
            scale = rng.choice([1, 3, 20, 255])
            r = np.clip(128 + rng.integers(-scale, scale + 1, n), 0, 255).astype(np.int64)
            d = np.clip(510 + rng.integers(-4 * scale, 4 * scale + 1, n), 0, 1020).astype(np.int64)
            if trial % 4 == 0:                      # correlated: a real contrast
                d = np.clip(510 + 2 * (r - 128) + rng.integers(-8, 9, n), 0, 1020)
            rh = (int(r.sum()) + n // 2) // n
            dh = (int(d.sum()) + n // 2) // n
            c = int(((r - rh) * (d - dh)).sum())
            srr = n * int((r * r).sum()) - int(r.sum()) ** 2
            sdd = n * int((d * d).sum()) - int(d.sum()) ** 2
            srd = n * int((r * d).sum()) - int(r.sum()) * int(d.sum())
            if sdd == 0:
                continue
            u = np.sqrt(sdd) / n * (1.0 - 2.0 ** -20)
            passes = _f32(abs(c)) >= _f32(quant_threshold(u, n) - _f32(n / 4.0))
            beats = best_f(srr, srd, sdd) < 4096 * srr
            if beats:
                assert passes, (b, trial, c, srd, sdd)
            elif not passes:
                rejected += 1
    assert rejected > 100
