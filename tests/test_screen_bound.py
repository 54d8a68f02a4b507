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
