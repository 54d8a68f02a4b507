"""The pool build's sort and window at the edges of its launch paths: one
LDS workgroup up to 4096 keys, two launches per digit above, with the tile
counts summed in the scatter up to 64 tiles (262144 keys) and scanned by a
launch of their own beyond. Keys: fp64 values (the order-preserving integer
images of Sec. 3.1's fractal dimensions) that tie everywhere, tie in few
values, differ only in their last bits, or span both signs. The permutation
must be the stable sort (numpy's stable argsort, unique under stability) and
each window [lo, hi) the positions p with -T <= s[p] - fd_r <= T,
T = tol + 1e-9, in fp64."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SIZES = [1, 2, 63, 1024, 4095, 4096, 4097, 8192, 262144, 262145, 300001]
KINDS = ["uniform", "all_equal", "few_values", "last_bits", "both_signs"]


def values(kind, n, rng):
    if kind == "uniform":
        return rng.uniform(2.0, 3.0, n)
    if kind == "all_equal":
        return np.full(n, 2.375)
    if kind == "few_values":
        return rng.choice(np.array([1.9, 2.25, 2.5, 2.5000000001, 3.1]), n)
    if kind == "last_bits":
        return np.float64(2.5) + rng.integers(-300, 300, n) * np.spacing(np.float64(2.5))
    # both signs, with tiny and subnormal magnitudes among them (no zeros:
    # -0.0 and 0.0 are equal numbers but distinct keys)
    x = rng.uniform(-1.5, 1.5, n)
    tiny = rng.choice(np.array([5e-324, -5e-324, 1e-300, -1e-300, 2.2e-308, -2.2e-308]), n)
    return np.where(rng.random(n) < 0.1, tiny, x)


@pytest.fixture(scope="module")
def fic():
    import paper_1206_4880_amd as p
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    p.fic.lib()
    return p


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", SIZES)
def test_pool_sort_and_window(fic, n, kind):
    rng = np.random.default_rng(1000 + n + 7 * KINDS.index(kind))
    fd = values(kind, n, rng)
    fr = np.concatenate([rng.choice(fd, 200), values(kind, 57, rng)])
    tol = 0.01 if kind != "last_bits" else 50 * float(np.spacing(np.float64(2.5)))
    dev = torch.device("cuda:0")
    perm, lo, hi = fic.build_domain_pool(torch.from_numpy(fr).to(dev), torch.from_numpy(fd).to(dev),
                                         tol)
    torch.cuda.synchronize()
    perm = perm.cpu().numpy().astype(np.int64)
    want = np.argsort(fd, kind="stable")
    assert np.array_equal(perm, want), "n=%d %s: first mismatch at %d" % (
        n, kind, int(np.flatnonzero(perm != want)[0]))
    s = fd[want]
    T = tol + 1e-9
    lo_want = np.array([np.count_nonzero(s - x < -T) for x in fr])
    hi_want = np.array([np.count_nonzero(s - x <= T) for x in fr])
    assert np.array_equal(lo.cpu().numpy().astype(np.int64), lo_want)
    assert np.array_equal(hi.cpu().numpy().astype(np.int64), hi_want)
