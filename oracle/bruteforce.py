"""Pixel-level brute force of the quantized range-domain fit.

TEST INFRASTRUCTURE ONLY (part of the oracle). This is the plain definition
the encoder must reach, written out over the whole grid and used to pin the
closed-form oracle in ``fic_oracle.c`` on tiny images:

  for each range r, over every domain d (2x2-summed to D, dbar = D/4), every
  isometry q, every k in [-16, 15] (s = k/16) and every j in [0, 127]
  (o = 2j), the squared error of
      r_i ~ s * ((T_q dbar)_i - mean(dbar)) + o
  is evaluated pixel by pixel; the minimum wins, ties to the lowest
  (d, q), then the smaller |k|, the smaller k and the smaller j.

To stay exact it works with e_i = 64n*r_i - k*(n*(T_q D)_i - sum D) - 128n*j,
so sum e_i^2 = (64n)^2 * SSE; the returned error is 4096*n*SSE = sum e_i^2 / n.
The isometries come from numpy's rot90 / flips / transpose, a derivation
independent of the index table in the C oracle.
"""
import numpy as np


def isometries(block):
    """The 8 square isometries in the numbering used throughout: identity,
    rotations by 90/180/270 degrees clockwise, mirror left-right, mirror
    up-down, transpose, anti-transpose."""
    return [
        block,
        np.rot90(block, -1),
        np.rot90(block, 2),
        np.rot90(block, 1),
        block[:, ::-1],
        block[::-1, :],
        block.T,
        np.rot90(block, 2).T,
    ]


def lattice(h, w, b, t):
    """Range origins (raster) and domain origins (raster) of the lattice."""
    ranges = [(y, x) for y in range(0, h - b + 1, b) for x in range(0, w - b + 1, b)]
    doms = [(y, x) for y in range(0, h - 2 * b + 1, t) for x in range(0, w - 2 * b + 1, t)]
    return ranges, doms


def shrink(img, y, x, b):
    """2x2 sums of the 2b x 2b block at (y, x): a b x b int64 block."""
    blk = img[y:y + 2 * b, x:x + 2 * b].astype(np.int64)
    return blk.reshape(b, 2, b, 2).sum(axis=(1, 3))


def brute_encode(img, b, t, pools=None):
    """Exhaustive grid search; pools[r] (optional) lists the allowed domains.

    Returns dict of arrays dom, iso, k, j, err (err = 4096*n*SSE)."""
    img = np.asarray(img, dtype=np.uint8)
    h, w = img.shape
    n = b * b
    ranges, doms = lattice(h, w, b, t)
    # all (domain, isometry) candidates as rows of T_q(D), in (d, q) order
    cand = np.array([iso.reshape(-1) for (y, x) in doms
                     for iso in isometries(shrink(img, y, x, b))], dtype=np.int64)
    sum_d = cand.sum(axis=1)                                   # (DQ,)
    ks = np.arange(-16, 16, dtype=np.int64)
    js = np.arange(0, 128, dtype=np.int64)
    res = {k: [] for k in ("dom", "iso", "k", "j", "err")}
    for ri, (y, x) in enumerate(ranges):
        r = img[y:y + b, x:x + b].astype(np.int64).reshape(-1)
        allowed = np.ones(len(doms), dtype=bool)
        if pools is not None:
            allowed[:] = False
            allowed[list(pools[ri])] = True
        dq_ok = np.flatnonzero(np.repeat(allowed, 8))
        if dq_ok.size == 0:
            res["dom"].append(-1); res["iso"].append(-1); res["k"].append(0)
            res["j"].append(-1); res["err"].append(-1)
            continue
        centred = n * cand[dq_ok] - sum_d[dq_ok, None]         # (DQ, n)
        rows = []
        for k in ks:
            # e[dq, j, i] = 64n r_i - k * centred[dq, i] - 128 n j
            base = 64 * n * r[None, :] - k * centred            # (DQ, n)
            e = base[:, None, :] - (128 * n * js)[None, :, None]
            score = (e * e).sum(axis=2)                        # (DQ, 128)
            jj = np.argmin(score, axis=1)                      # first min: smaller j
            rows.append(np.stack([score[np.arange(dq_ok.size), jj], dq_ok,
                                  np.full(dq_ok.size, abs(int(k))),
                                  np.full(dq_ok.size, int(k)), jj], axis=1))
        allrows = np.concatenate(rows, axis=0)
        # lexicographic minimum of (score, d*8+q, |k|, k, j)
        order = np.lexsort(allrows.T[::-1])
        score, dq, _, k, j = (int(v) for v in allrows[order[0]])
        d, q = dq // 8, dq % 8
        assert score % n == 0
        res["dom"].append(d); res["iso"].append(q); res["k"].append(k)
        res["j"].append(j); res["err"].append(score // n)
    return {k: np.array(v, dtype=np.int64) for k, v in res.items()}


def brute_pair(rblock, dsum_block):
    """Best (4096*n*SSE, k, j) of one range block against one already-shrunk
    and already-transformed domain block, over the whole (k, j) grid."""
    r = np.asarray(rblock, dtype=np.int64).reshape(-1)
    dd = np.asarray(dsum_block, dtype=np.int64).reshape(-1)
    n = r.size
    best = None
    for k in range(-16, 16):
        for j in range(128):
            e = 64 * n * r - k * (n * dd - dd.sum()) - 128 * n * j
            s = int((e * e).sum())
            key = (s, abs(k), k, j)
            if best is None or key < best:
                best = key
    s, _, k, j = best
    return s // n, k, j


def decode_sweep_float(img, codes, b, t):
    """One simultaneous decoding sweep evaluated in float64 (exact here):
    pixel = clamp(floor(s * (T_q dbar - mean dbar) + o + 1/2), 0, 255)."""
    img = np.asarray(img, dtype=np.uint8)
    h, w = img.shape
    ranges, doms = lattice(h, w, b, t)
    out = img.copy()
    for ri, (y, x) in enumerate(ranges):
        dy, dx = doms[int(codes["dom"][ri])]
        dbar = shrink(img, dy, dx, b).astype(np.float64) / 4.0
        tq = isometries(dbar)[int(codes["iso"][ri])]
        val = (codes["k"][ri] / 16.0) * (tq - dbar.mean()) + 2.0 * codes["j"][ri]
        out[y:y + b, x:x + b] = np.clip(np.floor(val + 0.5), 0, 255).astype(np.uint8)
    return out
