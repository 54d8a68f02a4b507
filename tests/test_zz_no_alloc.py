"""fic_encode_pifs_noalloc -- the encode entry point for callers that cannot
allocate -- against fic_encode_pifs on the same inputs, through the C ABI:
codes byte for byte, on two calls in a row (the second with a smaller image,
so it reuses the static scratch the first one left behind), for both
kernels, exhaustive and pooled; and the size limit answers
FIC_ERR_WORKSPACE before anything runs."""
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


def _img(n, h, seed):
    from synth import fbm
    return torch.from_numpy(fbm(n, n, h, np.random.default_rng(seed))).cuda()


def _pool(fic, x, b, t, tol):
    fr, _ = fic.fd_classify(x, b, b, want_fp32=False)
    fd, _ = fic.fd_classify(x, 2 * b, t, want_fp32=False)
    return fic.build_domain_pool(fr, fd, tol)


@pytest.mark.parametrize("kernel", ["mfma", "plain"])
def test_noalloc_equals_encode_pifs(fic, kernel):
    # a large call, then a smaller one on the same static scratch
    cases = [(_img(512, 0.4, 71), 8, 1, 0.05), (_img(128, 0.7, 72), 4, 2, None),
             (_img(96, 0.5, 73), 16, 2, 0.1)]
    if kernel == "plain":
        cases[0] = (_img(256, 0.4, 71), 8, 1, 0.05)
    for x, b, t, tol in cases:
        pool = _pool(fic, x, b, t, tol) if tol is not None else None
        ref = fic.encode_pifs(x, b, t, pool=pool, kernel=kernel)
        got = fic.fic.encode_pifs_noalloc(x, b, t, pool=pool, kernel=kernel)
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert np.array_equal(r, g), "%dx%d B=%d t=%d tol=%s" % (x.shape + (b, t, tol))
        assert not np.any(fic.unpack_codes(got)["flags"] & 0x80)


def test_noalloc_size_limit(fic):
    x = torch.zeros((1024, 1024), dtype=torch.uint8, device="cuda")
    with pytest.raises(fic.fic.FicError) as e:
        fic.fic.encode_pifs_noalloc(x, 8, 1)        # 170 MiB of workspace
    assert e.value.status == fic.fic.ERR_WORKSPACE
    assert fic.fic.lib().fic_noalloc_scratch_bytes() == 64 << 20
