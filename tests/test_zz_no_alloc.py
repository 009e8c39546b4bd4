"""The allocation-free trim entry point (wv_cdf_trim_noalloc) against wv_cdf_trim (needs an MI355X).

Two calls in a row through the C ABI, the second with fewer rows, each compared bit
for bit with the scratch-taking entry point on the same tables; and the row limit."""
import numpy as np
import pytest
import torch

from gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu

NSYM = 129


def _tables(n, seed):
    """CDF rows of n random 3-component mixtures, built by the library's CDF kernel."""
    from paper_2405_12631_amd import _lib as L, codec
    rng = np.random.default_rng(seed)
    w = rng.dirichlet(np.ones(3), n)
    mu = rng.uniform(-70, 70, (n, 3))
    sg = np.exp(rng.uniform(np.log(0.11), np.log(40.0), (n, 3)))
    prm = torch.from_numpy(np.concatenate([w, mu, sg], 1).astype(np.float32).ravel()).cuda()
    cdf = torch.empty(n * (NSYM + 1), dtype=torch.int16, device="cuda")
    L.call("wv_cdf_tables", codec._ptr(prm), n, 3, L.WV_DIST_GAUSS, -64, 64, 16, codec._ptr(cdf), codec._stream())
    return cdf


def _trim(cdf, n, noalloc):
    import ctypes
    from paper_2405_12631_amd import _lib as L, codec
    lolen = torch.full((2 * n,), 0xAB, dtype=torch.uint8, device="cuda")
    packed = torch.full((n * (NSYM - 1),), -1, dtype=torch.int16, device="cuda")
    if noalloc:
        rc = L.lib().wv_cdf_trim_noalloc(codec._ptr(cdf), n, NSYM, codec._ptr(lolen), codec._ptr(packed),
                                         packed.numel(), codec._stream())
    else:
        nb = ctypes.c_size_t()
        L.call("wv_cdf_trim_scratch_bytes", n, ctypes.byref(nb))
        scratch = torch.empty(max(nb.value, 8), dtype=torch.uint8, device="cuda")
        rc = L.lib().wv_cdf_trim(codec._ptr(cdf), n, NSYM, codec._ptr(lolen), codec._ptr(packed), packed.numel(),
                                 codec._ptr(scratch), scratch.numel(), codec._stream())
    assert rc == L.WV_OK, L.lib().wv_last_error()
    torch.cuda.synchronize()
    ll = lolen.cpu().numpy()
    total = int(ll[1::2].astype(np.int64).sum())
    return ll, packed[:total].cpu().numpy()


def test_trim_noalloc_equals_trim_two_calls():
    need_gpu()
    from paper_2405_12631_amd import _lib as L, codec
    for n, seed in ((300_000, 1), (1_000, 2)):     # 1172 blocks (two scan chunks), then a smaller call
        say("trim noalloc", n)
        cdf = _tables(n, seed)
        ref = _trim(cdf, n, noalloc=False)
        got = _trim(cdf, n, noalloc=True)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), n
        assert 0 < len(ref[1]) < n * (NSYM - 1)
    # Beyond the static array: refused before any launch.
    big = 8_388_609
    rc = L.lib().wv_cdf_trim_noalloc(codec._ptr(cdf), big, NSYM, codec._ptr(cdf), codec._ptr(cdf), big * 128,
                                     codec._stream())
    assert rc == L.WV_ENOMEM
