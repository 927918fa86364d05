"""pf_resample_noalloc (systematic resampling with its scratch in a static
device array, no allocation) against pf_test_resample (the same kernels with
allocated scratch): identical ancestors, on consecutive calls that reuse the
array with a smaller input after a larger one, at the size limit, and on the
error paths."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pf():
    from paper_1411_1702_amd import pf as _pf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _pf.lib()
    return _pf


def _weights(rng, n, power, zero_frac=0.2):
    g = rng.exponential(size=n) ** power
    g[rng.random(n) < zero_frac] = 0.0
    if g.sum() == 0:
        g[0] = 1.0
    return g / g.sum()


def _both(pf, g, r):
    n = len(g)
    gd = torch.as_tensor(g, dtype=torch.float64, device="cuda")
    a_ref = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    a_new = torch.full((n,), -2, dtype=torch.int32, device="cuda")
    s_ref = pf.lib().pf_test_resample(n, gd.data_ptr(), r, a_ref.data_ptr(), None)
    s_new = pf.lib().pf_resample_noalloc(n, gd.data_ptr(), r, a_new.data_ptr(), None)
    return s_ref, s_new, a_ref.cpu().numpy(), a_new.cpu().numpy()


def test_noalloc_matches_allocating_entry_point(pf, oracle):
    rng = np.random.default_rng(2024)
    # a large call, then smaller ones reusing the same static array
    for n, power in [(65536 + 13, 1), (1000, 3), (257, 5), (1, 1)]:
        g = _weights(rng, n, power)
        r = int(rng.integers(0, 2**63)) * 2 + 1
        print("noalloc resample: n", n, "power", power, flush=True)
        s_ref, s_new, a_ref, a_new = _both(pf, g, r)
        assert s_ref == pf.PF_OK and s_new == pf.PF_OK, (s_ref, s_new)
        assert np.array_equal(a_new, a_ref), (n, int((a_new != a_ref).sum()))
        st, want = oracle.resample(g, r)
        assert st == 0 and np.array_equal(a_new, want)


def test_noalloc_heavy_particles_and_limit(pf):
    rng = np.random.default_rng(7)
    # a few heavy particles (runs of copies longer than one lane writes)
    g = np.zeros(5000)
    g[[3, 1777, 4999]] = [0.5, 0.3, 0.2]
    s_ref, s_new, a_ref, a_new = _both(pf, g, 12345)
    assert s_ref == s_new == pf.PF_OK
    assert np.array_equal(a_new, a_ref)
    # the size limit, then a smaller call again
    n = 1 << 20
    g = _weights(rng, n, 2)
    print("noalloc resample: n", n, flush=True)
    s_ref, s_new, a_ref, a_new = _both(pf, g, 2**64 - 3)
    assert s_ref == s_new == pf.PF_OK
    assert np.array_equal(a_new, a_ref)
    g = _weights(rng, 3001, 1)
    s_ref, s_new, a_ref, a_new = _both(pf, g, 99)
    assert s_ref == s_new == pf.PF_OK
    assert np.array_equal(a_new, a_ref)


def test_noalloc_errors(pf):
    n = 300
    gd = torch.zeros(n, dtype=torch.float64, device="cuda")
    ad = torch.zeros(n, dtype=torch.int32, device="cuda")
    # every weight zero: degenerate, as for the allocating entry point
    assert pf.lib().pf_resample_noalloc(n, gd.data_ptr(), 5, ad.data_ptr(), None) == pf.PF_EDEGENERATE
    assert pf.lib().pf_test_resample(n, gd.data_ptr(), 5, ad.data_ptr(), None) == pf.PF_EDEGENERATE
    # sizes beyond the static array and NULL buffers are rejected before any launch
    assert pf.lib().pf_resample_noalloc((1 << 20) + 1, gd.data_ptr(), 5, ad.data_ptr(), None) == pf.PF_EINVAL
    assert b"2^20" in pf.lib().pf_last_error()
    assert pf.lib().pf_resample_noalloc(0, gd.data_ptr(), 5, ad.data_ptr(), None) == pf.PF_EINVAL
    assert pf.lib().pf_resample_noalloc(n, None, 5, ad.data_ptr(), None) == pf.PF_EINVAL
