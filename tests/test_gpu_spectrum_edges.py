"""The Hann-windowed transform of App. D on the device (sfhk_spectrum and sfhk_spectrum_noalloc)
against the oracle's direct sum at the edges of its interface: one and two samples, odd lengths,
zero padding (n_fft > n, odd and even), lengths that end inside a chunk of samples, one chunk per
span and (above 64 chunks) two chunks per span. The device advances its twiddles by a recurrence re-anchored on the exact
table, so it agrees with the direct sum to rounding level (relative L2 1e-12 over all bins)."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.common import rel_l2, require_gpu

pytestmark = pytest.mark.gpu

CASES = [(1, 1), (2, 2), (3, 3), (7, 7), (64, 64), (1000, 1024), (1023, 1023), (1025, 4096),
         (3000, 3001), (5000, 8191), (40000, 40000), (66000, 66000)]


@pytest.fixture(scope="module")
def S():
    require_gpu()
    import torch
    from paper_2601_17164_amd import sfhk
    yield sfhk, torch


def _signal(n, seed):
    rng = np.random.default_rng(seed)
    t = np.arange(n)
    # a few harmonics of a slow carrier plus noise, the shape of a dipole record
    return (np.sin(0.03 * t) + 0.3 * np.sin(0.27 * t + 1.0) + 1e-3 * rng.standard_normal(n))


@pytest.mark.parametrize("n,n_fft", CASES)
def test_spectrum_edges_match_the_direct_sum(S, n, n_fft):
    sfhk, torch = S
    dt = 0.05
    t_first = -0.5 * (n - 1) * dt
    tau_h = 0.5 * n * dt + dt
    d = _signal(n, seed=n + 7 * n_fft)
    print(f"n = {n}, n_fft = {n_fft}", flush=True)
    om_r, p_r, x_r = O.spectrum(d, t_first, dt, tau_h, n_fft)
    dd = torch.from_numpy(d).cuda()
    om_g, p_g, x_g = sfhk.spectrum(dd, t_first, dt, tau_h, n_fft)
    om_g, p_g, x_g = om_g.cpu().numpy(), p_g.cpu().numpy(), x_g.cpu().numpy()
    assert len(x_g) == n_fft // 2 + 1
    np.testing.assert_allclose(om_g, om_r, rtol=1e-15, atol=0.0)
    assert rel_l2(x_g, x_r) <= 1e-12
    assert rel_l2(p_g, p_r) <= 1e-12
    if n_fft <= sfhk.SPECTRUM_NOALLOC_MAX_FFT:
        om_n, p_n, x_n = sfhk.spectrum_noalloc(dd, t_first, dt, tau_h, n_fft)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(x_n.cpu().numpy(), x_g)
        np.testing.assert_array_equal(om_n.cpu().numpy(), om_g)
