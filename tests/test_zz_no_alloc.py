"""sfhk_spectrum_noalloc, the spectrum entry point that allocates nothing (its working memory is a
fixed device array of the library), against sfhk_spectrum through the C ABI: the same results bit
for bit, on two calls in a row with the second smaller than the first, and its size limit."""
import numpy as np
import pytest

from tests.common import require_gpu

pytestmark = pytest.mark.gpu


def _signal(n, seed):
    rng = np.random.default_rng(seed)
    t = np.arange(n)
    return np.sin(0.01 * t) * np.exp(-((t - n / 2) / (n / 5)) ** 2) + 1e-3 * rng.standard_normal(n)


def test_noalloc_spectrum_equals_the_allocating_one_on_two_calls():
    require_gpu()
    import torch
    from paper_2601_17164_amd import sfhk

    cases = [  # (n, n_fft, dt): the largest transform the fixed memory holds, then a smaller one
        (40001, sfhk.SPECTRUM_NOALLOC_MAX_FFT, 0.053867),
        (2208, 0, 0.099973),
    ]
    for i, (n, nf, dt) in enumerate(cases):
        print(f"case {i}: n={n} n_fft={nf}", flush=True)
        d = torch.from_numpy(_signal(n, 100 + i)).to("cuda:0")
        t_first = -0.5 * n * dt
        tau = 0.5 * n * dt
        got = sfhk.spectrum_noalloc(d, t_first, dt, tau, nf)
        ref = sfhk.spectrum(d, t_first, dt, tau, nf)
        torch.cuda.synchronize()
        nk = (nf or n) // 2 + 1
        assert got[1].numel() == nk
        for a, b in zip(got, ref):
            assert torch.equal(a, b)
        assert bool(torch.isfinite(got[1]).all()) and float(got[1].max()) > 0.0


def test_noalloc_spectrum_rejects_sizes_beyond_its_memory():
    require_gpu()
    import torch
    from paper_2601_17164_amd import sfhk

    d = torch.zeros(1024, dtype=torch.float64, device="cuda:0")
    with pytest.raises(sfhk.SfhkError) as e:
        sfhk.spectrum_noalloc(d, 0.0, 0.1, 10.0, sfhk.SPECTRUM_NOALLOC_MAX_FFT + 2)
    assert e.value.status == sfhk.SFHK_E_INVALID
    with pytest.raises(sfhk.SfhkError):
        sfhk.spectrum_noalloc(d, 0.0, -0.1, 10.0, 0)
