"""The Gabor time-frequency transform (sfhk_gabor; the emission-time analysis of Sec. III.A) on the
GPU against the oracle's plain sum over every sample, to the FP64 bar: max |G_gpu - G_ref| within
1e-9 of max |G_ref| (the GPU drops samples beyond 9.2 sigma, where the window is below 4e-19, and
sums each chunk of 1024 samples by Horner's rule in e^{i w dt}, anchored with a sincos per chunk)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_17164_amd import inputs as I
from tests.common import e_half, oracle_ground, oracle_potential, require_gpu

pytestmark = pytest.mark.gpu

TOL = 1e-9


@pytest.fixture(scope="module")
def S():
    require_gpu()
    import torch
    from paper_2601_17164_amd import sfhk
    yield sfhk, torch


def _gpu(S, d, *args):
    sfhk, torch = S
    pw, G = sfhk.gabor(torch.from_numpy(np.ascontiguousarray(d)).to("cuda:0"), *args)
    torch.cuda.synchronize()
    return pw.cpu().numpy(), G.cpu().numpy()


def _err(g, r):
    return float(np.max(np.abs(g - r)) / np.max(np.abs(r)))


def test_wave_packet_ragged_grid(S):
    dt, n = 0.05, 6001
    t = -150.0 + dt * np.arange(n)
    d = np.exp(-(t - 12.0) ** 2 / (2 * 81.0)) * np.cos(1.3 * t)
    args = (t[0], dt, 6.0, -160.0, 19.0, 19, 0.011, 300)  # centres beyond both ends of the record
    pg, Gg = _gpu(S, d, *args)
    pr, Gr = O.gabor(d, *args)
    e = _err(Gg, Gr)
    print(f"wave packet: {e:.3e}", flush=True)
    assert e <= TOL
    assert np.max(np.abs(pg - pr)) <= TOL * np.max(pr)


def _oracle_velocity(inst):
    r = O.propagate(oracle_potential(inst.potential), oracle_ground(inst.ground), e_half(inst),
                    inst.grid.t_a, inst.grid.h, inst.grid.n_steps, inst.t0, inst.q0, inst.p0,
                    inst.w, inst.gamma, inst.kay_max, inst.overlap_cut, 0, velocity=True)
    return -2.0 * r.V.real


def test_sfhk_velocity_map(S):
    """The oracle's config-0 dipole velocity as the signal of both sides; then the whole chain
    (GPU velocity -> GPU Gabor) against (oracle velocity -> oracle Gabor)."""
    sfhk, torch = S
    inst = I.config0()
    v = _oracle_velocity(inst)
    w0 = inst.pulse.omega
    T = inst.grid.h * inst.grid.n_steps
    args = (inst.grid.t_a, inst.grid.h, 1.0 / (3.0 * w0), inst.grid.t_a, T / 63, 64, w0 / 10, 400)
    pr, Gr = O.gabor(v, *args)
    pg, Gg = _gpu(S, v, *args)
    assert _err(Gg, Gr) <= TOL
    ctx = sfhk.Context(0)
    job = sfhk.make_job(ctx, inst, velocity=True)
    assert job.propagate(0)
    vg = job.velocity()
    pw, G = sfhk.gabor(vg, *args)
    torch.cuda.synchronize()
    e = _err(G.cpu().numpy(), Gr)
    print(f"velocity chain: {e:.3e}", flush=True)
    assert e <= TOL
    job.close()
    ctx.close()


def test_full_size_record_sampled(S):
    """2^15 samples (the screened workload's output grid), 512 centres x 2048 frequencies in one
    launch; the oracle on four centres and every 32nd frequency."""
    pulse = I.Pulse(1600.0, 1.5e14, 8.0)
    T, w0 = pulse.duration, pulse.omega
    n = 1 << 15
    dt = T / n
    t = -0.5 * T + dt * np.arange(n)
    rng = np.random.default_rng(12)
    d = np.zeros(n)
    for _ in range(12):  # a few bursts at random times and harmonic frequencies
        tb, wb = rng.uniform(-0.4 * T, 0.4 * T), w0 * rng.uniform(5, 160)
        d += np.exp(-(t - tb) ** 2 / 50.0) * np.cos(wb * t + rng.uniform(0, 6))
    sigma, n_c, n_w, ws = 1.0 / (3.0 * w0), 512, 2048, w0 / 10
    tc0, tcs = -0.5 * T + T / 1024, T / 512
    pg, Gg = _gpu(S, d, t[0], dt, sigma, tc0, tcs, n_c, ws, n_w)
    # the bar is over the map: max |dG| against the largest |G| (a centre where only the e^-146
    # tails of distant bursts reach the window has |G| ~ 1e-64, and dropping them there is the
    # truncation the kernel states)
    cs = (0, 237, 325, 511)  # record edges and the centres on the bursts at t = -65 and 241
    ref = np.stack([O.gabor(d, t[0], dt, sigma, tc0 + c * tcs, tcs, 1, 32 * ws, n_w // 32)[1][0]
                    for c in cs])
    e = _err(Gg[list(cs), ::32], ref)
    print(f"full size, sampled: {e:.3e}", flush=True)
    assert e <= TOL


def test_edges_and_errors(S):
    sfhk, torch = S
    d = np.ones(100)
    pw, G = _gpu(S, d, 0.0, 0.1, 0.5, 100.0, 1.0, 3, 0.5, 4)  # windows far from the record
    assert np.all(pw == 0) and np.all(G == 0)
    pw, G = _gpu(S, np.zeros(0), 0.0, 0.1, 0.5, 0.0, 1.0, 2, 0.5, 3)
    assert np.all(pw == 0)
    x = torch.ones(10, dtype=torch.float64, device="cuda:0")
    for args in ((0.0, 0.1, 0.0, 0.0, 1.0, 2, 0.5, 2), (0.0, 0.0, 1.0, 0.0, 1.0, 2, 0.5, 2),
                 (0.0, 0.1, 1.0, 0.0, 1.0, 70000, 0.5, 2), (0.0, 0.1, math.inf, 0.0, 1.0, 2, 0.5, 2)):
        with pytest.raises(sfhk.SfhkError) as ei:
            sfhk.gabor(x, *args)
        assert ei.value.status == sfhk.SFHK_E_INVALID
