"""The oracle's rounding contract against its correctly rounded build (no GPU).

The oracle follows a rounding contract (its own sequences for 1/sqrt, exp, sin and cos) so that
the GPU path can reproduce its chaotic trajectories bit for bit. The same source built with
-DOR_CORRECTLY_ROUNDED takes every square root, quotient, exponential, sine and cosine as the
plain operation rounded once. Where the problem is well conditioned the two builds must agree to
rounding level; where it is chaotic, their difference is the conditioning of the problem itself
(reported, not bounded)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_17164_amd import inputs as I
from tests.common import e_half, oracle_ground, oracle_potential, pulse_table, rel_l2

GAMMA = 0.5


def test_the_second_build_is_the_correctly_rounded_one():
    assert O.lib(False).or_correctly_rounded() == 0
    assert O.lib(True).or_correctly_rounded() == 1


def _both(fn, **kw):
    return fn(correctly_rounded=False, **kw), fn(correctly_rounded=True, **kw)


def _free_grid(n_steps):
    return np.zeros(2 * n_steps + 1)


def test_volkov_and_oscillator_agree_to_rounding():
    """Laser-only motion (App. A with V = 0) and the oscillator: no chaos, so the two builds'
    states, prefactors and integrands agree to a few ulps over the whole pulse (the prefactor's
    square root goes through the contract's rsqrt in one build and sqrt and / in the other)."""
    pulse = I.Pulse(800.0, 1e14, 2.0)
    grid = I.time_grid(pulse, 0.05)
    e = pulse_table(pulse, grid)
    q0, p0 = np.array([0.3, -0.2, 0.5]), np.array([0.1, 0.2, -0.3])
    g = oracle_ground(I.gto_h1s())
    a, b = _both(O.trajectory, pot=O.Potential("none"), ground=g, e_half=e, t_a=grid.t_a,
                 h=grid.h, n_steps=grid.n_steps, t0=grid.t_a + 100 * grid.h, q0=q0, p0=p0,
                 gamma=GAMMA)
    assert np.array_equal(a.alive, b.alive)
    assert np.max(np.abs(a.y - b.y)) <= 1e-13 * np.max(np.abs(a.y))
    assert np.max(np.abs(a.C - b.C) / np.maximum(np.abs(a.C), 1e-300)) <= 1e-14
    assert rel_l2(a.f, b.f) <= 1e-13
    n = 3000
    a, b = _both(O.trajectory, pot=O.Potential("harmonic", omega_ho=0.37), ground=g,
                 e_half=_free_grid(n), t_a=0.0, h=0.01, n_steps=n, t0=0.0,
                 q0=np.array([0.7, -0.4, 1.1]), p0=p0, gamma=GAMMA)
    assert np.max(np.abs(a.y - b.y)) <= 1e-13 * np.max(np.abs(a.y))
    assert np.max(np.abs(a.C - b.C) / np.abs(a.C)) <= 1e-13
    assert rel_l2(a.f, b.f) <= 1e-13


def test_kepler_orbit_agrees_to_rounding():
    """A bound, non-colliding Coulomb orbit (soft2 = 0, no field) over one period: the
    potential's 1/r goes through the contract rsqrt in one build and through sqrt and / in the
    other; a regular orbit lets the difference grow only linearly."""
    pot = O.Potential("softcore", z_inf=1.0, soft2=0.0)
    q0, p0 = np.array([1.0, 0.0, 0.0]), np.array([0.0, 0.8, 0.3])
    E = 0.5 * p0 @ p0 - 1.0
    n = 4000
    h = 2 * math.pi / (-2 * E) ** 1.5 / n
    a, b = _both(O.trajectory, pot=pot, ground=oracle_ground(I.gto_h1s()), e_half=_free_grid(n),
                 t_a=0.0, h=h, n_steps=n, t0=0.0, q0=q0, p0=p0, gamma=GAMMA)
    assert np.max(np.abs(a.y[:, :6] - b.y[:, :6])) <= 1e-11
    assert np.max(np.abs(a.y[:, 6:42] - b.y[:, 6:42])) <= 1e-11 * np.max(np.abs(a.y[:, 6:42]))


def _run(inst, kay, cr):
    return O.propagate(oracle_potential(inst.potential), oracle_ground(inst.ground), e_half(inst),
                       inst.grid.t_a, inst.grid.h, inst.grid.n_steps, inst.t0, inst.q0, inst.p0,
                       inst.w, inst.gamma, kay, inst.overlap_cut, velocity=True,
                       correctly_rounded=cr)


# measured (contract vs correctly rounded, relative L2 of F): config 0 4.7e-11, the screened
# subsets 1.0e-11 / 5.7e-12, the soft-core subset 9.6e-11. Trajectories live until |C|^2 = 1e4,
# and the near-core ones amplify a one-ulp difference by up to about 1e5 before they are removed.
@pytest.mark.parametrize("case", ["config0", "screened_16x16", "softcore_64x16"])
def test_workloads_agree_at_a_low_kay_limit(case):
    """With D_t = 1e4 (Sec. III.A removal) the unstable trajectories are removed before the
    rounding of either build is amplified far: F and V agree within 5e-10, and the removal
    counts are the same."""
    if case == "config0":
        inst = I.config0()
    elif case == "screened_16x16":
        inst = I.config1_birth_subset(I.config1(), list(range(0, 1024, 64)), 16)
    else:
        inst = I.softcore_full(n_birth=64, n_per_birth=16)
    a, b = _run(inst, 1e4, False), _run(inst, 1e4, True)
    assert a.kay_removed == b.kay_removed and a.nonfinite_removed == b.nonfinite_removed
    assert rel_l2(a.F, b.F) <= 5e-10
    assert rel_l2(a.V, b.V) <= 5e-10


def test_sfa_births_agree_to_rounding():
    """The SFA birth step (App. A saddle point, tunnel exit) with the contract sin/cos/exp/rsqrt
    against the correctly rounded functions: a smooth map of its inputs, so t_t, q0 and p0 agree
    to a few ulps."""
    inst = I.sfa_config0(n_birth=16, n_per_birth=16)
    pl = inst.pulse
    g = oracle_ground(inst.ground)
    a, b = _both(O.sfa_birth, e0=pl.e0, omega=pl.omega, n_cycles=pl.n_cycles, cep=pl.cep,
                 ground=g, t0=inst.t0, kperp=inst.meta["kperp"], u=inst.meta["u"])
    ok = np.isfinite(a.tt)
    assert ok.sum() > 200 and np.array_equal(ok, np.isfinite(b.tt))
    assert np.max(np.abs(a.tt[ok] - b.tt[ok]) / np.abs(a.tt[ok])) <= 1e-13
    assert np.max(np.abs(a.q0[:, ok] - b.q0[:, ok])) <= 1e-13 * np.max(np.abs(a.q0[:, ok]))
    assert np.max(np.abs(a.p0[:, ok] - b.p0[:, ok])) <= 1e-13 * np.max(np.abs(a.p0[:, ok]))
    assert rel_l2(a.w[ok], b.w[ok]) <= 1e-11
