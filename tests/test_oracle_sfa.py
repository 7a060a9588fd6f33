"""Pins of the oracle's SFA birth step (App. A: saddle-point equation, tunnel exit, action under
the barrier; App. B: tunnelling matrix elements) and of the contract sine/cosine its saddle-point
solve uses. Each pin compares the oracle with something that does not share its formulas: the
pulse evaluated from its definition with Python's complex functions, adaptive quadrature, the
Keldysh closed forms of a monochromatic field at its peak, and the plane-wave transform of the
GTOs by direct quadrature."""
import cmath
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import oracle as O
from paper_2601_17164_amd import inputs as I


def _ground(g):
    return O.Ground(g.l, np.array(g.alpha), np.array(g.coef), g.ip)


def _A(e0, om, nc, cep, t):
    """A(t) = -(e0/om) cos^2(pi t/T) sin(om t + cep), T = 2 pi nc/om, at complex t."""
    T = 2.0 * math.pi * nc / om
    return -(e0 / om) * cmath.cos(math.pi * t / T) ** 2 * cmath.sin(om * t + cep)


def _E(e0, om, nc, cep, t, h=1e-4):
    """E = -dA/dt at complex t by a complex-step-free 4th-order central difference along Re t."""
    f = lambda s: _A(e0, om, nc, cep, s)
    return -(8.0 * (f(t + h) - f(t - h)) - (f(t + 2 * h) - f(t - 2 * h))) / (12.0 * h)


# (pulse e0, omega, n_cycles, cep), ground state: the two workloads' pulses and a third with a CEP
PULSES = [
    (I.Pulse(800.0, 1e14, 2.0).e0, I.Pulse(800.0, 1e14, 2.0).omega, 2.0, 0.0, I.gto_h1s()),
    (I.Pulse(1600.0, 1.5e14, 8.0).e0, I.Pulse(1600.0, 1.5e14, 8.0).omega, 8.0, 0.0, I.gto_p058()),
    (0.08, 0.04, 3.0, 0.7, I.gto_h1s()),
]


def _samples(e0, om, nc, n, seed):
    rng = np.random.default_rng(seed)
    T = 2.0 * math.pi * nc / om
    t0 = rng.uniform(-0.45 * T, 0.45 * T, n)
    kp = rng.normal(0.0, 0.25, (2, n))
    return t0, kp


# ------------------------------------------------------------------------------------------
# contract sine and cosine
# ------------------------------------------------------------------------------------------
def test_sincos_contract_accuracy():
    """Within one ulp of the correctly rounded value for |x| <= 64 (the pulse phases stay below
    that), within two up to 2^20 (the reduced argument is one binary64 number)."""
    rng = np.random.default_rng(5)
    small = np.concatenate([rng.uniform(-64, 64, 4000), np.arange(-81, 82) * (math.pi / 4),
                            [0.0, -0.0, 1e-300, 5e-324, 1e-8],
                            np.nextafter(np.arange(1, 81) * (math.pi / 4), 0)])
    large = rng.uniform(-2.0 ** 20, 2.0 ** 20, 1000)
    for xs, bound in ((small, 1.0), (large, 2.0)):
        for x in xs:
            s, c = O.sincos_c(x)
            for got, ref, ref2 in ((s, O.sin_cr(x), math.sin(x)), (c, O.cos_cr(x), math.cos(x))):
                ulp = np.spacing(abs(ref)) if ref != 0.0 else 5e-324
                assert abs(got - ref) <= bound * ulp, (x, got, ref)
                assert abs(got - ref2) <= (bound + 1.0) * ulp, (x, got, ref2)


def test_sincos_contract_outside_domain():
    for x in (2.0 ** 20, -2.0 ** 21, math.inf, -math.inf, math.nan):
        s, c = O.sincos_c(x)
        assert math.isnan(s) and math.isnan(c)


# ------------------------------------------------------------------------------------------
# saddle point, tunnel exit
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("pi", range(len(PULSES)))
def test_saddle_point_equation_holds(pi):
    e0, om, nc, cep, g = PULSES[pi]
    t0, kp = _samples(e0, om, nc, 300, 11 + pi)
    r = O.sfa_birth(e0, om, nc, cep, _ground(g), t0, kp)
    ok = np.isfinite(r.tt)
    assert ok.mean() > 0.95
    for j in np.flatnonzero(ok):
        ts = complex(t0[j], r.tt[j])
        assert r.tt[j] > 0.0
        vz = r.p0[2, j] + _A(e0, om, nc, cep, ts) - _A(e0, om, nc, cep, t0[j])
        lhs = kp[0, j] ** 2 + kp[1, j] ** 2 + vz * vz + 2.0 * g.ip
        scale = 2.0 * g.ip + kp[0, j] ** 2 + kp[1, j] ** 2 + abs(vz) ** 2
        assert abs(lhs) <= 1e-12 * scale, (j, lhs)
        # p0 = (kx, ky, k_z), q0 on the polarisation axis
        assert r.p0[0, j] == kp[0, j] and r.p0[1, j] == kp[1, j]
        assert r.q0[0, j] == 0.0 and r.q0[1, j] == 0.0


@pytest.mark.parametrize("pi", range(len(PULSES)))
def test_saddle_point_is_the_one_nearest_the_real_axis(pi):
    """|Im A(t0 + i tau) - A(t0)| stays below kappa for 0 <= tau < t_t (no earlier root)."""
    e0, om, nc, cep, g = PULSES[pi]
    t0, kp = _samples(e0, om, nc, 60, 21 + pi)
    r = O.sfa_birth(e0, om, nc, cep, _ground(g), t0, kp)
    for j in np.flatnonzero(np.isfinite(r.tt)):
        kap = math.sqrt(2.0 * g.ip + kp[0, j] ** 2 + kp[1, j] ** 2)
        taus = np.linspace(0.0, r.tt[j], 4001)[:-1]
        ai = np.array([_A(e0, om, nc, cep, complex(t0[j], s)).imag for s in taus])
        assert np.max(np.abs(ai)) < kap * (1.0 + 1e-12)


@pytest.mark.parametrize("pi", range(len(PULSES)))
def test_tunnel_exit_is_real_part_of_the_integral_of_A(pi):
    e0, om, nc, cep, g = PULSES[pi]
    t0, kp = _samples(e0, om, nc, 40, 31 + pi)
    r = O.sfa_birth(e0, om, nc, cep, _ground(g), t0, kp)
    for j in np.flatnonzero(np.isfinite(r.tt)):
        # int_{t_s}^{t0} A dt along t = t0 + i s: dt = i ds, s from t_t down to 0
        re = quad(lambda s: (1j * _A(e0, om, nc, cep, complex(t0[j], s))).real, r.tt[j], 0.0,
                  epsabs=1e-13, epsrel=1e-12, limit=200)[0]
        assert abs(r.q0[2, j] - re) <= 1e-10 * max(1.0, abs(re)), (j, r.q0[2, j], re)


@pytest.mark.parametrize("kx", [0.0, 0.3])
@pytest.mark.parametrize("e0,om", [(0.05338, 0.056954), (0.2, 0.02), (0.03, 0.1)])
def test_keldysh_limit_at_the_field_peak(e0, om, kx):
    """A pulse of 10^8 cycles is monochromatic near t = 0 (envelope error ~ (pi t_t/T)^2):
    t_t = asinh(g)/w, q0_z = -(E0/w^2)(sqrt(1+g^2) - 1), k_z = 0 and
    Im S_down = (kappa^2/(2w)) [(1 + 1/(2 g^2)) asinh g - sqrt(1+g^2)/(2g)], g = kappa w/E0
    (Keldysh parameter with Ip -> kappa^2/2); Re S_down = Ip t0 = 0."""
    g = I.gto_h1s()
    ip = g.ip
    kap = math.sqrt(2.0 * ip + kx * kx)
    kg = kap * om / e0
    r = O.sfa_birth(e0, om, 1e8, 0.0, _ground(g), [0.0], [[kx], [0.0]], u=[1.0], mode=1)
    assert r.tt[0] == pytest.approx(math.asinh(kg) / om, rel=1e-12)
    assert r.q0[2, 0] == pytest.approx(-(e0 / om ** 2) * (math.sqrt(1 + kg * kg) - 1), rel=1e-12)
    assert abs(r.p0[2, 0]) <= 1e-12
    ims = (kap ** 2 / (2 * om)) * ((1 + 1 / (2 * kg * kg)) * math.asinh(kg)
                                   - math.sqrt(1 + kg * kg) / (2 * kg))
    # mode 1: w = e^{i S}/(E(t_s) k_s) with E(i t_t) = E0 cosh(w t_t), k_s = -i kappa
    ek = e0 * math.cosh(om * r.tt[0]) * (-1j * kap)
    want = math.exp(-ims) / ek
    assert abs(r.w[0] - want) <= 1e-11 * abs(want)


@pytest.mark.parametrize("pi", range(len(PULSES)))
def test_action_and_modified_weight_vs_quadrature(pi):
    """Mode 1 weight u e^{i kz q0z} e^{i S_down}/(E(t_s) k_s) with S_down by adaptive quadrature
    of its definition and E by differentiating A."""
    e0, om, nc, cep, g = PULSES[pi]
    t0, kp = _samples(e0, om, nc, 30, 41 + pi)
    u = np.linspace(0.5, 1.5, 30)
    r = O.sfa_birth(e0, om, nc, cep, _ground(g), t0, kp, u=u, mode=1)
    for j in np.flatnonzero(np.isfinite(r.tt)):
        kx, ky, kz, tt = kp[0, j], kp[1, j], r.p0[2, j], r.tt[j]
        a0 = _A(e0, om, nc, cep, t0[j])
        v2 = lambda s: (kx * kx + ky * ky + (kz + _A(e0, om, nc, cep, complex(t0[j], s)) - a0) ** 2)
        ir = quad(lambda s: v2(s).real / 2, 0.0, tt, epsabs=1e-14, epsrel=1e-13, limit=400)[0]
        ii = quad(lambda s: v2(s).imag / 2, 0.0, tt, epsabs=1e-14, epsrel=1e-13, limit=400)[0]
        ts = complex(t0[j], tt)
        S = g.ip * ts + 1j * complex(ir, ii)
        if S.imag > 600:
            assert abs(r.w[j]) < 1e-200
            continue
        ez = _E(e0, om, nc, cep, ts)
        kzs = kz + _A(e0, om, nc, cep, ts) - a0
        want = u[j] * cmath.exp(1j * kz * r.q0[2, j]) * cmath.exp(1j * S) / (ez * kzs)
        assert abs(r.w[j] - want) <= 1e-8 * abs(want), (j, r.w[j], want)


def _transform_1d(alpha, k, power):
    """int z^power exp(-alpha z^2 - i k z) dz by the trapezoidal rule (exact to rounding for a
    Gaussian integrand on a wide, fine grid; complex k is fine while the Gaussian dominates)."""
    c = (k.imag / (2 * alpha)) if isinstance(k, complex) else 0.0
    half = 12.0 / math.sqrt(alpha) + abs(c)
    z = np.linspace(c - half, c + half, 40001)
    f = z ** power * np.exp(-alpha * z * z - 1j * k * z)
    return np.trapezoid(f, z)


@pytest.mark.parametrize("which", ["s", "p"])
def test_tunnelling_element_vs_plane_wave_transform(which):
    """Mode 0 / mode 1 = -i sqrt(2 pi i/(E k)) E(t_s) <k_s|z|psi0> (E k), with <k|z|psi0> the
    transform int e^{-i k.r} z psi0(r) d^3r evaluated axis by axis by quadrature."""
    e0, om, nc, cep, g = PULSES[0] if which == "s" else PULSES[1]
    t0, kp = _samples(e0, om, nc, 8, 51)
    gr = _ground(g)
    r0 = O.sfa_birth(e0, om, nc, cep, gr, t0, kp, mode=0)
    r1 = O.sfa_birth(e0, om, nc, cep, gr, t0, kp, mode=1)
    for j in np.flatnonzero(np.isfinite(r0.tt) & (np.abs(r1.w) > 1e-250)):
        ts = complex(t0[j], r0.tt[j])
        kzs = r0.p0[2, j] + _A(e0, om, nc, cep, ts) - _A(e0, om, nc, cep, t0[j])
        me = 0.0
        for a, c in zip(g.alpha, g.coef):
            fx = _transform_1d(a, kp[0, j], 0)
            fy = _transform_1d(a, kp[1, j], 0)
            fz = _transform_1d(a, complex(kzs), 1 + g.l)
            me += c * fx * fy * fz
        ez = _E(e0, om, nc, cep, ts)
        ek = ez * kzs
        want = -1j * cmath.sqrt(2 * math.pi * 1j / ek) * ez * me * ek
        got = r0.w[j] / r1.w[j]
        assert abs(got - want) <= 1e-7 * abs(want), (j, got, want)


def test_field_sign_flip_mirrors_the_birth():
    """cep -> cep + pi flips A: the same t_t, and k_z, q0_z change sign."""
    e0, om, nc, cep, g = PULSES[2]
    t0, kp = _samples(e0, om, nc, 50, 61)
    a = O.sfa_birth(e0, om, nc, cep, _ground(g), t0, kp)
    b = O.sfa_birth(e0, om, nc, cep + math.pi, _ground(g), t0, kp)
    ok = np.isfinite(a.tt)
    np.testing.assert_allclose(b.tt[ok], a.tt[ok], rtol=1e-11)
    np.testing.assert_allclose(b.p0[2, ok], -a.p0[2, ok], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(b.q0[2, ok], -a.q0[2, ok], rtol=1e-9, atol=1e-12)


def test_no_saddle_and_nonfinite_samples_give_nan():
    e0, om, nc, cep, g = PULSES[0]
    r = O.sfa_birth(e0, om, nc, cep, _ground(g), [0.0, math.nan, 0.0, 0.0],
                    [[1e80, 0.0, math.inf, 0.1], [0.0, 0.0, 0.0, 0.0]])
    assert np.isnan(r.tt[:3]).all() and np.isnan(r.p0[2, :3]).all()
    assert np.isnan(r.q0[2, :3]).all() and np.isnan(r.w[:3]).all()
    assert np.isfinite(r.tt[3]) and np.isfinite(r.w[3])


def test_invalid_arguments_are_refused():
    e0, om, nc, cep, g = PULSES[0]
    gr = _ground(g)
    for args in ((e0, om, 1.0, cep), (e0, om, 0.5, cep), (-e0, om, nc, cep), (e0, 0.0, nc, cep)):
        with pytest.raises(ValueError):
            O.sfa_birth(*args, gr, [0.0], [[0.0], [0.0]])
    with pytest.raises(ValueError):
        O.sfa_birth(e0, om, nc, cep, gr, [0.0], [[0.0], [0.0]], mode=2)
