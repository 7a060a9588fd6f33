"""Values the paper prints (tests/golden/paper_values.json, each with its passage) against the
host conventions (field units, Ip, defaults) and the oracle (its laser field and partial-wave
labels): the hydrogen cutoff near 90 eV and the sub-cycle field peaks near +-110 a.u. of the
three-cycle 1600 nm pulse (Sec. III.C), the ionisation thresholds (Sec. III.A, III.B), the s, p, d
bands of the partial-wave analysis and the method's D_t and gamma (Sec. III.A)."""
import json
import os

import numpy as np

from oracle import oracle as O
from paper_2601_17164_amd import inputs as I, metrics
from tests.common import pulse_table

HERE = os.path.dirname(os.path.abspath(__file__))
G = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))
EV_PER_AU = 27.211386245988  # hartree in eV (CODATA 2018)


def _pulse(d):
    p = d["pulse"]
    return I.Pulse(p["wavelength_nm"], p["intensity_wcm2"], float(p["n_cycles"]))


def test_hydrogen_cutoff_near_90_eV():
    g = G["h_cutoff_eV"]
    pl = _pulse(g)
    band = metrics.bands(g["ip_au"], pl.up, pl.omega)["cutoff"]
    cut_ev = (g["ip_au"] + 3.17 * pl.up) * EV_PER_AU
    assert abs(cut_ev - g["value"]) <= g["tol"], cut_ev
    assert band[0] < cut_ev / EV_PER_AU < band[1]


def test_subcycle_field_peaks_near_110_au():
    """The oracle's laser field (the one its SFA step uses) and its field table in the library's
    fixed sequence agree; |E|
    has its sub-cycle maxima next to the central one close to +-110 a.u. with an intensity
    almost a factor of two below the peak. With the pulse read as three optical cycles in total
    (T = N_c 2 pi / omega) they sit at +-99.3 a.u. with intensity ratio 0.64; a six-cycle total
    would give +-107 a.u. but only 12% weaker, against the printed factor of almost two."""
    g = G["subcycle_field_peaks_au"]
    pl = _pulse(g)
    T = pl.duration
    t = np.linspace(-0.5 * T, 0.5 * T, 6001)
    e = O.field_E(t, pl.e0, pl.omega, T)
    grid = I.time_grid(pl, 0.1)
    tab = pulse_table(pl, grid)
    th = grid.t_a + 0.5 * grid.h * np.arange(tab.size)
    np.testing.assert_allclose(O.field_E(th[::97], pl.e0, pl.omega, T), tab[::97], rtol=0,
                               atol=1e-15 * pl.e0)
    a = np.abs(e)
    peaks = t[1:-1][(a[1:-1] > a[:-2]) & (a[1:-1] >= a[2:])]
    heights = a[1:-1][(a[1:-1] > a[:-2]) & (a[1:-1] >= a[2:])]
    main = peaks[np.argmax(heights)]
    assert abs(main) < 1.0
    o = np.argsort(-heights)
    side = sorted(peaks[o][1:3])
    for got, want in zip(side, g["value"]):
        assert abs(got - want) <= g["tol"], (got, want)
    ratio = (heights[o][1] / heights[o][0]) ** 2
    assert g["intensity_ratio_min"] <= ratio <= g["intensity_ratio_max"], ratio


def test_ionisation_thresholds():
    g = G["h_threshold_eV"]
    assert abs(g["ip_au"] * EV_PER_AU - g["value"]) <= g["tol"]
    assert I.gto_h1s().ip == g["ip_au"]
    g = G["ar_threshold_eV"]
    assert abs(I.gto_p058().ip * EV_PER_AU - g["value"]) <= g["tol"]


def test_partial_wave_band_edges_in_the_oracle():
    """Free motion along x at unit distance from the axis (|L| = |p|): just inside and just below
    each printed band edge, the oracle's filter keeps the step for that band's bit only."""
    g = G["partial_wave_bands"]
    ground = O.Ground(0, np.array([0.5]), np.array([1.0]), 0.5)
    n_steps, h = 4, 0.01
    e = np.zeros(2 * n_steps + 1)
    for k, (lo, hi) in enumerate(g["value"]):
        for lval in (lo + 1e-9 if lo == 0.0 else lo, hi - 1e-9):
            args = (O.Potential("none"), ground, e, 0.0, h, n_steps, np.zeros(1),
                    np.array([[0.0], [0.0], [1.0]]), np.array([[lval], [0.0], [0.0]]))
            for bit in range(3):
                f = O.propagate(*args, w=np.ones(1), overlap_cut=1e9, pw_mask=1 << bit,
                                pw_radius=g["radius_au"]).F
                assert np.any(f != 0) == (bit == k), (lval, bit)


def test_method_defaults():
    inst = I.config0(n_birth=2, n_per_birth=2)
    assert inst.kay_max == G["kay_D_t"]["value"]
    assert inst.gamma == G["gamma_au"]["value"]
