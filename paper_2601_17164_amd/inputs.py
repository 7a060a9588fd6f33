"""Seeded synthetic inputs for the SFHK hot path.

This module only describes problems and draws random numbers: laser-pulse parameters in atomic
units, the time grid, the tabulated laser field E_z(t), the GTO ground-state data and the
Gaussian phase-space samples. It holds none of the Herman-Kluk method's arithmetic and is the
only code that both the HIP path and the CPU oracle's tests use.

Workloads (shapes of the paper's hydrogen and argon runs, Sec. III):
  * ``config0``: soft-core H, 800 nm, 1e14 W/cm^2, 2-cycle sin^2 pulse, 64 births x 32 samples.
  * ``config1``: screened SAE potential, 1600 nm, 1.5e14 W/cm^2, 8 cycles, 1024 x 1024 samples,
    dipole resampled to 2^15 points.
  * ``batch_instances``: 64 instances of uneven size and pulse.
  * ``serving_request``: one request of the serving workload (seed 4000 + request id).
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")

# atomic-unit conversions
INTENSITY_AU_WCM2 = 3.50944758e16   # W/cm^2 per (a.u. field)^2
OMEGA_NM = 45.5633525               # omega [a.u.] = 45.5633525 / lambda [nm]

POT_NONE, POT_SOFTCORE, POT_SCREENED, POT_HARMONIC = 0, 1, 2, 3


@dataclass
class Potential:
    """V = -(z_inf + z_in exp(-r/r_scr)) / sqrt(r^2 + soft2) (SCREENED), -z_inf/sqrt(r^2+soft2)
    (SOFTCORE), omega_ho^2 r^2 / 2 (HARMONIC) or 0 (NONE)."""
    kind: int = POT_SOFTCORE
    z_inf: float = 1.0
    z_in: float = 0.0
    r_scr: float = 1.0
    soft2: float = 0.01
    omega_ho: float = 0.0

    @property
    def kind_name(self) -> str:
        return {0: "none", 1: "softcore", 2: "screened", 3: "harmonic"}[self.kind]


SOFTCORE_H = Potential(POT_SOFTCORE, 1.0, 0.0, 1.0, 0.01, 0.0)
SCREENED_SAE = Potential(POT_SCREENED, 1.0, 17.0, 0.6, 0.01, 0.0)


@dataclass
class Ground:
    l: int
    alpha: np.ndarray
    coef: np.ndarray
    ip: float


def load_gto(name: str) -> Ground:
    with open(os.path.join(DATA, name)) as f:
        d = json.load(f)
    return Ground(int(d["l"]), np.array(d["alpha"], dtype=np.float64),
                  np.array(d["coef"], dtype=np.float64), float(d["ip"]))


def gto_h1s() -> Ground:
    return load_gto("gto_s_h1s.json")


def gto_p058() -> Ground:
    return load_gto("gto_p_ip058.json")


@dataclass
class Pulse:
    """Linearly polarised (z) sin^2 pulse of n_cycles optical cycles in total, centred at t = 0."""
    wavelength_nm: float
    intensity_wcm2: float
    n_cycles: float
    cep: float = 0.0

    @property
    def omega(self) -> float:
        return OMEGA_NM / self.wavelength_nm

    @property
    def e0(self) -> float:
        return math.sqrt(self.intensity_wcm2 / INTENSITY_AU_WCM2)

    @property
    def duration(self) -> float:
        return self.n_cycles * 2.0 * math.pi / self.omega

    @property
    def up(self) -> float:
        return self.e0 ** 2 / (4.0 * self.omega ** 2)


@dataclass
class Grid:
    t_a: float
    h: float
    n_steps: int

    def t(self, n):
        return self.t_a + np.asarray(n) * self.h


def time_grid(pulse: Pulse, dt: float) -> Grid:
    """t_n = t_a + n h, t_a = -T/2, n_steps = ceil(T/dt), h = T/n_steps (ends at the pulse end)."""
    T = pulse.duration
    n = int(math.ceil(T / dt))
    return Grid(-0.5 * T, T / n, n)


def birth_times(grid: Grid, n_birth: int) -> np.ndarray:
    """Midpoints of n_birth equal bins over the pulse."""
    T = grid.h * grid.n_steps
    i = np.arange(n_birth, dtype=np.float64)
    return grid.t_a + (i + 0.5) * (T / n_birth)


def gaussian_samples(seed: int, n_birth: int, n_per_birth: int, gamma: float):
    """q0 ~ N(0, 1/(2 gamma)), p0 ~ N(0, gamma/2) per axis (variances), drawn birth-major, then
    sample, then (q0x, q0y, q0z, p0x, p0y, p0z). Returns q0, p0 as [3, n] arrays."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((n_birth, n_per_birth, 6))
    sq = math.sqrt(1.0 / (2.0 * gamma))
    sp = math.sqrt(gamma / 2.0)
    z = z.reshape(-1, 6)
    q0 = np.ascontiguousarray((z[:, :3] * sq).T)
    p0 = np.ascontiguousarray((z[:, 3:] * sp).T)
    return q0, p0


@dataclass
class Instance:
    """One SFHK problem: potential, ground state, pulse, grid and samples. The laser field of the
    pulse is tabulated by the library (or, on the test side, by the oracle); e_half gives an explicit
    table E_z(t_a + m h/2), m = 0..2 n_steps, instead (test cases with a field other than the
    pulse's, such as none)."""
    name: str
    potential: Potential
    ground: Ground
    pulse: Pulse
    grid: Grid
    e_half: Optional[np.ndarray]
    t0: np.ndarray
    q0: np.ndarray
    p0: np.ndarray
    w: Optional[np.ndarray] = None   # complex weights; None -> exp(i p0.q0)/n
    gamma: float = 0.5
    kay_max: float = 1e30
    overlap_cut: float = 60.0
    n_out: int = 0                   # 0: dipole on the step grid
    n_birth: int = 0
    n_per_birth: int = 0
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_traj(self) -> int:
        return int(self.t0.shape[0])

    def subset(self, idx) -> "Instance":
        idx = np.asarray(idx)
        meta = dict(self.meta)
        if "kperp" in meta:
            meta["kperp"] = np.ascontiguousarray(meta["kperp"][:, idx])
            meta["u"] = meta["u"][idx].copy()
        return replace(self, name=self.name + "[subset]", t0=self.t0[idx].copy(),
                       q0=np.ascontiguousarray(self.q0[:, idx]),
                       p0=np.ascontiguousarray(self.p0[:, idx]),
                       w=None if self.w is None else self.w[idx].copy(), meta=meta)

    def nominal_steps(self) -> int:
        """Sum over trajectories of (n_steps - birth step + 1) for births snapped to the grid."""
        u = (self.t0 - self.grid.t_a) / self.grid.h
        n0 = np.clip(np.ceil(u - 0.5), 0, self.grid.n_steps)
        return int(np.sum(self.grid.n_steps - n0 + 1))


def make_instance(name, potential, ground, pulse, dt, n_birth, n_per_birth, seed, gamma=0.5,
                  kay_max=1e30, n_out=0, overlap_cut=60.0) -> Instance:
    grid = time_grid(pulse, dt)
    tb = birth_times(grid, n_birth)
    t0 = np.repeat(tb, n_per_birth)
    q0, p0 = gaussian_samples(seed, n_birth, n_per_birth, gamma)
    return Instance(name, potential, ground, pulse, grid, None, t0, q0, p0, None, gamma,
                    kay_max, overlap_cut, n_out, n_birth, n_per_birth, seed)


def config0(n_birth=64, n_per_birth=32, seed=0) -> Instance:
    """Soft-core H, FP64, 2048 trajectories, dt = 0.1, output on the step grid."""
    return make_instance("softcore-H 800nm 1e14 2cyc", SOFTCORE_H, gto_h1s(),
                         Pulse(800.0, 1e14, 2.0), 0.1, n_birth, n_per_birth, seed)


def config1(n_birth=1024, n_per_birth=1024, seed=1, n_out=1 << 15) -> Instance:
    """Screened SAE potential, 2^20 trajectories, dt = 0.05, dipole on 2^15 points."""
    return make_instance("screened-SAE 1600nm 1.5e14 8cyc", SCREENED_SAE, gto_p058(),
                         Pulse(1600.0, 1.5e14, 8.0), 0.05, n_birth, n_per_birth, seed,
                         n_out=n_out)


def softcore_full(n_birth=512, n_per_birth=1024, seed=5) -> Instance:
    """Config 0's atom (soft-core H, s-wave GTO, Ip 0.5) at config 1's pulse (1600 nm,
    1.5e14 W/cm^2, 8 cycles), dt 0.1: the soft-core kernel at full size, 2^19 trajectories."""
    return make_instance("soft-core H 1600nm 1.5e14 8cyc", SOFTCORE_H, gto_h1s(),
                         Pulse(1600.0, 1.5e14, 8.0), 0.1, n_birth, n_per_birth, seed)


def config1_birth_subset(inst: Instance, births, n_per_birth=None) -> Instance:
    """Trajectories of the given birth groups (and optionally only the first samples of each)."""
    m = inst.n_per_birth if n_per_birth is None else n_per_birth
    idx = np.concatenate([b * inst.n_per_birth + np.arange(m) for b in births])
    return inst.subset(idx)


def random_instance(rng: np.random.Generator, seed: int, name: str,
                    traj_scale: float = 1.0, sfa: bool = False) -> Instance:
    """One instance of the uneven batch / serving mix: wavelength U(800, 2000) nm, intensity
    log-uniform in [0.8e14, 3e14] W/cm^2, 2..10 cycles, potential of config 0 or 1 (with its dt,
    Ip and GTO), N = 64 round(2^U(14, 20) / 64) trajectories (times traj_scale). sfa=True: the
    same instance with SFA birth samples (sfa_instance) instead of Gaussian ones."""
    lam = rng.uniform(800.0, 2000.0)
    inten = math.exp(rng.uniform(math.log(0.8e14), math.log(3e14)))
    ncyc = int(rng.integers(2, 11))
    which = int(rng.integers(0, 2))
    n = 64 * max(1, round(2.0 ** rng.uniform(14.0, 20.0) * traj_scale / 64.0))
    n_birth = int(min(max(2 ** int(math.floor(math.log2(n) / 2)), 64), 1024))
    n_per = int(math.ceil(n / n_birth))
    pulse = Pulse(lam, inten, float(ncyc))
    make = sfa_instance if sfa else make_instance
    if which == 0:
        return make(name, SOFTCORE_H, gto_h1s(), pulse, 0.1, n_birth, n_per, seed)
    return make(name, SCREENED_SAE, gto_p058(), pulse, 0.05, n_birth, n_per, seed)


def batch_instances(n=64, seed=3, traj_scale=1.0):
    """The uneven multi-instance batch: instance i draws from PCG64(seed) in order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [random_instance(rng, seed * 100003 + i, f"batch{i}", traj_scale) for i in range(n)]


def serving_request(req_id: int, traj_scale=1.0, sfa: bool = False) -> Instance:
    """Request req_id of the serving workload (independent of every other request); sfa=True
    gives it SFA birth samples, born on the device when the request is admitted."""
    s = 4000 + int(req_id)
    rng = np.random.Generator(np.random.PCG64(s))
    return random_instance(rng, s, f"req{req_id}", traj_scale, sfa=sfa)


def sfa_samples(seed: int, pulse: Pulse, grid: Grid, n_birth: int, n_per_birth: int, ip: float):
    """Samples of the SFA birth step: birth times are the n_birth bin midpoints snapped to the
    nearest grid step (ties to the lower), so each trajectory is born exactly at a step; transverse
    momenta k_perp ~ N(0, s^2) per axis with s^2 = E0 / (2 sqrt(2 Ip)) (the width of the
    quasi-static transverse momentum distribution at the field peak), drawn birth-major, then
    sample, then (kx, ky); Monte-Carlo weights u = dt0 / (n_per_birth pdf(k_perp)), dt0 = T/n_birth,
    so sum_j u_j f_j estimates int dt0 d^2k_perp f. Returns t0 [n], kperp [2, n], u [n]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((n_birth, n_per_birth, 2)).reshape(-1, 2)
    s2 = pulse.e0 / (2.0 * math.sqrt(2.0 * ip))
    kperp = np.ascontiguousarray((z * math.sqrt(s2)).T)
    tb = birth_times(grid, n_birth)
    n0 = np.clip(np.ceil((tb - grid.t_a) / grid.h - 0.5), 0, grid.n_steps)
    t0 = np.repeat(grid.t_a + n0 * grid.h, n_per_birth)
    T = grid.h * grid.n_steps
    r2 = np.sum(kperp * kperp, axis=0)
    u = (T / n_birth) * (2.0 * math.pi * s2) * np.exp(r2 / (2.0 * s2)) / n_per_birth
    return t0, kperp, u


def sfa_instance(name, potential, ground, pulse, dt, n_birth, n_per_birth, seed, mode=0,
                 gamma=0.5, kay_max=1e30, n_out=0, overlap_cut=60.0) -> Instance:
    """An instance whose initial conditions come from the SFA birth step: t0, k_perp and u are
    here (``meta``); q0, p0 and w are zero until the birth step fills them."""
    grid = time_grid(pulse, dt)
    t0, kperp, u = sfa_samples(seed, pulse, grid, n_birth, n_per_birth, ground.ip)
    n = t0.shape[0]
    return Instance(name, potential, ground, pulse, grid, None, t0, np.zeros((3, n)),
                    np.zeros((3, n)), np.zeros(n, dtype=np.complex128), gamma, kay_max,
                    overlap_cut, n_out, n_birth, n_per_birth, seed,
                    meta=dict(kperp=kperp, u=u, mode=mode))


def sfa_config0(n_birth=64, n_per_birth=32, seed=10, mode=0) -> Instance:
    """Config 0 (soft-core H, 800 nm, 1e14 W/cm^2, 2 cycles, dt 0.1) born by the SFA step."""
    return sfa_instance("softcore-H 800nm 1e14 2cyc sfa", SOFTCORE_H, gto_h1s(),
                        Pulse(800.0, 1e14, 2.0), 0.1, n_birth, n_per_birth, seed, mode)


def softcore_sfa_full(n_birth=512, n_per_birth=1024, seed=12, mode=0) -> Instance:
    """The soft-core probe's atom, pulse and sizes (softcore_full) born by the SFA step."""
    return sfa_instance("softcore-H 1600nm 1.5e14 8cyc sfa", SOFTCORE_H, gto_h1s(),
                        Pulse(1600.0, 1.5e14, 8.0), 0.1, n_birth, n_per_birth, seed, mode)


def sfa_config1(n_birth=1024, n_per_birth=1024, seed=11, mode=0, n_out=1 << 15) -> Instance:
    """Config 1 (screened SAE, 1600 nm, 1.5e14 W/cm^2, 8 cycles, dt 0.05) born by the SFA step."""
    return sfa_instance("screened-SAE 1600nm 1.5e14 8cyc sfa", SCREENED_SAE, gto_p058(),
                        Pulse(1600.0, 1.5e14, 8.0), 0.05, n_birth, n_per_birth, seed, mode,
                        n_out=n_out)


def harmonic_instance(omega_ho, pulse, dt, n_birth, n_per_birth, seed, gamma=0.5) -> Instance:
    return make_instance("harmonic", Potential(POT_HARMONIC, 0, 0, 1, 0, omega_ho), gto_h1s(),
                         pulse, dt, n_birth, n_per_birth, seed, gamma=gamma)
