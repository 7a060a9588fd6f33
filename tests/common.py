"""Shared test helpers: run the oracle on a synthetic instance, compare results."""
from __future__ import annotations

import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2601_17164_amd import inputs as I

_KIND_NAME = {I.POT_NONE: "none", I.POT_SOFTCORE: "softcore", I.POT_SCREENED: "screened",
              I.POT_HARMONIC: "harmonic"}


def oracle_potential(p: I.Potential) -> O.Potential:
    return O.Potential(_KIND_NAME[p.kind], p.z_inf, p.z_in, p.r_scr, p.soft2, p.omega_ho)


def oracle_ground(g: I.Ground) -> O.Ground:
    return O.Ground(g.l, g.alpha, g.coef, g.ip)


def pulse_table(pulse: I.Pulse, grid: I.Grid) -> np.ndarray:
    """The oracle's field table of the pulse on the grid (E_z at the half steps)."""
    return O.field_table_c(pulse.e0, pulse.omega, pulse.n_cycles, pulse.cep, grid.t_a, grid.h,
                           grid.n_steps)


def e_half(inst: I.Instance) -> np.ndarray:
    """The instance's explicit field table, else the oracle's table of its pulse."""
    return inst.e_half if inst.e_half is not None else pulse_table(inst.pulse, inst.grid)


def run_oracle(inst: I.Instance, n_threads: int = 0, kay_max=None) -> O.PropagateResult:
    return O.propagate(oracle_potential(inst.potential), oracle_ground(inst.ground), e_half(inst),
                       inst.grid.t_a, inst.grid.h, inst.grid.n_steps, inst.t0, inst.q0, inst.p0,
                       inst.w, inst.gamma, inst.kay_max if kay_max is None else kay_max,
                       inst.overlap_cut, n_threads)


def oracle_sfa_births(inst: I.Instance, mode=None, n_threads: int = 0) -> I.Instance:
    """The instance with q0, p0 and w from the oracle's SFA birth step (``inst.meta`` holds the
    birth samples k_perp and Monte-Carlo weights u)."""
    from dataclasses import replace
    pl = inst.pulse
    m = inst.meta["mode"] if mode is None else mode
    b = O.sfa_birth(pl.e0, pl.omega, pl.n_cycles, pl.cep, oracle_ground(inst.ground), inst.t0,
                    inst.meta["kperp"], inst.meta["u"], m, n_threads)
    return replace(inst, q0=b.q0, p0=b.p0, w=b.w, meta=dict(inst.meta, tt=b.tt, mode=m))


def rel_l2(a, b) -> float:
    a, b = np.asarray(a), np.asarray(b)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def require_gpu():
    if not gpu_available():
        pytest.skip("needs a GPU")
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if not os.path.exists(os.path.join(here, "paper_2601_17164_amd", "libsfhk.so")):
        pytest.fail("libsfhk.so is not built: run `python -m paper_2601_17164_amd.build`")
