"""Thin ctypes binding of ``libsfhk.so`` (the C ABI declared in ``include/sfhk.h``).

Argument marshalling only: every step of the hot path (trajectory propagation with monodromy and
action, HK prefactor, Kay removal, dipole integrand, reduction, spectrum) runs in the HIP kernels
of the library. PyTorch provides device memory and the HIP stream. The library must have been
built (``python -m paper_2601_17164_amd.build``); importing this module on a machine without it
raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as ct
import os
import weakref
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# SFHK_LIB may name another build of the library (for side-by-side timing of two builds)
LIB_PATH = os.environ.get("SFHK_LIB", os.path.join(HERE, "libsfhk.so"))

SFHK_OK, SFHK_E_INVALID, SFHK_E_NOMEM, SFHK_E_DEVICE, SFHK_E_NOT_DONE, SFHK_E_BUDGET = (
    0, -1, -2, -3, -4, -5)
SFHK_FP64, SFHK_FP32_MIXED = 0, 1
SFHK_BIRTH_GTO, SFHK_BIRTH_MODIFIED = 0, 1
# partial-wave filter bits (sfhk_params.pw_mask): bands l in [k - 1/2, k + 1/2), far region
PW_S, PW_P, PW_D, PW_FAR, PW_ALL = 1 << 0, 1 << 1, 1 << 2, 1 << 8, 0x1FF
SFHK_MAX_PRIM = 8


class SfhkError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status} ({msg})")
        self.status = status


class _Potential(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("z_inf", ct.c_double), ("z_in", ct.c_double),
                ("r_scr", ct.c_double), ("soft2", ct.c_double), ("omega_ho", ct.c_double)]


class _Ground(ct.Structure):
    _fields_ = [("l", ct.c_int32), ("n_prim", ct.c_int32), ("alpha", ct.POINTER(ct.c_double)),
                ("coef", ct.POINTER(ct.c_double)), ("ip", ct.c_double)]


class _Pulse(ct.Structure):
    _fields_ = [("e0", ct.c_double), ("omega", ct.c_double), ("n_cycles", ct.c_double),
                ("cep", ct.c_double)]


class _Grid(ct.Structure):
    _fields_ = [("t_a", ct.c_double), ("h", ct.c_double), ("n_steps", ct.c_int64),
                ("e_half", ct.c_void_p), ("pulse", ct.POINTER(_Pulse))]


class _Params(ct.Structure):
    _fields_ = [("gamma", ct.c_double), ("kay_max", ct.c_double), ("overlap_cut", ct.c_double),
                ("r_fp64", ct.c_double), ("precision", ct.c_int32), ("n_out", ct.c_int64),
                ("velocity", ct.c_int32), ("pw_mask", ct.c_int32), ("pw_radius", ct.c_double),
                ("compact_every", ct.c_int32)]


class _Stats(ct.Structure):
    _fields_ = [("n_traj", ct.c_int64), ("n_steps", ct.c_int64), ("steps_evaluated", ct.c_int64),
                ("steps_fp64", ct.c_int64), ("kay_removed", ct.c_int64),
                ("nonfinite_removed", ct.c_int64), ("tiles_total", ct.c_int64),
                ("tiles_done", ct.c_int64), ("prims_evaluated", ct.c_int64),
                ("integrands_evaluated", ct.c_int64), ("reserved", ct.c_int64)]


_lib = None

# exported symbols and their signatures (restype, argtypes)
_VP = ct.c_void_p
_SIGS = {
    "sfhk_ctx_create": (ct.c_int, [ct.c_int, ct.c_size_t, ct.POINTER(_VP)]),
    "sfhk_ctx_destroy": (None, [_VP]),
    "sfhk_ctx_bytes_in_use": (ct.c_size_t, [_VP]),
    "sfhk_job_footprint": (ct.c_size_t, [ct.c_int64, ct.c_int64, ct.c_int64, ct.c_int32,
                                         ct.c_int32]),
    "sfhk_job_create": (ct.c_int, [_VP, ct.POINTER(_Potential), ct.POINTER(_Ground),
                                   ct.POINTER(_Grid), ct.POINTER(_Params), ct.c_int64, _VP, _VP,
                                   _VP, _VP, _VP, ct.POINTER(_VP)]),
    "sfhk_job_destroy": (None, [_VP]),
    "sfhk_propagate": (ct.c_int, [_VP, ct.c_int64, _VP]),
    "sfhk_propagate_many": (ct.c_int, [ct.POINTER(_VP), ct.c_int32, ct.c_int64, _VP]),
    "sfhk_dipole": (ct.c_int, [_VP, _VP, _VP, _VP]),
    "sfhk_velocity": (ct.c_int, [_VP, _VP, _VP, _VP]),
    "sfhk_job_n_out": (ct.c_int64, [_VP]),
    "sfhk_job_is_done": (ct.c_int32, [_VP]),
    "sfhk_job_checkpoint_bytes": (ct.c_int64, [_VP]),
    "sfhk_job_checkpoint": (ct.c_int, [_VP, _VP, _VP]),
    "sfhk_job_restore": (ct.c_int, [_VP, _VP, _VP]),
    "sfhk_spectrum": (ct.c_int, [_VP, ct.c_int64, ct.c_double, ct.c_double, ct.c_double,
                                 ct.c_int64, _VP, _VP, _VP, _VP]),
    "sfhk_spectrum_noalloc": (ct.c_int, [_VP, ct.c_int64, ct.c_double, ct.c_double, ct.c_double,
                                         ct.c_int64, _VP, _VP, _VP, _VP]),
    "sfhk_job_stats": (ct.c_int, [_VP, ct.POINTER(_Stats), _VP]),
    "sfhk_job_trajectories": (ct.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "sfhk_batch_create": (ct.c_int, [_VP, ct.c_int32, ct.c_int64, ct.c_int64, ct.c_int32,
                                     ct.POINTER(_VP)]),
    "sfhk_batch_set_jobs": (ct.c_int, [_VP, ct.POINTER(_VP), ct.c_int32, _VP]),
    "sfhk_batch_run": (ct.c_int, [_VP, _VP]),
    "sfhk_batch_workers": (ct.c_int32, [_VP]),
    "sfhk_batch_destroy": (None, [_VP]),
    "sfhk_last_error": (ct.c_char_p, []),
    "sfhk_status_string": (ct.c_char_p, [ct.c_int]),
    "sfhk_traj_exp": (ct.c_int, [_VP, _VP, ct.c_int64, _VP]),
    "sfhk_traj_rsqrt": (ct.c_int, [_VP, _VP, ct.c_int64, _VP]),
    "sfhk_traj_sincos": (ct.c_int, [_VP, _VP, _VP, ct.c_int64, _VP]),
    "sfhk_gabor": (ct.c_int, [_VP, ct.c_int64, ct.c_double, ct.c_double, ct.c_double,
                              ct.c_double, ct.c_double, ct.c_int64, ct.c_double, ct.c_int64,
                              _VP, _VP, _VP]),
    "sfhk_sfa_birth": (ct.c_int, [ct.POINTER(_Pulse), ct.POINTER(_Ground), ct.c_int32, ct.c_int64,
                                  _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
}


def exported_symbols() -> list:
    return sorted(_SIGS)


def lib():
    """Load libsfhk.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2601_17164_amd.build` (no CPU fallback exists)")
        L = ct.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int, where: str, not_done_ok: bool = False):
    """Raise SfhkError for a failed call. SFHK_E_NOT_DONE is a normal outcome only of the
    propagation calls (more steps remain); everywhere else it is an error."""
    if status != SFHK_OK and not (not_done_ok and status == SFHK_E_NOT_DONE):
        msg = lib().sfhk_last_error().decode(errors="replace")
        raise SfhkError(status, where, msg)
    return status


def _stream_ptr(stream: Optional[torch.cuda.Stream]):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


def _dptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return ct.c_void_p(t.data_ptr())


class Context:
    """sfhk_ctx: a device and an HBM budget for the jobs it holds."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = _VP()
        _check(lib().sfhk_ctx_create(int(device), int(hbm_budget_bytes), ct.byref(h)),
               "sfhk_ctx_create")
        self.handle = h
        self.device = int(device)
        self._jobs = weakref.WeakSet()  # live jobs: closed before the context

    def bytes_in_use(self) -> int:
        return int(lib().sfhk_ctx_bytes_in_use(self.handle))

    def close(self):
        if self.handle:
            for job in list(self._jobs):
                job.close()
            lib().sfhk_ctx_destroy(self.handle)
            self.handle = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def job_footprint(n_traj: int, n_steps: int, n_out: int = 0, precision: int = SFHK_FP64,
                  velocity: bool = False) -> int:
    return int(lib().sfhk_job_footprint(int(n_traj), int(n_steps), int(n_out), int(precision),
                                        int(bool(velocity))))


@dataclass
class Stats:
    n_traj: int
    n_steps: int
    steps_evaluated: int
    steps_fp64: int
    kay_removed: int
    nonfinite_removed: int
    tiles_total: int
    tiles_done: int
    prims_evaluated: int
    integrands_evaluated: int


class Job:
    """sfhk_job: one SFHK instance (its trajectories' state, dipole sums and field table live in
    HBM until the job is closed)."""

    def __init__(self, ctx: Context, potential, ground, grid_t_a: float, grid_h: float,
                 n_steps: int, e_half: Optional[torch.Tensor], t0: torch.Tensor, q0: torch.Tensor,
                 p0: torch.Tensor, w: Optional[torch.Tensor] = None, gamma: float = 0.5,
                 kay_max: float = 1e30, overlap_cut: float = 60.0, r_fp64: float = 2.0,
                 precision: int = SFHK_FP64, n_out: int = 0,
                 stream: Optional[torch.cuda.Stream] = None, velocity: bool = False,
                 pw_mask: int = 0, pw_radius: float = 3.0, compact_every: int = 0,
                 pulse=None):
        """``e_half`` is the field at the half steps (device, 2 n_steps + 1 values) or None;
        ``pulse`` (e0, omega, n_cycles, cep) has the library tabulate the field, or check the given
        table against it. At least one of the two is needed. ``compact_every`` > 0 (FP64 only)
        regroups the trajectories left by the Kay test every that many steps
        (sfhk_params.compact_every); such a job runs through ``propagate`` only."""
        alpha = np.ascontiguousarray(ground.alpha, dtype=np.float64)
        coef = np.ascontiguousarray(ground.coef, dtype=np.float64)
        pot = _Potential(int(potential.kind), float(potential.z_inf), float(potential.z_in),
                         float(potential.r_scr), float(potential.soft2), float(potential.omega_ho))
        gs = _Ground(int(ground.l), len(alpha), alpha.ctypes.data_as(ct.POINTER(ct.c_double)),
                     coef.ctypes.data_as(ct.POINTER(ct.c_double)), float(ground.ip))
        pl = None
        if pulse is not None:
            pl = _Pulse(float(pulse.e0), float(pulse.omega), float(pulse.n_cycles),
                        float(pulse.cep))
        if e_half is not None and (tuple(e_half.shape) != (2 * int(n_steps) + 1,)
                                   or e_half.dtype != torch.float64):
            raise ValueError("e_half must be float64 of shape (2 n_steps + 1,)")
        grid = _Grid(float(grid_t_a), float(grid_h), int(n_steps), _dptr(e_half),
                     ct.pointer(pl) if pl is not None else None)
        prm = _Params(float(gamma), float(kay_max), float(overlap_cut), float(r_fp64),
                      int(precision), int(n_out), int(bool(velocity)), int(pw_mask),
                      float(pw_radius), int(compact_every))
        n = int(t0.shape[0])
        for name, t, shp in (("t0", t0, (n,)), ("q0", q0, (3, n)), ("p0", p0, (3, n))):
            if tuple(t.shape) != shp or t.dtype != torch.float64:
                raise ValueError(f"{name} must be float64 of shape {shp}")
        if w is not None and (tuple(w.shape) != (2, n) or w.dtype != torch.float64):
            raise ValueError("w must be float64 of shape (2, n) (re, im)")
        h = _VP()
        _check(lib().sfhk_job_create(ctx.handle, ct.byref(pot), ct.byref(gs), ct.byref(grid),
                                     ct.byref(prm), n, _dptr(t0), _dptr(q0), _dptr(p0), _dptr(w),
                                     _stream_ptr(stream), ct.byref(h)), "sfhk_job_create")
        self.handle = h
        self.ctx = ctx
        ctx._jobs.add(self)
        self.n_traj = n
        self.n_steps = int(n_steps)
        self.t_a = float(grid_t_a)
        self.h = float(grid_h)

    @property
    def n_out(self) -> int:
        return int(lib().sfhk_job_n_out(self.handle))

    @property
    def done(self) -> bool:
        """All steps issued (no synchronisation)."""
        return bool(lib().sfhk_job_is_done(self.handle))

    def propagate(self, max_steps: int = 0, stream=None) -> bool:
        """Returns True when every trajectory reached the end of the grid."""
        rc = _check(lib().sfhk_propagate(self.handle, int(max_steps), _stream_ptr(stream)),
                    "sfhk_propagate", not_done_ok=True)
        return rc == SFHK_OK

    def dipole(self, want_f: bool = False, stream=None):
        dev = torch.device("cuda", self.ctx.device)
        d = torch.empty(self.n_out, dtype=torch.float64, device=dev)
        f = torch.empty(2, self.n_steps + 1, dtype=torch.float64, device=dev) if want_f else None
        _check(lib().sfhk_dipole(self.handle, _dptr(d), _dptr(f), _stream_ptr(stream)),
               "sfhk_dipole")
        return (d, f) if want_f else d

    def velocity(self, want_v: bool = False, stream=None):
        """The dipole velocity -2 Re V on the output grid (and V on the step grid, [2, n+1])."""
        dev = torch.device("cuda", self.ctx.device)
        v = torch.empty(self.n_out, dtype=torch.float64, device=dev)
        vf = torch.empty(2, self.n_steps + 1, dtype=torch.float64, device=dev) if want_v else None
        _check(lib().sfhk_velocity(self.handle, _dptr(v), _dptr(vf), _stream_ptr(stream)),
               "sfhk_velocity")
        return (v, vf) if want_v else v

    def stats(self, stream=None) -> Stats:
        s = _Stats()
        _check(lib().sfhk_job_stats(self.handle, ct.byref(s), _stream_ptr(stream)),
               "sfhk_job_stats")
        return Stats(s.n_traj, s.n_steps, s.steps_evaluated, s.steps_fp64, s.kay_removed,
                     s.nonfinite_removed, s.tiles_total, s.tiles_done,
                     s.prims_evaluated, s.integrands_evaluated)

    def checkpoint(self, stream=None) -> torch.Tensor:
        """The job's propagation state as a device byte tensor (sfhk_job_checkpoint)."""
        n = int(lib().sfhk_job_checkpoint_bytes(self.handle))
        buf = torch.empty(n, dtype=torch.uint8, device=f"cuda:{self.ctx.device}")
        _check(lib().sfhk_job_checkpoint(self.handle, _dptr(buf), _stream_ptr(stream)),
               "sfhk_job_checkpoint")
        return buf

    def restore(self, checkpoint: torch.Tensor, stream=None):
        """Load a checkpoint taken from a job of the same inputs (sfhk_job_restore)."""
        if checkpoint.dtype != torch.uint8 or not checkpoint.is_cuda:
            raise ValueError("checkpoint must be a device uint8 tensor")
        _check(lib().sfhk_job_restore(self.handle, _dptr(checkpoint), _stream_ptr(stream)),
               "sfhk_job_restore")

    def trajectories(self, stream=None):
        dev = torch.device("cuda", self.ctx.device)
        y = torch.empty(43, self.n_traj, dtype=torch.float64, device=dev)
        c = torch.empty(2, self.n_traj, dtype=torch.float64, device=dev)
        death = torch.empty(self.n_traj, dtype=torch.int64, device=dev)
        _check(lib().sfhk_job_trajectories(self.handle, _dptr(y), _dptr(c), _dptr(death),
                                           _stream_ptr(stream)), "sfhk_job_trajectories")
        return y, c, death

    def close(self):
        if self.handle:
            lib().sfhk_job_destroy(self.handle)
            self.handle = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def propagate_many(jobs: Sequence[Job], max_steps: int = 0, stream=None) -> bool:
    arr = (_VP * len(jobs))(*[j.handle for j in jobs])
    rc = _check(lib().sfhk_propagate_many(arr, len(jobs), int(max_steps), _stream_ptr(stream)),
                "sfhk_propagate_many", not_done_ok=True)
    return rc == SFHK_OK


class Batch:
    """sfhk_batch: a graph-captured, batched propagation over a job table of fixed capacity.
    workers_per_cu > 0 selects the persistent (queue) form, 0 hardware dispatch."""

    def __init__(self, ctx: Context, max_jobs: int, max_tiles: int, max_steps: int = 0,
                 workers_per_cu: int = 8):
        h = _VP()
        _check(lib().sfhk_batch_create(ctx.handle, int(max_jobs), int(max_tiles), int(max_steps),
                                       int(workers_per_cu), ct.byref(h)), "sfhk_batch_create")
        self.handle = h
        self.ctx = ctx
        self._jobs = []

    @property
    def workers(self) -> int:
        return int(lib().sfhk_batch_workers(self.handle))

    def set_jobs(self, jobs: Sequence[Job], stream=None):
        arr = (_VP * max(1, len(jobs)))(*[j.handle for j in jobs])
        _check(lib().sfhk_batch_set_jobs(self.handle, arr, len(jobs), _stream_ptr(stream)),
               "sfhk_batch_set_jobs")
        self._jobs = list(jobs)

    def run(self, stream=None) -> bool:
        """One graph replay; True when every staged job has finished."""
        rc = _check(lib().sfhk_batch_run(self.handle, _stream_ptr(stream)), "sfhk_batch_run",
                    not_done_ok=True)
        return rc == SFHK_OK

    def close(self):
        if self.handle:
            lib().sfhk_batch_destroy(self.handle)
            self.handle = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tiles_of(inst) -> int:
    return (inst.n_traj + 63) // 64


def spectrum(d: torch.Tensor, t_first: float, dt: float, tau_h: float, n_fft: int = 0,
             stream=None):
    """Hann-windowed Fourier transform of d on the device: returns (omega, power, X complex)."""
    n = int(d.shape[0])
    nf = int(n_fft) if n_fft else n
    nk = nf // 2 + 1
    om = torch.empty(nk, dtype=torch.float64, device=d.device)
    pw = torch.empty(nk, dtype=torch.float64, device=d.device)
    x = torch.empty(nk, 2, dtype=torch.float64, device=d.device)
    _check(lib().sfhk_spectrum(_dptr(d), n, float(t_first), float(dt), float(tau_h), nf,
                               _dptr(om), _dptr(pw), _dptr(x), _stream_ptr(stream)),
           "sfhk_spectrum")
    return om, pw, torch.view_as_complex(x)


SPECTRUM_NOALLOC_MAX_FFT = 65536


def spectrum_noalloc(d: torch.Tensor, t_first: float, dt: float, tau_h: float, n_fft: int = 0,
                     out=None, stream=None):
    """sfhk_spectrum_noalloc: the same transform as ``spectrum`` in the library's fixed working
    memory (the library allocates nothing; n_fft <= SPECTRUM_NOALLOC_MAX_FFT). ``out`` may give
    the (omega, power, X as [nk, 2]) tensors to write; returns (omega, power, X complex)."""
    n = int(d.shape[0])
    nf = int(n_fft) if n_fft else n
    nk = nf // 2 + 1
    if out is None:
        out = (torch.empty(nk, dtype=torch.float64, device=d.device),
               torch.empty(nk, dtype=torch.float64, device=d.device),
               torch.empty(nk, 2, dtype=torch.float64, device=d.device))
    om, pw, x = out
    _check(lib().sfhk_spectrum_noalloc(_dptr(d), n, float(t_first), float(dt), float(tau_h), nf,
                                       _dptr(om), _dptr(pw), _dptr(x), _stream_ptr(stream)),
           "sfhk_spectrum_noalloc")
    return om, pw, torch.view_as_complex(x)


def gabor(d: torch.Tensor, t_first: float, dt: float, sigma: float, tc_first: float,
          tc_step: float, n_c: int, w_step: float, n_w: int, stream=None):
    """sfhk_gabor on the device: returns (|G|^2 [n_c, n_w], G complex [n_c, n_w])."""
    pw = torch.empty(n_c, n_w, dtype=torch.float64, device=d.device)
    g = torch.empty(n_c, n_w, 2, dtype=torch.float64, device=d.device)
    _check(lib().sfhk_gabor(_dptr(d), int(d.shape[0]), float(t_first), float(dt), float(sigma),
                            float(tc_first), float(tc_step), int(n_c), float(w_step), int(n_w),
                            _dptr(pw), _dptr(g), _stream_ptr(stream)), "sfhk_gabor")
    return pw, torch.view_as_complex(g)


def traj_exp(x: torch.Tensor, stream=None) -> torch.Tensor:
    """exp as evaluated inside the screened potential (device)."""
    y = torch.empty_like(x)
    _check(lib().sfhk_traj_exp(_dptr(x), _dptr(y), int(x.numel()), _stream_ptr(stream)),
           "sfhk_traj_exp")
    return y


def traj_rsqrt(x: torch.Tensor, stream=None) -> torch.Tensor:
    """1/sqrt(x) as evaluated on the trajectory path (device)."""
    y = torch.empty_like(x)
    _check(lib().sfhk_traj_rsqrt(_dptr(x), _dptr(y), int(x.numel()), _stream_ptr(stream)),
           "sfhk_traj_rsqrt")
    return y


def traj_sincos(x: torch.Tensor, stream=None):
    """sin, cos as evaluated in the SFA birth step's saddle-point solve (device)."""
    s, c = torch.empty_like(x), torch.empty_like(x)
    _check(lib().sfhk_traj_sincos(_dptr(x), _dptr(s), _dptr(c), int(x.numel()),
                                  _stream_ptr(stream)), "sfhk_traj_sincos")
    return s, c


def sfa_birth(pulse, ground, t0: torch.Tensor, kperp: torch.Tensor,
              u: Optional[torch.Tensor] = None, mode: int = SFHK_BIRTH_GTO, stream=None) -> dict:
    """sfhk_sfa_birth: SFA birth step on the device. ``pulse`` has e0, omega, n_cycles, cep;
    ``ground`` has l, alpha, coef, ip; t0 [n], kperp [2, n], u [n] or None (float64 tensors).
    Returns device tensors q0 [3, n], p0 [3, n], w [2, n] (re, im) and tt [n]."""
    n = int(t0.shape[0])
    if tuple(kperp.shape) != (2, n) or kperp.dtype != torch.float64 or t0.dtype != torch.float64:
        raise ValueError("t0 must be float64 [n] and kperp float64 [2, n]")
    if u is not None and (tuple(u.shape) != (n,) or u.dtype != torch.float64):
        raise ValueError("u must be float64 [n]")
    alpha = np.ascontiguousarray(ground.alpha, dtype=np.float64)
    coef = np.ascontiguousarray(ground.coef, dtype=np.float64)
    gs = _Ground(int(ground.l), len(alpha), alpha.ctypes.data_as(ct.POINTER(ct.c_double)),
                 coef.ctypes.data_as(ct.POINTER(ct.c_double)), float(ground.ip))
    pl = _Pulse(float(pulse.e0), float(pulse.omega), float(pulse.n_cycles), float(pulse.cep))
    dev = t0.device
    out = dict(q0=torch.empty(3, n, dtype=torch.float64, device=dev),
               p0=torch.empty(3, n, dtype=torch.float64, device=dev),
               w=torch.empty(2, n, dtype=torch.float64, device=dev),
               tt=torch.empty(n, dtype=torch.float64, device=dev))
    _check(lib().sfhk_sfa_birth(ct.byref(pl), ct.byref(gs), int(mode), n, _dptr(t0), _dptr(kperp),
                                _dptr(u), _dptr(out["q0"]), _dptr(out["p0"]), _dptr(out["w"]),
                                _dptr(out["tt"]), _stream_ptr(stream)), "sfhk_sfa_birth")
    return out


# ------------------------------------------------------------------------------------------------
# convenience: one instance (see inputs.Instance) end to end on the device
# ------------------------------------------------------------------------------------------------
def to_device(inst, device="cuda:0"):
    """Upload an instance's samples (float64) and its explicit field table, if it has one, to the
    device (a pulse instance's field is tabulated by the library)."""
    dev = torch.device(device)
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    w = None
    if inst.w is not None:
        w = f(np.stack([np.real(inst.w), np.imag(inst.w)]))
    e = f(inst.e_half) if inst.e_half is not None else None
    return dict(e_half=e, t0=f(inst.t0), q0=f(inst.q0), p0=f(inst.p0), w=w)


def make_job(ctx: Context, inst, dev_arrays=None, precision=SFHK_FP64, n_out=None, stream=None,
             r_fp64=2.0, velocity=False, pw_mask=0, pw_radius=3.0, compact_every=0) -> Job:
    a = dev_arrays if dev_arrays is not None else to_device(inst, f"cuda:{ctx.device}")
    return Job(ctx, inst.potential, inst.ground, inst.grid.t_a, inst.grid.h, inst.grid.n_steps,
               a["e_half"], a["t0"], a["q0"], a["p0"], a["w"], inst.gamma, inst.kay_max,
               inst.overlap_cut, r_fp64, precision, inst.n_out if n_out is None else n_out,
               stream, velocity, pw_mask, pw_radius, compact_every,
               pulse=inst.pulse if inst.e_half is None else None)
