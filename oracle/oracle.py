"""ctypes wrapper around the plain FP64 CPU oracle (``sfhk_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py``. The HIP library never imports or calls it, and it never imports the HIP
library.

Each function follows the paper named in ``sfhk_oracle.c``: the trajectory/monodromy/action
propagation and HK prefactor of App. A, the Kay removal of Sec. III.A, the GTO dipole matrix
element of App. C.1, the induced dipole of Eq. (2), and the Hann-windowed transform of App. D.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sfhk_oracle.c")
# SFHK_ORACLE_LIB points the wrapper at another build (the mutation tests use it).
LIB = os.environ.get("SFHK_ORACLE_LIB", os.path.join(HERE, "libsfhk_oracle.so"))

# x86-64 with FMA3 (every Haswell+/Zen host); no contraction, so every rounding is the one
# written in the source.
CFLAGS = ["-O2", "-mfma", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-std=gnu11", "-Wall", "-Wno-unused-function"]


# The same source built with every square root, quotient, exponential, sine and cosine rounded
# once (-DOR_CORRECTLY_ROUNDED) instead of the rounding contract's sequences.
LIB_CR = os.environ.get("SFHK_ORACLE_LIB_CR", os.path.join(HERE, "libsfhk_oracle_cr.so"))


def _compile(out: str, defines=()) -> None:
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, *[f"-D{d}" for d in defines], "-o", tmp, SRC, "-lquadmath", "-lm",
           "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/libsfhk_oracle.so`` (and its correctly rounded
    build ``oracle/libsfhk_oracle_cr.so``)."""
    if force or not os.path.exists(LIB):
        _compile(LIB)
    if force or not os.path.exists(LIB_CR):
        _compile(LIB_CR, ["OR_CORRECTLY_ROUNDED"])
    return LIB


_lib = None
_lib_cr = None


class _Potential(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("z_inf", ct.c_double), ("z_in", ct.c_double),
                ("r_scr", ct.c_double), ("soft2", ct.c_double), ("omega_ho", ct.c_double)]


class _Ground(ct.Structure):
    _fields_ = [("l", ct.c_int32), ("n_prim", ct.c_int32), ("alpha", ct.POINTER(ct.c_double)),
                ("coef", ct.POINTER(ct.c_double)), ("ip", ct.c_double)]


class _HK(ct.Structure):
    _fields_ = [("gamma", ct.c_double), ("kay_max", ct.c_double), ("overlap_cut", ct.c_double),
                ("pw_mask", ct.c_int32), ("pw_radius", ct.c_double), ("kay_whole", ct.c_int32)]


class _Grid(ct.Structure):
    _fields_ = [("t_a", ct.c_double), ("h", ct.c_double), ("n_steps", ct.c_int64),
                ("e_half", ct.POINTER(ct.c_double))]


class _Pulse(ct.Structure):
    _fields_ = [("e0", ct.c_double), ("omega", ct.c_double), ("n_cycles", ct.c_double),
                ("cep", ct.c_double)]


class _Diag(ct.Structure):
    _fields_ = [("n0", ct.POINTER(ct.c_int64)), ("death", ct.POINTER(ct.c_int64)),
                ("y_final", ct.POINTER(ct.c_double)), ("c_final", ct.POINTER(ct.c_double))]


class _Stats(ct.Structure):
    _fields_ = [("steps_evaluated", ct.c_int64), ("kay_removed", ct.c_int64),
                ("nonfinite_removed", ct.c_int64)]


def lib(correctly_rounded: bool = False):
    """The oracle's library; correctly_rounded=True: its build with the plain, once-rounded
    elementary operations."""
    global _lib, _lib_cr
    if correctly_rounded:
        if _lib_cr is None:
            if not os.path.exists(LIB_CR):
                build(force=False)
            _lib_cr = _declare(ct.CDLL(LIB_CR))
            assert _lib_cr.or_correctly_rounded() == 1
        return _lib_cr
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        _lib = _declare(ct.CDLL(LIB))
    return _lib


def _declare(L):
    """Set the argument and result types of the oracle's exported functions."""
    D, P = ct.c_double, ct.POINTER(ct.c_double)
    L.or_exp_cr.restype = D
    L.or_exp_cr.argtypes = [D]
    L.or_exp_cw.restype = D
    L.or_exp_cw.argtypes = [D]
    L.or_rsqrt_c.restype = D
    L.or_rsqrt_c.argtypes = [D]
    for nm in ("or_sin_cr", "or_cos_cr"):
        getattr(L, nm).restype = D
        getattr(L, nm).argtypes = [D]
    L.or_sincos_c.argtypes = [D, P, P]
    L.or_sfa_birth.restype = ct.c_int
    L.or_sfa_birth.argtypes = [ct.POINTER(_Pulse), ct.POINTER(_Ground), ct.c_int32,
                               ct.c_int64, P, P, P, ct.c_int, P, P, P, P]
    for nm in ("or_field_A", "or_field_E", "or_field_intA"):
        getattr(L, nm).restype = D
        getattr(L, nm).argtypes = [D, D, D, D, D]
    L.or_potential_eval.argtypes = [ct.POINTER(_Potential), P, P, P, P]
    L.or_hk_det.argtypes = [P, D, P]
    L.or_overlap.argtypes = [ct.POINTER(_Ground), D, D, P, P, P]
    L.or_propagate.restype = ct.c_int
    L.or_propagate.argtypes = [ct.POINTER(_Potential), ct.POINTER(_Ground), ct.POINTER(_HK),
                               ct.POINTER(_Grid), ct.c_int64, P, P, P, P, ct.c_int, P, P,
                               ct.POINTER(_Diag), ct.POINTER(_Stats)]
    L.or_overlap_v.argtypes = [ct.POINTER(_Ground), D, D, P, P, P]
    L.or_gabor.restype = ct.c_int
    L.or_gabor.argtypes = [P, ct.c_int64, D, D, D, D, D, ct.c_int64, D, ct.c_int64, P, P]
    L.or_trajectory.restype = ct.c_int
    L.or_trajectory.argtypes = [ct.POINTER(_Potential), ct.POINTER(_Ground), ct.POINTER(_HK),
                                ct.POINTER(_Grid), D, P, P, P, P, P, P, P, P,
                                ct.POINTER(ct.c_int8)]
    L.or_dipole.argtypes = [P, ct.c_int64, P]
    L.or_resample.argtypes = [P, ct.c_int64, ct.c_int64, P]
    L.or_spectrum.restype = ct.c_int
    L.or_spectrum.argtypes = [P, ct.c_int64, D, D, D, ct.c_int64, P, P, P]
    L.or_field_table_c.argtypes = [D, D, D, D, D, D, ct.c_int64, P]
    L.or_correctly_rounded.restype = ct.c_int
    L.or_correctly_rounded.argtypes = []
    return L


def _p(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------------------------------------
# problem description
# ------------------------------------------------------------------------------------------
KIND = {"none": 0, "softcore": 1, "screened": 2, "harmonic": 3}


@dataclass
class Potential:
    kind: str = "softcore"
    z_inf: float = 1.0
    z_in: float = 0.0
    r_scr: float = 1.0
    soft2: float = 0.01
    omega_ho: float = 0.0

    def c(self):
        return _Potential(KIND[self.kind], self.z_inf, self.z_in, self.r_scr, self.soft2,
                          self.omega_ho)


@dataclass
class Ground:
    l: int
    alpha: np.ndarray
    coef: np.ndarray
    ip: float
    _keep: list = field(default_factory=list, repr=False)

    def c(self):
        a, c = _f64(self.alpha), _f64(self.coef)
        self._keep = [a, c]
        return _Ground(self.l, len(a), _p(a), _p(c), self.ip)


def exp_cr(x: float) -> float:
    return lib().or_exp_cr(float(x))


def exp_cw(x: float) -> float:
    """The exponential the screened potential uses (Cody-Waite + degree-13 Taylor)."""
    return lib().or_exp_cw(float(x))


def rsqrt_c(x: float) -> float:
    """The reciprocal square root of the trajectory arithmetic."""
    return lib().or_rsqrt_c(float(x))


def sin_cr(x: float) -> float:
    return lib().or_sin_cr(float(x))


def cos_cr(x: float) -> float:
    return lib().or_cos_cr(float(x))


def sincos_c(x: float):
    """The sine and cosine of the SFA saddle-point solve (Cody-Waite + Taylor, degree 17/18)."""
    s, c = ct.c_double(), ct.c_double()
    lib().or_sincos_c(float(x), ct.byref(s), ct.byref(c))
    return s.value, c.value


@dataclass
class SfaBirth:
    q0: np.ndarray   # [3, n]
    p0: np.ndarray   # [3, n]
    w: np.ndarray    # complex [n]
    tt: np.ndarray   # [n] imaginary part of the saddle-point time


def sfa_birth(e0, omega, n_cycles, cep, ground: "Ground", t0, kperp, u=None, mode=0,
              n_threads=0, correctly_rounded=False) -> SfaBirth:
    """SFA birth step (App. A saddle point and tunnel exit, App. B tunnelling element):
    (t0, k_perp) -> (q0, p0, w, t_t); see ``or_sfa_birth`` in ``sfhk_oracle.h``."""
    t0 = _f64(t0)
    kperp = _f64(kperp).reshape(2, -1)
    n = t0.shape[0]
    assert kperp.shape[1] == n
    uu = None if u is None else _f64(u)
    q0, p0, w2, tt = np.zeros((3, n)), np.zeros((3, n)), np.zeros((2, n)), np.zeros(n)
    g = ground.c()
    pl = _Pulse(float(e0), float(omega), float(n_cycles), float(cep))
    rc = lib(correctly_rounded).or_sfa_birth(ct.byref(pl), ct.byref(g), int(mode), n, _p(t0), _p(kperp),
                            None if uu is None else _p(uu), int(n_threads), _p(q0), _p(p0),
                            _p(w2), _p(tt))
    if rc != 0:
        raise ValueError(f"or_sfa_birth failed ({rc})")
    return SfaBirth(q0, p0, w2[0] + 1j * w2[1], tt)


def field_A(t, e0, omega, T, cep=0.0):
    return np.array([lib().or_field_A(float(x), e0, omega, T, cep) for x in np.atleast_1d(t)])


def field_E(t, e0, omega, T, cep=0.0):
    return np.array([lib().or_field_E(float(x), e0, omega, T, cep) for x in np.atleast_1d(t)])


def field_table_c(e0, omega, n_cycles, cep, t_a, h, n_steps, correctly_rounded=False):
    """E_z(t_a + m h/2), m = 0..2 n_steps, in the fixed sequence of ``or_field_table_c`` (the
    table the device tabulates from the same pulse)."""
    out = np.zeros(2 * int(n_steps) + 1)
    lib(correctly_rounded).or_field_table_c(float(e0), float(omega), float(n_cycles), float(cep),
                                           float(t_a), float(h), int(n_steps), _p(out))
    return out


def field_intA(t, e0, omega, T, cep=0.0):
    return np.array([lib().or_field_intA(float(x), e0, omega, T, cep)
                     for x in np.atleast_1d(t)])


def potential_eval(pot: Potential, q):
    q = _f64(q)
    V = np.zeros(1)
    g = np.zeros(3)
    H = np.zeros(9)
    lib().or_potential_eval(ct.byref(pot.c()), _p(q), _p(V), _p(g), _p(H))
    return V[0], g, H.reshape(3, 3)


def hk_det(m36, gamma):
    """det G for a monodromy given as 6 columns (Q(3), P(3)) flattened column-major."""
    m = _f64(m36).reshape(36)
    out = np.zeros(2)
    lib().or_hk_det(_p(m), float(gamma), _p(out))
    return complex(out[0], out[1])


def overlap_v(ground: Ground, gamma, q, p, cut=60.0):
    """<psi0|k_z|p,q,gamma> (App. C.2) in the scale of ``overlap``."""
    q, p = _f64(q), _f64(p)
    out = np.zeros(2)
    g = ground.c()
    lib().or_overlap_v(ct.byref(g), float(gamma), float(cut), _p(q), _p(p), _p(out))
    return complex(out[0], out[1])


def overlap(ground: Ground, gamma, q, p, cut=60.0):
    q, p = _f64(q), _f64(p)
    out = np.zeros(2)
    g = ground.c()
    lib().or_overlap(ct.byref(g), float(gamma), float(cut), _p(q), _p(p), _p(out))
    return complex(out[0], out[1])


@dataclass
class PropagateResult:
    F: np.ndarray          # complex, n_steps+1
    n0: np.ndarray
    death: np.ndarray
    y_final: np.ndarray    # [43, n_traj]
    c_final: np.ndarray    # complex [n_traj]
    steps_evaluated: int
    kay_removed: int
    nonfinite_removed: int
    V: Optional[np.ndarray] = None  # complex, n_steps+1: the dipole velocity (velocity=True)


def propagate(pot: Potential, ground: Ground, e_half, t_a, h, n_steps, t0, q0, p0, w=None,
              gamma=0.5, kay_max=1e30, overlap_cut=60.0, n_threads=0,
              velocity=False, pw_mask=0, pw_radius=3.0,
              correctly_rounded=False, kay_whole=False) -> PropagateResult:
    """Run the oracle over all trajectories; q0, p0 are [3, n] arrays, w is complex [n] or None.
    velocity=True also accumulates the dipole velocity V(t_n) (App. C.2). pw_mask != 0 keeps
    only the steps of the selected partial waves near the core (``or_hk`` in sfhk_oracle.h).
    correctly_rounded=True runs the build whose square roots, quotients and exponentials are
    the plain operations rounded once. kay_whole=True takes the other reading of the Kay removal:
    a trajectory that ever exceeds D_t contributes nothing at all (default: it stops contributing
    from the first step where it does)."""
    L = lib(correctly_rounded)
    e_half = _f64(e_half)
    if len(e_half) != 2 * n_steps + 1:
        raise ValueError("field table must hold 2*n_steps+1 half-step samples")
    t0, q0, p0 = _f64(t0), _f64(q0), _f64(p0)
    n = t0.shape[0]
    assert q0.shape == (3, n) and p0.shape == (3, n)
    wp = None
    if w is not None:
        wa = np.ascontiguousarray(np.stack([np.real(w), np.imag(w)]).astype(np.float64))
        wp = _p(wa)
    f = np.zeros(2 * (n_steps + 1))
    v = np.zeros(2 * (n_steps + 1)) if velocity else None
    n0 = np.zeros(n, dtype=np.int64)
    death = np.zeros(n, dtype=np.int64)
    yf = np.zeros((43, n))
    cf = np.zeros((2, n))
    diag = _Diag(n0.ctypes.data_as(ct.POINTER(ct.c_int64)),
                 death.ctypes.data_as(ct.POINTER(ct.c_int64)), _p(yf), _p(cf))
    st = _Stats()
    grid = _Grid(float(t_a), float(h), int(n_steps), _p(e_half))
    hk = _HK(float(gamma), float(kay_max), float(overlap_cut), int(pw_mask), float(pw_radius),
             int(bool(kay_whole)))
    g = ground.c()
    rc = L.or_propagate(ct.byref(pot.c()), ct.byref(g), ct.byref(hk), ct.byref(grid), n,
                        _p(t0), _p(q0), _p(p0), wp, int(n_threads), _p(f),
                        None if v is None else _p(v), ct.byref(diag), ct.byref(st))
    if rc != 0:
        raise RuntimeError(f"or_propagate failed: {rc}")
    F = f[: n_steps + 1] + 1j * f[n_steps + 1:]
    V = None if v is None else v[: n_steps + 1] + 1j * v[n_steps + 1:]
    return PropagateResult(F, n0, death, yf, cf[0] + 1j * cf[1], st.steps_evaluated,
                           st.kay_removed, st.nonfinite_removed, V)


@dataclass
class TrajectoryRecord:
    y: np.ndarray       # [n_steps+1, 43]
    C: np.ndarray       # complex [n_steps+1]
    f: np.ndarray       # complex [n_steps+1]
    O: np.ndarray       # complex [n_steps+1]
    det: np.ndarray     # complex [n_steps+1]
    alive: np.ndarray   # bool [n_steps+1]


def trajectory(pot: Potential, ground: Ground, e_half, t_a, h, n_steps, t0, q0, p0, w=1.0,
               gamma=0.5, kay_max=1e30, overlap_cut=60.0, pw_mask=0,
               pw_radius=3.0, correctly_rounded=False) -> TrajectoryRecord:
    L = lib(correctly_rounded)
    e_half = _f64(e_half)
    nb = n_steps + 1
    y = np.zeros((nb, 43))
    c = np.zeros((nb, 2))
    f = np.zeros((nb, 2))
    o = np.zeros((nb, 2))
    d = np.zeros((nb, 2))
    al = np.zeros(nb, dtype=np.int8)
    q0, p0 = _f64(q0), _f64(p0)
    wa = np.array([np.real(w), np.imag(w)], dtype=np.float64)
    grid = _Grid(float(t_a), float(h), int(n_steps), _p(e_half))
    hk = _HK(float(gamma), float(kay_max), float(overlap_cut), int(pw_mask), float(pw_radius), 0)
    g = ground.c()
    rc = L.or_trajectory(ct.byref(pot.c()), ct.byref(g), ct.byref(hk), ct.byref(grid),
                         float(t0), _p(q0), _p(p0), _p(wa), _p(y), _p(c), _p(f), _p(o), _p(d),
                         al.ctypes.data_as(ct.POINTER(ct.c_int8)))
    if rc != 0:
        raise RuntimeError("or_trajectory failed")
    cx = lambda a: a[:, 0] + 1j * a[:, 1]
    return TrajectoryRecord(y, cx(c), cx(f), cx(o), cx(d), al.astype(bool))


def dipole(F) -> np.ndarray:
    f = _f64(np.real(F))
    out = np.zeros_like(f)
    lib().or_dipole(_p(f), len(f) - 1, _p(out))
    return out


def resample(d, n_out) -> np.ndarray:
    d = _f64(d)
    out = np.zeros(int(n_out))
    lib().or_resample(_p(d), len(d) - 1, int(n_out), _p(out))
    return out


def spectrum(d, t_first, dt, tau_h, n_fft=0):
    """Returns (omega, power, X) for k = 0..n_fft/2."""
    d = _f64(d)
    n = len(d)
    nf = int(n_fft) if n_fft else n
    nk = nf // 2 + 1
    om, pw, xx = np.zeros(nk), np.zeros(nk), np.zeros(2 * nk)
    rc = lib().or_spectrum(_p(d), n, float(t_first), float(dt), float(tau_h), nf, _p(om),
                           _p(pw), _p(xx))
    if rc != 0:
        raise RuntimeError("or_spectrum failed")
    return om, pw, xx[0::2] + 1j * xx[1::2]


def gabor(d, t_first, dt, sigma, tc_first, tc_step, n_c, w_step, n_w):
    """Gabor transform (see ``or_gabor``): returns (power [n_c, n_w], G complex [n_c, n_w])."""
    d = _f64(d)
    pw = np.zeros((n_c, n_w))
    g = np.zeros((n_c, n_w, 2))
    rc = lib().or_gabor(_p(d), d.shape[0], float(t_first), float(dt), float(sigma),
                        float(tc_first), float(tc_step), int(n_c), float(w_step), int(n_w),
                        _p(pw), _p(g))
    if rc != 0:
        raise ValueError(f"or_gabor failed ({rc})")
    return pw, g[..., 0] + 1j * g[..., 1]
