"""Algorithmic FP64 operation count of one trajectory-step of the hot path.

Convention: +, -, *, /, sqrt, 1/sqrt, exp, sin and cos count 1 each; a fused multiply-add counts
2; negation and comparisons count 0. The reciprocal square root and the exponential of the
trajectory arithmetic count 1 each, however many operations their fixed sequences take. The counts are of the operation sequence the kernels and the
oracle both follow (one RK4 step of the 43 ODEs of App. A, the HK prefactor with its square-root
branch, the GTO dipole element of App. C.1, the phase and the per-step sum of Eq. 2):

  right-hand side, (q, p, S) part incl. the potential's gradient and Hessian, per evaluation:
      soft-core 39, screened 62, harmonic 33, none 30            (x 4 stages)
  RK4 combination: 13 per component for q, p (6 components), 7 for S    = 85
  monodromy: per column 4 Hessian products (15 each) + 6 x 13 combination = 138   (x 6) = 828
  HK prefactor: G (45), det G (64), |det|^2 (3), |det| = |det|^2 rsqrt(|det|^2) (2),
      principal sqrt: w (2), rsqrt w (1), sqrt w (1), Im/(2 sqrt w) (2); branch dot product and
      sign (4), C (2)                                                       = 126
  GTO element, per step: |p|^2, |q|^2, p.q (15), 2 gamma q_z (1), the final complex product (6) = 22
  GTO element, per evaluated primitive: s-wave 12, p-wave 19
  phase Ip t_n - S, sincos and the product w C O e^{i phase}: 24; complex accumulation: 2

A step that removes the trajectory (Kay) evaluates less than this; such steps are under 1e-4 of
all steps on the benchmark workloads, so every evaluated step is priced at the full count.
"""
from __future__ import annotations

RHS = {0: 30, 1: 39, 2: 62, 3: 33}
RK4_QPS = 85
MONODROMY = 828
HK = 126
GTO_FIXED = 22
GTO_PRIM = {0: 12, 1: 19}
PHASE = 24
ACCUM = 2


def fixed_per_step(pot_kind: int) -> int:
    """FP64 operations per trajectory-step excluding the GTO primitives."""
    return 4 * RHS[pot_kind] + RK4_QPS + MONODROMY + HK + GTO_FIXED + PHASE + ACCUM


def flops(pot_kind: int, l: int, steps_evaluated: int, prims_evaluated: int) -> int:
    """Algorithmic FP64 operations of a propagation that evaluated the given counts."""
    return fixed_per_step(pot_kind) * int(steps_evaluated) + GTO_PRIM[l] * int(prims_evaluated)
