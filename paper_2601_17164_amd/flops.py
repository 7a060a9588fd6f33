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
  skip test of the GTO element, per step: |p|^2, |q|^2 (10) and the bound p^2 A + q^2 B (3) = 13
  per evaluated integrand (a step of a lane with some primitive within the cut): p.q (5),
      2 gamma q_z (1), the element's final complex product (6), the phase Ip t_n - S, its sincos
      and the product w C O e^{i phase} (24), the complex accumulation (2)            = 38
  GTO element, per evaluated primitive: s-wave 12, p-wave 19

A step that removes the trajectory (Kay) evaluates less than this; such steps are under 1e-4 of
all steps on the benchmark workloads, so every evaluated step is priced at the full count.
"""
from __future__ import annotations

RHS = {0: 30, 1: 39, 2: 62, 3: 33}
RK4_QPS = 85
MONODROMY = 828
HK = 126
SKIP_TEST = 13
INTEGRAND = 38
GTO_PRIM = {0: 12, 1: 19}


def fixed_per_step(pot_kind: int) -> int:
    """FP64 operations of every trajectory-step (integrand and primitives excluded)."""
    return 4 * RHS[pot_kind] + RK4_QPS + MONODROMY + HK + SKIP_TEST


def flops(pot_kind: int, l: int, steps_evaluated: int, prims_evaluated: int,
          integrands_evaluated: int) -> int:
    """Algorithmic FP64 operations of a propagation that evaluated the given counts (steps, GTO
    primitives, and steps whose dipole integrand was evaluated)."""
    return (fixed_per_step(pot_kind) * int(steps_evaluated) + INTEGRAND * int(integrands_evaluated)
            + GTO_PRIM[l] * int(prims_evaluated))


# SFA birth step, saddle-point kernel (same convention; exp, sin, cos, 1/sqrt count 1):
#   Im A(t0 + i tau): three sinh = (w_m tau, exp, 1/e, difference, half) 5 each, combination 7 = 22
#   march step: tau = k dtau (1) + 22 = 23;  bisection step: midpoint (3) + 22 = 25 (16 steps)
#   Newton step: Im A and its derivative from the same exponentials (w_m tau, exp, 1/e, sinh 2,
#   cosh 2: 7 each = 21; combinations 7 + 10), f (1), the step (2) = 41 (4 steps)
#   per sample: three (sin, cos) of w_m t0 + cep (4 each), the frequencies and K (5), kappa^2 (5),
#   kappa (2), dtau (1), t_t (3), three cosh - 1 (8 each), k_z (7), q0_z (10)             = 69
SFA_MARCH_STEP = 23
SFA_BISECT_STEP = 25
SFA_BISECT_STEPS = 16
SFA_NEWTON_STEP = 41
SFA_NEWTON_STEPS = 4
SFA_FIXED = 69


def sfa_saddle_flops(march_steps: int, n_found: int) -> int:
    """Algorithmic FP64 operations of the saddle-point kernel: march_steps is the sum over
    samples of the march index at which the crossing was found (ceil(t_t / dtau))."""
    return (SFA_MARCH_STEP * int(march_steps)
            + (SFA_BISECT_STEP * SFA_BISECT_STEPS + SFA_NEWTON_STEP * SFA_NEWTON_STEPS
               + SFA_FIXED) * int(n_found))
