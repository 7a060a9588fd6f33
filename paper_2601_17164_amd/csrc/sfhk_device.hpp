// sfhk_device.hpp -- device arithmetic of the SFHK hot path (gfx950, FP64).
//
// Rounding contract. Trajectories of the near-core workloads are chaotic: one rounding difference
// in q, p or the monodromy grows to O(1) within the pulse. Every operation on the trajectory path
// (equations of motion, RK4 combination, det G, Kay test, square-root branch) is therefore written
// as an explicit sequence of IEEE-754 binary64 operations with round-to-nearest-even: +, -, *, /,
// sqrt, and __builtin_fma where a fused multiply-add is part of the sequence. This file must be
// compiled with -ffp-contract=off so the compiler adds no fusion of its own. gfx950's binary64
// division is correctly rounded, and the square roots and the screened potential's exponential
// are fixed sequences of such operations (rsqrt_c and exp_cw below), so a CPU implementation of
// the same sequence agrees bit for bit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>


#define SFHK_FMA(a, b, c) __builtin_fma((a), (b), (c))

namespace sfhk {

// ----------------------------------------------------------------------------------------------
// the exponential of the rounding contract (inside the screened potential). Cody-Waite argument
// reduction x = k ln2 + r, ln2 = kLn2Hi + kLn2Lo with kLn2Hi holding 32 significant bits; exp(r)
// by the degree-13 Taylor polynomial in Horner form with fused multiply-adds; scaling by 2^k.
// Results below 2^-1021 are flushed to zero (x < -708), so the scaling is always exact. Within
// about one ulp of exp; no tables and no memory traffic.
// ----------------------------------------------------------------------------------------------
struct InvFactorials {
  double v[14];
  constexpr InvFactorials() : v() {
    double f = 1.0;
    for (int n = 0; n < 14; ++n) {
      if (n > 0) f *= (double)n;  // n! is exact in binary64 for n <= 18
      v[n] = 1.0 / f;             // correctly rounded quotient (evaluated by the compiler)
    }
  }
};
constexpr InvFactorials kInvFact{};

// fma(a, b, c) as the three-operand v_fma_f64: under the propagate kernel's register pressure
// the compiler otherwise emits a copy of the addend plus the two-operand v_fmac_f64 for every
// Horner step. Same IEEE fused multiply-add, one instruction.
__device__ __forceinline__ double fma3(double a, double b, double c) {
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}

// the sequence alone: exp_cw for arguments in [-708, 709] (a NaN runs through and stays NaN)
__device__ __forceinline__ double exp_cw_core(double x) {
  constexpr double kInvLn2 = 0x1.71547652b82fep+0;  // 1/ln2 rounded to binary64
  constexpr double kLn2Hi = 0x1.62e42feep-1;         // ln2 truncated to 32 significant bits
  constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;   // ln2 - kLn2Hi rounded to binary64
  const double k = rint(x * kInvLn2);
  double r = SFHK_FMA(-k, kLn2Hi, x);
  r = SFHK_FMA(-k, kLn2Lo, r);
  double p = kInvFact.v[13];
#pragma unroll
  for (int n = 12; n >= 3; --n) p = fma3(p, r, kInvFact.v[n]);
#pragma unroll
  for (int n = 2; n >= 0; --n) p = SFHK_FMA(p, r, kInvFact.v[n]);  // 1/2, 1, 1: inline constants
  return ldexp(p, (int)k);
}

// exp_cw on x <= 0 (and NaN)
__device__ __forceinline__ double exp_cw_nonpos(double x) {
  const double y = exp_cw_core(x);
  return x < -708.0 ? 0.0 : y;
}

// the sequence runs for every x; the three out-of-range cases are selected afterwards
__device__ __forceinline__ double exp_cw(double x) {
  double y = exp_cw_core(x);
  y = x < -708.0 ? 0.0 : y;
  y = x > 709.0 ? __builtin_inf() : y;
  return x != x ? x : y;
}

// ----------------------------------------------------------------------------------------------
// the reciprocal square root of the rounding contract: the binary64 bit-pattern seed with magic
// constant 0x5FE6EB50C7B537A9 (Lomont; relative error below 3.5%), three Newton steps
// y <- y (3/2 - (x/2) y^2) and a final step y + y (1/2 - (x/2) y^2); within one ulp of 1/sqrt(x).
// About 16 VALU operations, against about 36 for a correctly rounded sqrt followed by a division.
// Arguments outside [2^-1000, 2^1000] are scaled by an even power of two first (exact).
// ----------------------------------------------------------------------------------------------
__device__ __forceinline__ double rsqrt_core(double x) {
  const unsigned long long b = __double_as_longlong(x);
  double y = __longlong_as_double(0x5FE6EB50C7B537A9ULL - (b >> 1));
  const double h = 0.5 * x;
#pragma unroll
  for (int it = 0; it < 3; ++it) y = y * SFHK_FMA(-h, y * y, 1.5);
  return SFHK_FMA(y, SFHK_FMA(-h, y * y, 0.5), y);
}

__device__ __forceinline__ double rsqrt_rare(double x) {
  if (x != x || x < 0.0) return __builtin_nan("");
  if (x == 0.0) return __builtin_inf();
  if (x == __builtin_inf()) return 0.0;
  if (x < 0x1p-1000) return rsqrt_core(x * 0x1p1000) * 0x1p500;
  return rsqrt_core(x * 0x1p-1000) * 0x1p-500;
}

// rsqrt_c per lane, for code that already runs only on lanes with special cases
__device__ __forceinline__ double rsqrt_lane(double x) {
  return (x >= 0x1p-1000 && x <= 0x1p1000) ? rsqrt_core(x) : rsqrt_rare(x);
}

// The in-range sequence runs unconditionally; lanes outside [2^-1000, 2^1000] are redone under a
// wave-uniform test, so the common path has no divergent branch to merge.
__device__ __forceinline__ double rsqrt_c(double x) {
  double y = rsqrt_core(x);
  const bool rare = !(x >= 0x1p-1000 && x <= 0x1p1000);
  if (__builtin_expect(__any(rare), 0)) {
    if (rare) y = rsqrt_rare(x);
  }
  return y;
}

// ----------------------------------------------------------------------------------------------
// atomic model potential V_a (App. A): central, grad V = g q, Hess V = g I + c q q^T
// ----------------------------------------------------------------------------------------------
enum PotKind : int { POT_NONE = 0, POT_SOFTCORE = 1, POT_SCREENED = 2, POT_HARMONIC = 3 };

struct PotParams {
  double z_inf, z_in, r_scr, soft2, omega_ho;
  double inv_rscr;  // 1 / r_scr (correctly rounded quotient)
  // screened potential: for 2^-1000 <= r^2 <= r2_fast both square roots are in the core range of
  // rsqrt_c (set by the host; -1 disables the fast form)
  double r2_fast;
};

// The screened potential's terms. FAST: the sequence for lanes with 2^-1000 <= r^2 <= r2_fast,
// where the square roots' range tests and the r = 0 selects of the careful form are known to
// pick the ordinary branch, so both forms give the same bits there; the careful form keeps every
// special case. Both keep the exponential's underflow select: distant trajectories hit it often.
template <bool FAST>
__device__ __forceinline__ void screened_terms(const PotParams& P, double r2, double& V, double& g,
                                               double& c) {
  // V = -Z(r)/rho, Z = z_inf + z_in exp(-r/r_scr), rho = (r^2 + a)^(1/2)
  double s = r2 + P.soft2;
  double ir = FAST ? rsqrt_core(s) : rsqrt_lane(s);  // 1/rho
  const bool pos = FAST || r2 > 0.0;
  const double inv_r = FAST ? rsqrt_core(r2) : rsqrt_lane(r2);  // +inf at r = 0, unused there
  const double r = pos ? r2 * inv_r : 0.0;
  double ir2 = ir * ir;
  double ir3 = ir2 * ir;
  const double xe = -(r * P.inv_rscr);
  double e = 0.0;  // exp_cw_nonpos gives exactly 0 below -708: a wave with every lane there skips it
  if (!FAST || __any(!(xe < -708.0))) e = exp_cw_nonpos(xe);
  double ez = P.z_in * e;
  double Z = P.z_inf + ez;
  double d1 = ez * P.inv_rscr;  // -Z'
  double d2 = d1 * P.inv_rscr;  //  Z''
  V = -(Z * ir);
  double vp = SFHK_FMA(Z * r, ir3, d1 * ir);           // V'
  double w1 = SFHK_FMA(-2.0, r2, P.soft2);             // a - 2 r^2
  double ta = d2 * ir;
  double tb = (d1 * r) * ir3;
  double tc = ((Z * w1) * ir3) * ir2;
  double vpp = tc - SFHK_FMA(2.0, tb, ta);             // V''
  const double gp = vp * inv_r;
  const double cp = (vpp - gp) * (inv_r * inv_r);
  g = pos ? gp : vpp;  // r = 0 exactly (measure zero): finite isotropic choice
  c = pos ? cp : 0.0;
}

// r^2 = x^2 + y^2 + z^2 in the contract's order
__device__ __forceinline__ double norm2(double x, double y, double z) {
  double r2 = x * x;
  r2 = SFHK_FMA(y, y, r2);
  return SFHK_FMA(z, z, r2);
}

// V, g, c of the central potential at radius^2 r2 = norm2(q)
template <int KIND>
__device__ __forceinline__ void pot_gc(const PotParams& P, double r2, double& V, double& g, double& c) {
  if constexpr (KIND == POT_SOFTCORE) {
    // V = -Z u, u = (r^2 + a)^(-1/2); dV/dr / r = Z u^3; (V'' - V'/r)/r^2 = -3 Z u^5
    double s = r2 + P.soft2;
    double u = rsqrt_c(s);
    double u2 = u * u;
    double u3 = u2 * u;
    double u5 = u3 * u2;
    V = -(P.z_inf * u);
    g = P.z_inf * u3;
    c = (-3.0 * P.z_inf) * u5;
  } else if constexpr (KIND == POT_SCREENED) {
    // lanes outside the fast range are redone in the careful form under a wave-uniform test
    screened_terms<true>(P, r2, V, g, c);
    const bool slow = !(r2 >= 0x1p-1000 && r2 <= P.r2_fast);
    if (__builtin_expect(__any(slow), 0)) {
      if (slow) screened_terms<false>(P, r2, V, g, c);
    }
  } else if constexpr (KIND == POT_HARMONIC) {
    double w2 = P.omega_ho * P.omega_ho;
    V = (0.5 * w2) * r2;
    g = w2;
    c = 0.0;
  } else {
    V = 0.0;
    g = 0.0;
    c = 0.0;
  }
}

// kind known only at run time (uniform across the wave): a scalar branch per evaluation
__device__ __forceinline__ void pot_gc_rt(int kind, const PotParams& P, double r2, double& V,
                                          double& g, double& c) {
  if (kind == POT_SCREENED)
    pot_gc<POT_SCREENED>(P, r2, V, g, c);
  else if (kind == POT_SOFTCORE)
    pot_gc<POT_SOFTCORE>(P, r2, V, g, c);
  else if (kind == POT_HARMONIC)
    pot_gc<POT_HARMONIC>(P, r2, V, g, c);
  else
    pot_gc<POT_NONE>(P, r2, V, g, c);
}

struct Hess3 {
  double h00, h11, h22, h01, h02, h12;
};

__device__ __forceinline__ Hess3 hess_from(double g, double c, double x, double y, double z) {
  double cx = c * x, cy = c * y, cz = c * z;
  Hess3 H;
  H.h00 = SFHK_FMA(cx, x, g);
  H.h11 = SFHK_FMA(cy, y, g);
  H.h22 = SFHK_FMA(cz, z, g);
  H.h01 = cx * y;
  H.h02 = cx * z;
  H.h12 = cy * z;
  return H;
}

// (H v)_i with the row order of the contract: H_i0 v0, then + H_i1 v1, then + H_i2 v2
__device__ __forceinline__ void hess_mv(const Hess3& H, double v0, double v1, double v2, double& t0,
                                        double& t1, double& t2) {
  t0 = H.h00 * v0;
  t0 = SFHK_FMA(H.h01, v1, t0);
  t0 = SFHK_FMA(H.h02, v2, t0);
  t1 = H.h01 * v0;
  t1 = SFHK_FMA(H.h11, v1, t1);
  t1 = SFHK_FMA(H.h12, v2, t1);
  t2 = H.h02 * v0;
  t2 = SFHK_FMA(H.h12, v1, t2);
  t2 = SFHK_FMA(H.h22, v2, t2);
}

// ----------------------------------------------------------------------------------------------
// one classical RK4 step of the 43 ODEs (App. A): qdot = p, pdot = -grad V - E z^,
// Qdot_j = P_j, Pdot_j = -Hess V Q_j, Sdot = p^2/2 - V - z E. The (q, p, S) stages run first and
// leave the four stage Hessians; the six monodromy columns then take their RK4 step with them.
// Every component sees exactly the operation sequence of a plain 43-component RK4:
//   ys = fma(c, k, y); acc = fma(2, k2, k1); acc = fma(2, k3, acc); acc += k4; y = fma(h/6, acc, y)
// ----------------------------------------------------------------------------------------------
struct Traj {
  double q[3], p[3], S;
  double M[36];  // 6 columns (Q(3), P(3)): column j = d(q_t, p_t)/d z_j, z = (q0, p0)
};

// the (q, p, S) right-hand side; q2 = norm2(q), p2 = norm2(p)
__device__ __forceinline__ void qps_rhs(int kind, const PotParams& P, const double* q, double q2,
                                        double p2, double E, double* kp, double& kS, Hess3& H) {
  double V, g, c;
  pot_gc_rt(kind, P, q2, V, g, c);
  H = hess_from(g, c, q[0], q[1], q[2]);
  kp[0] = -(g * q[0]);
  kp[1] = -(g * q[1]);
  kp[2] = -SFHK_FMA(g, q[2], E);
  double L = SFHK_FMA(0.5, p2, -V);
  kS = SFHK_FMA(-q[2], E, L);
}

__device__ __forceinline__ void qps_rhs(int kind, const PotParams& P, const double* q, const double* p,
                                        double E, double* kp, double& kS, Hess3& H) {
  qps_rhs(kind, P, q, norm2(q[0], q[1], q[2]), norm2(p[0], p[1], p[2]), E, kp, kS, H);
}

// q2 = norm2(T.q) and p2 = norm2(T.p) of the state the step starts from (the caller has them)
__device__ __forceinline__ void rk4_step(int kind, const PotParams& P, Traj& T, double q2, double p2,
                                         double ea, double eb, double ec, double h, double h2,
                                         double h6) {
  Hess3 H1, H2, H3, H4;
  {
    double accq[3], accp[3], accS, ysq[3], ysp[3], ysS, kp[3], kS;
    // stage 1
    qps_rhs(kind, P, T.q, q2, p2, ea, kp, kS, H1);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      accq[i] = T.p[i];
      accp[i] = kp[i];
      ysq[i] = SFHK_FMA(h2, T.p[i], T.q[i]);
      ysp[i] = SFHK_FMA(h2, kp[i], T.p[i]);
    }
    accS = kS;
    ysS = SFHK_FMA(h2, kS, T.S);
    // stage 2
    qps_rhs(kind, P, ysq, ysp, eb, kp, kS, H2);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double kq = ysp[i];
      accq[i] = SFHK_FMA(2.0, kq, accq[i]);
      accp[i] = SFHK_FMA(2.0, kp[i], accp[i]);
      ysq[i] = SFHK_FMA(h2, kq, T.q[i]);
      ysp[i] = SFHK_FMA(h2, kp[i], T.p[i]);
    }
    accS = SFHK_FMA(2.0, kS, accS);
    ysS = SFHK_FMA(h2, kS, T.S);
    // stage 3
    qps_rhs(kind, P, ysq, ysp, eb, kp, kS, H3);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double kq = ysp[i];
      accq[i] = SFHK_FMA(2.0, kq, accq[i]);
      accp[i] = SFHK_FMA(2.0, kp[i], accp[i]);
      ysq[i] = SFHK_FMA(h, kq, T.q[i]);
      ysp[i] = SFHK_FMA(h, kp[i], T.p[i]);
    }
    accS = SFHK_FMA(2.0, kS, accS);
    ysS = SFHK_FMA(h, kS, T.S);
    (void)ysS;
    // stage 4
    qps_rhs(kind, P, ysq, ysp, ec, kp, kS, H4);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      accq[i] = accq[i] + ysp[i];
      accp[i] = accp[i] + kp[i];
      T.q[i] = SFHK_FMA(h6, accq[i], T.q[i]);
      T.p[i] = SFHK_FMA(h6, accp[i], T.p[i]);
    }
    accS = accS + kS;
    T.S = SFHK_FMA(h6, accS, T.S);
  }
  // monodromy columns
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double* Q = T.M + 6 * j;
    double* Pc = Q + 3;
    double aQ[3], aP[3], sQ[3], sP[3], t[3];
    hess_mv(H1, Q[0], Q[1], Q[2], t[0], t[1], t[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double kP = -t[i];
      aQ[i] = Pc[i];
      aP[i] = kP;
      sQ[i] = SFHK_FMA(h2, Pc[i], Q[i]);
      sP[i] = SFHK_FMA(h2, kP, Pc[i]);
    }
    hess_mv(H2, sQ[0], sQ[1], sQ[2], t[0], t[1], t[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double kQ = sP[i], kP = -t[i];
      aQ[i] = SFHK_FMA(2.0, kQ, aQ[i]);
      aP[i] = SFHK_FMA(2.0, kP, aP[i]);
      sQ[i] = SFHK_FMA(h2, kQ, Q[i]);
      sP[i] = SFHK_FMA(h2, kP, Pc[i]);
    }
    hess_mv(H3, sQ[0], sQ[1], sQ[2], t[0], t[1], t[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double kQ = sP[i], kP = -t[i];
      aQ[i] = SFHK_FMA(2.0, kQ, aQ[i]);
      aP[i] = SFHK_FMA(2.0, kP, aP[i]);
      sQ[i] = SFHK_FMA(h, kQ, Q[i]);
      sP[i] = SFHK_FMA(h, kP, Pc[i]);
    }
    hess_mv(H4, sQ[0], sQ[1], sQ[2], t[0], t[1], t[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      aQ[i] = aQ[i] + sP[i];
      aP[i] = aP[i] + (-t[i]);
      Q[i] = SFHK_FMA(h6, aQ[i], Q[i]);
      Pc[i] = SFHK_FMA(h6, aP[i], Pc[i]);
    }
  }
}

__device__ __forceinline__ void rk4_step(int kind, const PotParams& P, Traj& T, double ea, double eb,
                                         double ec, double h, double h2, double h6) {
  rk4_step(kind, P, T, norm2(T.q[0], T.q[1], T.q[2]), norm2(T.p[0], T.p[1], T.p[2]), ea, eb, ec, h,
           h2, h6);
}

// ----------------------------------------------------------------------------------------------
// HK prefactor (App. A): G = (M_pp + M_qq)/2 + i (M_pq / (4 gamma) - gamma M_qp), det G by
// cofactors along the first row; complex product (a b)_re = fma(a.re, b.re, -(a.im b.im)),
// (a b)_im = fma(a.re, b.im, a.im b.re)
// ----------------------------------------------------------------------------------------------
struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {SFHK_FMA(a.re, b.re, -(a.im * b.im)), SFHK_FMA(a.re, b.im, a.im * b.re)};
}
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }

__device__ __forceinline__ cplx hk_det(const double* M, double gamma, double inv4g) {
  cplx G[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double mqq = M[6 * k + i], mpq = M[6 * k + 3 + i];
      double mqp = M[6 * (3 + k) + i], mpp = M[6 * (3 + k) + 3 + i];
      G[i][k].re = 0.5 * (mpp + mqq);
      G[i][k].im = SFHK_FMA(mpq, inv4g, -(gamma * mqp));
    }
  cplx m0 = csub(cmul(G[1][1], G[2][2]), cmul(G[1][2], G[2][1]));
  cplx m1 = csub(cmul(G[1][0], G[2][2]), cmul(G[1][2], G[2][0]));
  cplx m2 = csub(cmul(G[1][0], G[2][1]), cmul(G[1][1], G[2][0]));
  return cadd(csub(cmul(G[0][0], m0), cmul(G[0][1], m1)), cmul(G[0][2], m2));
}

// principal square root (cut on the negative real axis) of z with |z| = mod: with
// w = (mod + |Re z|)/2, sqrt w = w rsqrt(w) and 1/(2 sqrt w) = rsqrt(w)/2
__device__ __forceinline__ cplx csqrt_principal(cplx z, double mod) {
  const double w = 0.5 * (mod + fabs(z.re));
  if (w == 0.0) return {0.0, 0.0};
  const double rw = rsqrt_c(w);
  const double t = w * rw;
  if (z.re >= 0.0) return {t, (0.5 * z.im) * rw};
  return {(0.5 * fabs(z.im)) * rw, copysign(t, z.im)};
}

// C = principal square root of d = det G, for a2 = |d|^2 (a lane that passed the Kay test). For
// 2^-1000 <= a2 <= 2^1000 the careful form's tests always pick the ordinary branch (|d| > 0 and
// w = (|d| + |Re d|)/2 within the square root's core range), so both give the same bits there;
// lanes outside are recomputed in the careful form under a wave-uniform test.
__device__ __forceinline__ cplx hk_sqrt(cplx d, double a2) {
  const double mod = a2 * rsqrt_core(a2);
  const double w = 0.5 * (mod + fabs(d.re));
  const double rw = rsqrt_core(w);
  const double t = w * rw;
  cplx c = d.re >= 0.0 ? cplx{t, (0.5 * d.im) * rw} : cplx{(0.5 * fabs(d.im)) * rw, copysign(t, d.im)};
  const bool slow = !(a2 >= 0x1p-1000 && a2 <= 0x1p1000);
  if (__builtin_expect(__any(slow), 0)) {
    if (slow) c = csqrt_principal(d, a2 > 0.0 ? a2 * rsqrt_c(a2) : 0.0);
  }
  return c;
}

}  // namespace sfhk
