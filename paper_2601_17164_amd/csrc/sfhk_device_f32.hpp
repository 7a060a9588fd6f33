// sfhk_device_f32.hpp -- FP32 arithmetic of the mixed-precision form of the SFHK hot path (gfx950).
//
// In the mixed form, q, p and the monodromy M are carried in FP32 and integrated in FP32 away from
// the nucleus; the action is accumulated in FP64 from FP32 Lagrangian values; steps that start
// within r_fp64 of the nucleus run the FP64 step of sfhk_device.hpp on the exactly promoted state
// and are rounded back. The square roots and the exponential here are the hardware FP32
// approximations (v_rsq_f32, v_exp_f32): this path is compared with the FP64 oracle in dB, not bit
// for bit. Packed FP32 instructions are not used (they are disabled for every kernel).
#pragma once
#include "sfhk_device.hpp"

namespace sfhk {

struct PotParamsF {
  float z_inf, z_in, soft2, omega_ho, inv_rscr;
};

struct TrajF {
  float q[3], p[3];
  float M[36];  // same column layout as Traj::M
  double S;
};

// central potential in FP32: grad V = g q, Hess V = g I + c q q^T (the formulas of pot_gc)
__device__ __forceinline__ void pot_gc_f32(int kind, const PotParamsF& P, float x, float y, float z,
                                           float& V, float& g, float& c) {
  const float r2 = __builtin_fmaf(z, z, __builtin_fmaf(y, y, x * x));
  if (kind == POT_SCREENED) {
    const float ir = __builtin_amdgcn_rsqf(r2 + P.soft2);  // 1/rho
    float inv_r = 0.0f, r = 0.0f;
    if (r2 > 0.0f) {
      inv_r = __builtin_amdgcn_rsqf(r2);
      r = r2 * inv_r;
    }
    const float ir2 = ir * ir, ir3 = ir2 * ir;
    const float e = __builtin_amdgcn_exp2f(-(r * P.inv_rscr) * 1.44269504088896341f);
    const float ez = P.z_in * e;
    const float Z = P.z_inf + ez;
    const float d1 = ez * P.inv_rscr, d2 = d1 * P.inv_rscr;
    V = -(Z * ir);
    const float vp = __builtin_fmaf(Z * r, ir3, d1 * ir);
    const float w1 = __builtin_fmaf(-2.0f, r2, P.soft2);
    const float vpp = ((Z * w1) * ir3) * ir2 - __builtin_fmaf(2.0f, (d1 * r) * ir3, d2 * ir);
    if (r2 > 0.0f) {
      g = vp * inv_r;
      c = (vpp - g) * (inv_r * inv_r);
    } else {
      g = vpp;
      c = 0.0f;
    }
  } else if (kind == POT_SOFTCORE) {
    const float u = __builtin_amdgcn_rsqf(r2 + P.soft2);
    const float u2 = u * u, u3 = u2 * u;
    V = -(P.z_inf * u);
    g = P.z_inf * u3;
    c = (-3.0f * P.z_inf) * (u3 * u2);
  } else if (kind == POT_HARMONIC) {
    const float w2 = P.omega_ho * P.omega_ho;
    V = (0.5f * w2) * r2;
    g = w2;
    c = 0.0f;
  } else {
    V = 0.0f;
    g = 0.0f;
    c = 0.0f;
  }
}

struct Hess3F {
  float h00, h11, h22, h01, h02, h12;
};

__device__ __forceinline__ Hess3F hess_from_f32(float g, float c, float x, float y, float z) {
  const float cx = c * x, cy = c * y, cz = c * z;
  return {__builtin_fmaf(cx, x, g), __builtin_fmaf(cy, y, g), __builtin_fmaf(cz, z, g), cx * y, cx * z,
          cy * z};
}

__device__ __forceinline__ void hess_mv_f32(const Hess3F& H, float v0, float v1, float v2, float& t0,
                                            float& t1, float& t2) {
  t0 = __builtin_fmaf(H.h02, v2, __builtin_fmaf(H.h01, v1, H.h00 * v0));
  t1 = __builtin_fmaf(H.h12, v2, __builtin_fmaf(H.h11, v1, H.h01 * v0));
  t2 = __builtin_fmaf(H.h22, v2, __builtin_fmaf(H.h12, v1, H.h02 * v0));
}

// (q, p) right-hand side in FP32; the Lagrangian is returned in FP64 (computed in FP32, promoted)
__device__ __forceinline__ void qp_rhs_f32(int kind, const PotParamsF& P, const float* q, const float* p,
                                           float E, float* kp, double& kS, Hess3F& H) {
  float V, g, c;
  pot_gc_f32(kind, P, q[0], q[1], q[2], V, g, c);
  H = hess_from_f32(g, c, q[0], q[1], q[2]);
  kp[0] = -(g * q[0]);
  kp[1] = -(g * q[1]);
  kp[2] = -__builtin_fmaf(g, q[2], E);
  const float p2 = __builtin_fmaf(p[2], p[2], __builtin_fmaf(p[1], p[1], p[0] * p[0]));
  kS = (double)__builtin_fmaf(-q[2], E, __builtin_fmaf(0.5f, p2, -V));
}

// one classical RK4 step of the 43 ODEs with q, p, M in FP32 and S accumulated in FP64
__device__ __forceinline__ void rk4_step_f32(int kind, const PotParamsF& P, TrajF& T, float ea, float eb,
                                             float ec, float h, float h2, float h6, double h6d) {
  Hess3F H1, H2, H3, H4;
  {
    float accq[3], accp[3], ysq[3], ysp[3], kp[3];
    double kS, accS;
    qp_rhs_f32(kind, P, T.q, T.p, ea, kp, kS, H1);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      accq[i] = T.p[i];
      accp[i] = kp[i];
      ysq[i] = __builtin_fmaf(h2, T.p[i], T.q[i]);
      ysp[i] = __builtin_fmaf(h2, kp[i], T.p[i]);
    }
    accS = kS;
    qp_rhs_f32(kind, P, ysq, ysp, eb, kp, kS, H2);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const float kq = ysp[i];
      accq[i] = __builtin_fmaf(2.0f, kq, accq[i]);
      accp[i] = __builtin_fmaf(2.0f, kp[i], accp[i]);
      ysq[i] = __builtin_fmaf(h2, kq, T.q[i]);
      ysp[i] = __builtin_fmaf(h2, kp[i], T.p[i]);
    }
    accS = SFHK_FMA(2.0, kS, accS);
    qp_rhs_f32(kind, P, ysq, ysp, eb, kp, kS, H3);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const float kq = ysp[i];
      accq[i] = __builtin_fmaf(2.0f, kq, accq[i]);
      accp[i] = __builtin_fmaf(2.0f, kp[i], accp[i]);
      ysq[i] = __builtin_fmaf(h, kq, T.q[i]);
      ysp[i] = __builtin_fmaf(h, kp[i], T.p[i]);
    }
    accS = SFHK_FMA(2.0, kS, accS);
    qp_rhs_f32(kind, P, ysq, ysp, ec, kp, kS, H4);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T.q[i] = __builtin_fmaf(h6, accq[i] + ysp[i], T.q[i]);
      T.p[i] = __builtin_fmaf(h6, accp[i] + kp[i], T.p[i]);
    }
    T.S = SFHK_FMA(h6d, accS + kS, T.S);
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    float* Q = T.M + 6 * j;
    float* Pc = Q + 3;
    float aQ[3], aP[3], sQ[3], sP[3], t[3];
    hess_mv_f32(H1, Q[0], Q[1], Q[2], t[0], t[1], t[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      aQ[i] = Pc[i];
      aP[i] = -t[i];
      sQ[i] = __builtin_fmaf(h2, Pc[i], Q[i]);
      sP[i] = __builtin_fmaf(h2, -t[i], Pc[i]);
    }
    hess_mv_f32(H2, sQ[0], sQ[1], sQ[2], t[0], t[1], t[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const float kQ = sP[i];
      aQ[i] = __builtin_fmaf(2.0f, kQ, aQ[i]);
      aP[i] = __builtin_fmaf(-2.0f, t[i], aP[i]);
      sQ[i] = __builtin_fmaf(h2, kQ, Q[i]);
      sP[i] = __builtin_fmaf(h2, -t[i], Pc[i]);
    }
    hess_mv_f32(H3, sQ[0], sQ[1], sQ[2], t[0], t[1], t[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const float kQ = sP[i];
      aQ[i] = __builtin_fmaf(2.0f, kQ, aQ[i]);
      aP[i] = __builtin_fmaf(-2.0f, t[i], aP[i]);
      sQ[i] = __builtin_fmaf(h, kQ, Q[i]);
      sP[i] = __builtin_fmaf(h, -t[i], Pc[i]);
    }
    hess_mv_f32(H4, sQ[0], sQ[1], sQ[2], t[0], t[1], t[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Q[i] = __builtin_fmaf(h6, aQ[i] + sP[i], Q[i]);
      Pc[i] = __builtin_fmaf(h6, aP[i] - t[i], Pc[i]);
    }
  }
}

struct cplxf {
  float re, im;
};
__device__ __forceinline__ cplxf cmulf(cplxf a, cplxf b) {
  return {__builtin_fmaf(a.re, b.re, -(a.im * b.im)), __builtin_fmaf(a.re, b.im, a.im * b.re)};
}

// det G of the HK prefactor from the FP32 monodromy (G as in hk_det), returned in FP64
__device__ __forceinline__ cplx hk_det_f32(const float* M, float gamma, float inv4g) {
  cplxf G[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float mqq = M[6 * k + i], mpq = M[6 * k + 3 + i];
      const float mqp = M[6 * (3 + k) + i], mpp = M[6 * (3 + k) + 3 + i];
      G[i][k] = {0.5f * (mpp + mqq), __builtin_fmaf(mpq, inv4g, -(gamma * mqp))};
    }
  auto sub = [](cplxf a, cplxf b) { return cplxf{a.re - b.re, a.im - b.im}; };
  const cplxf m0 = sub(cmulf(G[1][1], G[2][2]), cmulf(G[1][2], G[2][1]));
  const cplxf m1 = sub(cmulf(G[1][0], G[2][2]), cmulf(G[1][2], G[2][0]));
  const cplxf m2 = sub(cmulf(G[1][0], G[2][1]), cmulf(G[1][1], G[2][0]));
  // the three cofactor products are summed in FP64 so that |det| up to the Kay limit stays finite
  const cplxf a = cmulf(G[0][0], m0), b = cmulf(G[0][1], m1), d = cmulf(G[0][2], m2);
  return {((double)a.re - (double)b.re) + (double)d.re, ((double)a.im - (double)b.im) + (double)d.im};
}

}  // namespace sfhk
