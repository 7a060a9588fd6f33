/*
 * oracle_sanitize_driver.c -- runs the oracle's entry points on small synthetic cases so the test
 * suite can execute them under AddressSanitizer and UndefinedBehaviorSanitizer (and compare the
 * printed results with a plain build). Test infrastructure only.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/sfhk_oracle.h"

/* inputs only: a 64-bit LCG mapped to (0, 1) and a Box-Muller pair */
static uint64_t lcg = 0x9E3779B97F4A7C15ull;
static double uniform01(void) {
  lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
  return ((double)(lcg >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}
static double normal(void) {
  const double u = uniform01(), v = uniform01();
  return sqrt(-2.0 * log(u)) * cos(6.283185307179586 * v);
}

static double checksum(const double* a, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += fabs(a[i]) * (double)(1 + (i % 7));
  return s;
}

static int run_case(const char* name, const or_potential* pot, const or_ground* gs, double lambda_nm,
                    double intensity, double n_cycles, double dt, int n_birth, int n_per) {
  const double omega = 45.5633525 / lambda_nm, e0 = sqrt(intensity / 3.50944758e16);
  const double T = n_cycles * 6.283185307179586 / omega;
  const int64_t ns = (int64_t)ceil(T / dt);
  const double h = T / (double)ns, t_a = -0.5 * T;
  double* e_half = malloc(sizeof(double) * (size_t)(2 * ns + 1));
  for (int64_t m = 0; m <= 2 * ns; ++m) e_half[m] = or_field_E(t_a + 0.5 * (double)m * h, e0, omega, T, 0.0);
  const int64_t n = (int64_t)n_birth * n_per;
  double *t0 = malloc(sizeof(double) * (size_t)n), *q0 = malloc(sizeof(double) * 3 * (size_t)n),
         *p0 = malloc(sizeof(double) * 3 * (size_t)n);
  for (int b = 0; b < n_birth; ++b)
    for (int k = 0; k < n_per; ++k) {
      const int64_t j = (int64_t)b * n_per + k;
      t0[j] = t_a + ((double)b + 0.5) * T / (double)n_birth;
      for (int i = 0; i < 3; ++i) {
        q0[i * n + j] = normal();
        p0[i * n + j] = 0.5 * normal();
      }
    }
  q0[1 * n + 3] = NAN; /* a non-finite sample: removed and counted, not an error */
  or_hk hk = {0.5, 1e30, 60.0, 0x1FF ^ 0x80, 3.0, 0};
  or_grid grid = {t_a, h, ns, e_half};
  double* f = calloc((size_t)(2 * (ns + 1)), sizeof(double));
  int64_t *n0 = malloc(sizeof(int64_t) * (size_t)n), *death = malloc(sizeof(int64_t) * (size_t)n);
  double *y = malloc(sizeof(double) * 43 * (size_t)n), *c = malloc(sizeof(double) * 2 * (size_t)n);
  or_diag diag = {n0, death, y, c};
  or_stats st;
  double* v = (double*)calloc((size_t)(2 * (ns + 1)), sizeof(double));
  int rc = or_propagate(pot, gs, &hk, &grid, n, t0, q0, p0, NULL, 2, f, v, &diag, &st);
  if (rc) return rc;
  double* d = malloc(sizeof(double) * (size_t)(ns + 1));
  or_dipole(f, ns, d);
  const int64_t n_out = 512;
  double* dr = malloc(sizeof(double) * (size_t)n_out);
  or_resample(d, ns, n_out, dr);
  const int64_t nk = n_out / 2 + 1;
  double *om = malloc(sizeof(double) * (size_t)nk), *pw = malloc(sizeof(double) * (size_t)nk),
         *x = malloc(sizeof(double) * 2 * (size_t)nk);
  rc = or_spectrum(dr, n_out, t_a, T / (double)n_out, 0.5 * T, n_out, om, pw, x);
  if (rc) return rc;
  double *gp = malloc(sizeof(double) * 8 * 16), *gg = malloc(sizeof(double) * 2 * 8 * 16);
  rc = or_gabor(dr, n_out, t_a, T / (double)n_out, 0.1 * T, t_a, T / 8.0, 8, 0.2, 16, gp, gg);
  if (rc) return rc;
  const double gsum = checksum(gp, 8 * 16);
  free(gp);
  free(gg);
  /* one recorded trajectory */
  double *yr = calloc((size_t)(43 * (ns + 1)), sizeof(double)), *cr = calloc((size_t)(2 * (ns + 1)), sizeof(double));
  double *fr = calloc((size_t)(2 * (ns + 1)), sizeof(double)), *orr = calloc((size_t)(2 * (ns + 1)), sizeof(double));
  double* dr2 = calloc((size_t)(2 * (ns + 1)), sizeof(double));
  int8_t* al = calloc((size_t)(ns + 1), sizeof(int8_t));
  const double q1[3] = {q0[0], q0[n], q0[2 * n]}, p1[3] = {p0[0], p0[n], p0[2 * n]}, w1[2] = {1.0, 0.0};
  rc = or_trajectory(pot, gs, &hk, &grid, t0[0], q1, p1, w1, yr, cr, fr, orr, dr2, al);
  if (rc) return rc;
  printf("%s steps=%lld kay=%lld nonfinite=%lld |F|=%.17g |V|=%.17g |d|=%.17g |P|=%.17g |G|=%.17g |y|=%.17g |traj|=%.17g\n",
         name, (long long)st.steps_evaluated, (long long)st.kay_removed,
         (long long)st.nonfinite_removed, checksum(f, 2 * (ns + 1)), checksum(v, 2 * (ns + 1)),
         checksum(dr, n_out), checksum(pw, nk), gsum, checksum(y, 43 * n), checksum(yr, 43 * (ns + 1)));
  free(v);
  free(e_half); free(t0); free(q0); free(p0); free(f); free(n0); free(death); free(y); free(c);
  free(d); free(dr); free(om); free(pw); free(x); free(yr); free(cr); free(fr); free(orr); free(dr2);
  free(al);
  return 0;
}

int main(void) {
  static const double alpha[6] = {0.03, 0.105, 0.3675, 1.28625, 4.501875, 15.7565625};
  static const double coef_s[6] = {0.01, 0.05, 0.2, 0.3, 0.2, 0.05};
  static const double coef_p[6] = {1e-4, 0.046, 0.21, 0.14, 0.2, -0.064};
  or_ground s_wave = {0, 6, alpha, coef_s, 0.5}, p_wave = {1, 6, alpha, coef_p, 0.58};
  or_potential soft = {1, 1.0, 0.0, 1.0, 0.01, 0.0}, scr = {2, 1.0, 17.0, 0.6, 0.01, 0.0};
  int rc = run_case("softcore", &soft, &s_wave, 800.0, 1e14, 2.0, 0.1, 16, 8);
  if (!rc) rc = run_case("screened", &scr, &p_wave, 1600.0, 1.5e14, 2.0, 0.05, 8, 8);
  /* elementary pieces on awkward arguments */
  const double xs[8] = {0.0, -0.0, 1e-310, 5e-324, 1e308, INFINITY, -1.0, NAN};
  double acc = 0.0;
  for (int i = 0; i < 8; ++i) {
    const double a = or_rsqrt_c(xs[i]), b = or_exp_cw(-fabs(xs[i]) * 1e-306), c2 = or_exp_cr(xs[i] * 1e-306);
    acc += (isfinite(a) ? a * 1e-160 : 1.0) + (isfinite(b) ? b : 1.0) + (isfinite(c2) ? c2 : 1.0);
  }
  double m36[36], det[2];
  for (int i = 0; i < 36; ++i) m36[i] = (i % 7 == 0) ? 1.0 : 0.001 * (double)i;
  or_hk_det(m36, 0.5, det);
  double V, g[3], H[9];
  const double q[3] = {0.0, 0.0, 0.0};
  or_potential_eval(&scr, q, &V, g, H);
  printf("pieces %.17g det=(%.17g, %.17g) V0=%.17g\n", acc, det[0], det[1], V);
  /* contract sine/cosine and the SFA birth step (a NaN, a sample without saddle, both modes) */
  double sc = 0.0;
  for (int i = 0; i < 8; ++i) {
    double s, c;
    or_sincos_c(xs[i] * 1e-300 + (double)i, &s, &c);
    sc += (isfinite(s) ? s : 1.0) + (isfinite(c) ? c : 1.0) + or_sin_cr((double)i) + or_cos_cr((double)i);
  }
  const double e0 = sqrt(1e14 / 3.50944758e16), om = 45.5633525 / 800.0;
  or_pulse pl = {e0, om, 2.0, 0.3};
  enum { NB = 7 };
  double bt0[NB] = {0.0, 10.0, -60.0, 25.0, NAN, 0.0, -100.0};
  double kp[2 * NB] = {0.0, 0.1, 0.3, 0.0, 0.0, 1e80, 0.2, 0.0, -0.2, 0.0, 0.05, 0.0, 0.0, 0.1};
  double bq[3 * NB], bp[3 * NB], bw[2 * NB], btt[NB];
  for (int mode = 0; mode < 2 && !rc; ++mode) {
    const or_ground* gsb = mode ? &p_wave : &s_wave;
    rc = or_sfa_birth(&pl, gsb, mode, NB, bt0, kp, NULL, 3, bq, bp, bw, btt);
    double sb = 0.0;
    for (int j = 0; j < NB; ++j)
      if (isfinite(btt[j])) sb += btt[j] + bp[2 * NB + j] + bq[2 * NB + j] + bw[j] + bw[NB + j];
    printf("sfa mode %d: %.17g\n", mode, sb);
  }
  printf("sincos %.17g\n", sc);
  return rc ? 1 : 0;
}
