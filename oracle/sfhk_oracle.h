/*
 * sfhk_oracle.h -- plain FP64 CPU oracle for the strong-field Herman-Kluk (SFHK) hot path.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg may load this library. It shares no code, header, table or constant generator with the
 * HIP path, and the HIP path never calls it.
 *
 * Method: Tran, Truong, Goetz, Le, "Highly accurate semiclassical strong-field Herman-Kluk
 * propagator method for high-harmonic generation" (Sec. II.A and Appendices A, C, D).
 * All quantities are in atomic units.
 */
#ifndef SFHK_ORACLE_H
#define SFHK_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Atomic model potential V_a(r) of the Hamiltonian (App. A).
 *   kind 0 NONE      V = 0 (laser-only: Volkov motion)
 *   kind 1 SOFTCORE  V = -z_inf / sqrt(r^2 + soft2)
 *   kind 2 SCREENED  V = -(z_inf + z_in exp(-r / r_scr)) / sqrt(r^2 + soft2)
 *   kind 3 HARMONIC  V = omega_ho^2 r^2 / 2  (closed-form test case) */
typedef struct {
  int32_t kind;
  double z_inf, z_in, r_scr, soft2, omega_ho;
} or_potential;

/* Ground state psi_0 as a GTO expansion (App. B/C): l = 0 means sum_j c_j exp(-a_j r^2),
 * l = 1 means z sum_j c_j exp(-a_j r^2). ip is the ionization potential I_p. */
typedef struct {
  int32_t l;
  int32_t n_prim;
  const double* alpha;
  const double* coef;
  double ip;
} or_ground;

/* HK / reduction parameters: coherent-state width gamma (App. A), Kay limit D_t on |C|^2
 * (Sec. III.A), overlap skip threshold on -Re(exponent) of each GTO primitive, and the
 * partial-wave filter of the returning trajectories (Sec. III.A): pw_mask = 0 keeps every step;
 * otherwise a step's term counts when r < pw_radius and l = |q x p| lies in a selected band,
 * bit k (k = 0..6) for l in [k - 1/2, k + 1/2) (s, p, d, ... waves; k = 0 is [0, 1/2)), bit 7
 * for l >= 13/2, or, with bit 8, when r >= pw_radius.
 * kay_whole selects the reading of the Kay removal (the paper removes trajectories with
 * |C|^2 > D_t without saying from when): 0, a trajectory stops contributing from the first step
 * where |det G| > D_t and keeps its earlier terms; 1, a trajectory that exceeds D_t at any step
 * is removed entirely and contributes nothing (found by a first pass over the trajectory). */
typedef struct {
  double gamma;
  double kay_max;
  double overlap_cut;
  int32_t pw_mask;
  double pw_radius;
  int32_t kay_whole;
} or_hk;

/* Time grid: t_n = t_a + n h, n = 0..n_steps. The field table holds E_z(t_a + m h / 2),
 * m = 0..2 n_steps. */
typedef struct {
  double t_a;
  double h;
  int64_t n_steps;
  const double* e_half;
} or_grid;

/* Per-trajectory diagnostics (all arrays of length n_traj; any pointer may be NULL). */
typedef struct {
  int64_t* n0;        /* birth step */
  int64_t* death;     /* first step at which the trajectory was removed, -1 if it survived */
  double* y_final;    /* [43][n_traj]: q(3) p(3) M columns (6 x (Q(3) P(3))) S at the last step
                         evaluated (the removal step for removed trajectories) */
  double* c_final;    /* [2][n_traj]: HK prefactor C at the last step it was accepted */
} or_diag;

/* Counters returned by or_propagate. */
typedef struct {
  int64_t steps_evaluated; /* (trajectory, t_n) pairs evaluated, removal steps included */
  int64_t kay_removed;
  int64_t nonfinite_removed;
} or_stats;

/* Correctly rounded exp (computed in binary128 and rounded once). */
double or_exp_cr(double x);
/* The exponential inside the screened potential: Cody-Waite reduction, degree-13 Taylor
 * polynomial, scaling by 2^k; zero below x = -708. Within about 1 ulp of exp. */
double or_exp_cw(double x);
/* The reciprocal square root of the trajectory arithmetic: bit-pattern seed, three Newton steps
 * and a refined final step; within one ulp of 1/sqrt(x). */
double or_rsqrt_c(double x);

/* Correctly rounded sine and cosine (binary128 evaluation rounded once). */
double or_sin_cr(double x);
double or_cos_cr(double x);
/* Sine and cosine of the SFA birth step's saddle-point solve: Cody-Waite reduction by pi/2 in
 * three parts, Taylor polynomials of degree 17 / 18, quadrant select; within about one ulp.
 * |x| >= 2^20 or non-finite x gives NaN. */
void or_sincos_c(double x, double* s, double* c);

/* Laser field of a linearly polarised sin^2 pulse of total duration T centred at t = 0
 * (Sec. II.B, field equation; E = -dA/dt as in App. A):
 *   A(t) = -(E0/omega) cos^2(pi t/T) sin(omega t + cep) for |t| <= T/2, else 0. */
double or_field_A(double t, double e0, double omega, double T, double cep);
double or_field_E(double t, double e0, double omega, double T, double cep);
/* The field table E_z(t_a + m h/2), m = 0..2 n_steps, of the sin^2 pulse (e0, omega, n_cycles,
 * cep) evaluated in a fixed operation sequence with the contract sine and cosine (or_sincos_c), so
 * that an independent implementation of the same sequence gives the same table bit for bit:
 * T = ((2 pi) n_cycles) / omega, t = t_a + m (h / 2); E = 0 where |t| > T/2, otherwise
 * (s1, c1) = sincos(pi t / T), (sx, cx) = sincos(omega t + cep),
 * E = (e0 c1^2) cx - ((e0 pi) / (omega T)) (2 s1 c1) sx, the two products evaluated as written. */
void or_field_table_c(double e0, double omega, double n_cycles, double cep, double t_a, double h,
                      int64_t n_steps, double* e_half);
/* int_{-T/2}^{t} A(t') dt' (closed form; requires omega T != 2 pi). */
double or_field_intA(double t, double e0, double omega, double T, double cep);

/* Potential value, gradient and Hessian at q. */
void or_potential_eval(const or_potential* pot, const double q[3], double* V, double grad[3],
                       double hess[9]);

/* HK prefactor pieces at monodromy M (y layout above, M as 6 columns of 6): returns
 * det G (re, im) of the matrix inside the square root of the HK prefactor. */
void or_hk_det(const double* m36, double gamma, double det[2]);

/* <psi_0 | z | p, q, gamma> for the GTO ground state (App. C.1), overall constant 1. */
void or_overlap(const or_ground* gs, double gamma, double cut, const double q[3],
                const double p[3], double out[2]);

/* <psi0|k_z|p, q, gamma> for the GTO ground state (App. C.2), in the scale of or_overlap (the
 * ratio of the two elements' written-out constants kept: printed forms times 2 for s, 4 i gamma
 * for p). */
void or_overlap_v(const or_ground* gs, double gamma, double cut, const double q[3],
                  const double p[3], double out[2]);

/* Propagate n_traj trajectories and accumulate F(t_n) = sum_j f_j(t_n) (complex) into
 * f_out[2][n_steps+1] (re block then im block) and, when v_out is not NULL, the dipole velocity
 * V(t_n) = sum_j w_j C <psi0|k_z|p_t,q_t,gamma> e^{i(S - Ip t_n)} (App. C.2, or_overlap_v) into
 * v_out[2][n_steps+1]. q0, p0 are [3][n_traj] (SoA). w is
 * [2][n_traj] complex birth weights or NULL for exp(i p0.q0)/n_traj.
 * n_threads <= 0 uses every online CPU. Returns 0 or a negative error code. */
int or_propagate(const or_potential* pot, const or_ground* gs, const or_hk* hk,
                 const or_grid* grid, int64_t n_traj, const double* t0, const double* q0,
                 const double* p0, const double* w, int n_threads, double* f_out,
                 double* v_out, or_diag* diag, or_stats* stats);

/* Record one trajectory at every step n = 0..n_steps (entries before its birth step are 0):
 * y_rec[(n_steps+1)][43], c_rec/f_rec/o_rec/det_rec[(n_steps+1)][2], alive_rec[n_steps+1]. */
int or_trajectory(const or_potential* pot, const or_ground* gs, const or_hk* hk,
                  const or_grid* grid, double t0, const double q0[3], const double p0[3],
                  const double w[2], double* y_rec, double* c_rec, double* f_rec, double* o_rec,
                  double* det_rec, int8_t* alive_rec);

/* Linearly polarised (z) sin^2 pulse, A(t) = -(e0/omega) cos^2(pi t/T) sin(omega t + cep) with
 * T = 2 pi n_cycles / omega (Sec. II.B field; E = -dA/dt). */
typedef struct {
  double e0, omega, n_cycles, cep;
} or_pulse;

/* SFA birth step (App. A: saddle-point equation, tunnel exit, action under the barrier; App. B:
 * tunnelling matrix elements). For each sample j with birth time t0[j] and transverse momentum
 * kperp = [2][n] (kx, ky): the saddle point t_s = t0 + i t_t of [k + A(t_s) - A(t0)]^2/2 + Ip = 0
 * nearest the real axis, with k = p0 = (kx, ky, k_z); the tunnel exit q0 = (0, 0,
 * Re int_{t_s}^{t0} A); S_down = Ip t_s - int_{t_s}^{t0} [k + A - A(t0)]^2/2; and the weight
 *   w = u e^{i p0.q0} (-i) sqrt(2 pi i / (E(t_s).k_s)) <k_s| r.E(t_s) |psi0> e^{i S_down}
 * (mode 0, Eq. A.2 with the GTO element of App. B.1 and its constant written out), or
 *   w = u e^{i p0.q0} e^{i S_down} / (E(t_s).k_s)   (mode 1, modified saddle point, App. B.2),
 * k_s = k + A(t_s) - A(t0). u = [n] Monte-Carlo weights or NULL for 1/n. Outputs q0, p0 [3][n],
 * w [2][n] (re, im), tt [n] (t_t; may be NULL). A sample whose saddle is not found gets NaN.
 * Requires n_cycles > 1. Returns 0 or a negative error code. */
int or_sfa_birth(const or_pulse* pulse, const or_ground* gs, int32_t mode, int64_t n,
                 const double* t0, const double* kperp, const double* u, int n_threads,
                 double* q0, double* p0, double* w, double* tt);

/* d = -2 Re F on the step grid (Eq. 2 and App. C.1: "+ c.c." with a leading minus). */
void or_dipole(const double* f, int64_t n_steps, double* d_out);

/* Linear interpolation of d (n_steps+1 points, t_n = t_a + n h, h = T / n_steps) onto
 * t_k = t_a + k T / n_out, k = 0..n_out-1. */
void or_resample(const double* d, int64_t n_steps, int64_t n_out, double* out);

/* Hann-windowed Fourier transform (App. D):
 *   X_k = dt sum_n d_n W_H(t_n) exp(i omega_k t_n),  t_n = t_first + n dt,
 *   W_H(t) = (1 + cos(pi t / tau_h)) / 2,  omega_k = 2 pi k / (n_fft dt),  k = 0..n_fft/2,
 * with d zero-padded to n_fft samples. Direct O(n_fft^2) sum. x_out may be NULL. */
int or_spectrum(const double* d, int64_t n, double t_first, double dt, double tau_h,
                int64_t n_fft, double* omega_out, double* power_out, double* x_out);

/* Gabor time-frequency transform (the emission-time analysis of Sec. III.A):
 *   G(t_c, w_k) = dt sum_n d_n exp(-(t_n - t_c)^2 / (2 sigma^2)) exp(i w_k t_n),
 * t_n = t_first + n dt (n samples), t_c = tc_first + c tc_step (c < n_c), w_k = k w_step (k < n_w).
 * power_out[n_c][n_w] = |G|^2; g_out (nullable) [n_c][n_w][2] = (Re G, Im G). Direct sum over
 * every sample. Returns 0 or a negative error code (sigma <= 0, dt <= 0, negative counts). */
int or_gabor(const double* d, int64_t n, double t_first, double dt, double sigma, double tc_first,
             double tc_step, int64_t n_c, double w_step, int64_t n_w, double* power_out,
             double* g_out);

#ifdef __cplusplus
}
#endif
#endif
