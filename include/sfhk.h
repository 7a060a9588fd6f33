/*
 * sfhk.h -- C ABI of the MI355X (gfx950) hot path of the semiclassical strong-field Herman-Kluk
 * (SFHK) method for high-harmonic generation (Tran, Truong, Goetz, Le).
 *
 * The hot path: many independent classical trajectories, each integrating Hamilton's equations of
 * H = p^2/2 + V_a(q) + q.E(t) together with its 6x6 stability (monodromy) matrix and its action
 * (App. A); per time step the Herman-Kluk prefactor and phase of each coherent-state trajectory
 * times the GTO dipole matrix element <psi0|z|p_t,q_t,gamma> (App. C.1), summed into the induced
 * dipole D(t) = -<psi0 e^{i Ip t}|z|psi_c(t)> + c.c. (Eq. 2); then the Hann-windowed Fourier
 * transform of D(t) (App. D).
 *
 * Conventions of every entry point:
 *  - Atomic units. Pointers are DEVICE pointers unless stated otherwise; the caller owns them.
 *  - Calls are asynchronous on the given HIP stream (hipStream_t passed as void*; NULL = the null
 *    stream) unless stated otherwise; results are ready when the stream reaches that point.
 *  - Errors are returned as negative sfhk_status codes; nothing throws across the ABI. The text of
 *    the most recent error on the calling thread is available from sfhk_last_error().
 *  - A context is used from one host thread at a time. Jobs of one context may be propagated from
 *    that thread on any stream; calls that touch the same job must be ordered by the caller.
 */
#ifndef SFHK_H
#define SFHK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SFHK_OK = 0,
  SFHK_E_INVALID = -1,  /* an argument is out of range (message names it) */
  SFHK_E_NOMEM = -2,    /* device allocation failed */
  SFHK_E_DEVICE = -3,   /* a HIP runtime call failed */
  SFHK_E_NOT_DONE = -4, /* sfhk_propagate stopped after max_steps; call again to continue */
  SFHK_E_BUDGET = -5    /* the job does not fit in the context's remaining HBM budget */
} sfhk_status;

/* Atomic model potential V_a (App. A, Hamiltonian of the HK propagation):
 *   SFHK_POT_NONE      V = 0 (laser-only motion)
 *   SFHK_POT_SOFTCORE  V = -z_inf / sqrt(r^2 + soft2)
 *   SFHK_POT_SCREENED  V = -(z_inf + z_in exp(-r / r_scr)) / sqrt(r^2 + soft2)
 *   SFHK_POT_HARMONIC  V = omega_ho^2 r^2 / 2 (closed-form test case) */
typedef enum { SFHK_POT_NONE = 0, SFHK_POT_SOFTCORE = 1, SFHK_POT_SCREENED = 2, SFHK_POT_HARMONIC = 3 } sfhk_pot_kind;

/* SFHK_FP64: every step in FP64 under the rounding contract. SFHK_FP32_MIXED: position, momentum
 * and monodromy integrated in FP32 away from the nucleus (steps that start at r < r_fp64 in FP64),
 * the action, the HK square root and branch, the dipole integrand and the per-step sums in FP64.
 * The FP32 state resolves trajectories stretched by up to a few hundred: on the screened-potential
 * workload with SFA-born samples its spectra stay within -40 dB of the FP64 ones in the plateau
 * and cutoff bands up to kay_max = 1e6 (at 1e8: -43 dB plateau, -16 dB cutoff); with larger
 * limits the contributions of strongly stretched trajectories, which FP32 cannot integrate, make
 * the difference O(1). */
typedef enum { SFHK_FP64 = 0, SFHK_FP32_MIXED = 1 } sfhk_precision;

typedef struct {
  int32_t kind;
  double z_inf, z_in, r_scr, soft2, omega_ho;
} sfhk_potential;

/* Ground state psi0 as GTOs (App. B.1/C.1): l = 0: sum_j coef_j exp(-alpha_j r^2);
 * l = 1: z sum_j coef_j exp(-alpha_j r^2). alpha/coef are HOST arrays of n_prim <= SFHK_MAX_PRIM
 * entries, read during sfhk_job_create. ip is the ionization potential I_p. */
#define SFHK_MAX_PRIM 8
typedef struct {
  int32_t l;
  int32_t n_prim;
  const double* alpha;
  const double* coef;
  double ip;
} sfhk_ground;

/* A linearly polarised sin^2 pulse along z (Sec. II.B field; App. A): vector potential
 * A(t) = -(e0/omega) cos^2(pi t/T) sin(omega t + cep) for |t| <= T/2 (else 0),
 * T = 2 pi n_cycles / omega, and field E = -dA/dt. */
typedef struct {
  double e0, omega, n_cycles, cep;
} sfhk_pulse;

/* Time grid and laser field (Sec. II.B field, linear polarisation along z): t_n = t_a + n h,
 * n = 0..n_steps. The propagation reads E_z at the half steps t_a + m h/2, m = 0..2 n_steps:
 *  - pulse given, e_half NULL: the library tabulates the pulse's field on the device, in the fixed
 *    sequence T = ((2 pi) n_cycles) / omega, t = t_a + m (h / 2); E = 0 where |t| > T/2, else
 *    (s1, c1) = sincos(pi t / T), (sx, cx) = sincos(omega t + cep),
 *    E = (e0 c1^2) cx - ((e0 pi) / (omega T)) (2 s1 c1) sx (each product as written), with the
 *    sine and cosine of sfhk_traj_sincos, so that an independent evaluation of the same sequence
 *    gives the same table bit for bit; within 1e-15 e0 of the field's exact values;
 *  - e_half given (a DEVICE array of 2 n_steps + 1 values, copied during sfhk_job_create; the caller
 *    may free it afterwards): that table is used; if pulse is also given, the table must agree with
 *    the pulse's within 1e-9 e0 at every half step (else SFHK_E_INVALID), so a job cannot run in a
 *    field other than the pulse its births (sfhk_sfa_birth) were drawn from.
 * pulse is a HOST pointer read during sfhk_job_create. */
typedef struct {
  double t_a;
  double h;
  int64_t n_steps;
  const double* e_half;
  const sfhk_pulse* pulse;
} sfhk_grid;

/* Method parameters:
 *   gamma        coherent-state width (App. A), > 0
 *   kay_max      Kay removal limit D_t on |C|^2 (Sec. III.A): a trajectory stops contributing
 *                from the first step where |det G| > kay_max (also when its state is not finite)
 *   overlap_cut  a GTO primitive is skipped when the real part of its exponent is < -overlap_cut
 *   r_fp64       SFHK_FP32_MIXED only: steps that start at r < r_fp64 run in FP64
 *   precision    sfhk_precision
 *   n_out        0: dipole on the step grid (n_steps + 1 points); > 0: linearly resampled onto
 *                t_k = t_a + k (n_steps h) / n_out, k = 0..n_out-1
 *   velocity     1: also accumulate the dipole velocity (App. C.2; read with sfhk_velocity); its
 *                accumulators double the job's accumulator memory. 0: dipole only
 *   pw_mask      partial-wave filter of the returning trajectories (Sec. III.A). 0: every step
 *                counts. Otherwise a step's dipole (and velocity) term counts only when
 *                r < pw_radius and l = |q x p| lies in a selected band: bit k (k = 0..6) for
 *                l in [k - 1/2, k + 1/2) (k = 0: [0, 1/2); s, p, d, ... waves), bit 7 for
 *                l >= 13/2; bit 8 keeps the steps at r >= pw_radius. 0x1FF equals no filter. The
 *                comparison is of r^2 = fma(q_z, q_z, fma(q_y, q_y, q_x q_x)) and
 *                l^2 = fma(L_z, L_z, fma(L_y, L_y, L_x L_x)), L_x = fma(q_y, p_z, -(q_z p_y)) and
 *                cyclic, with pw_radius^2 and the squared band edges.
 *   pw_radius    radius of the filter's near-core region (> 0 when pw_mask != 0)
 *   compact_every  0 (no regrouping) or E in [16, 2^24], FP64 jobs only (SFHK_E_INVALID
 *                otherwise): sfhk_propagate runs the job's tiles four at a time, and at every step
 *                k E the four tiles of one first birth step move the trajectories not removed by
 *                the Kay test (Sec. III.A) into their first tiles, so that tiles emptied by
 *                removals stop costing work. Trajectories are unchanged bit for bit; which ones
 *                share a tile depends only on the removal steps, so results are bitwise
 *                reproducible (chunked or not, checkpointed or not), and they differ from
 *                compact_every = 0 only in how the dipole's terms are grouped within a tile before
 *                the exact per-step sum (rounding level). Such jobs run through sfhk_propagate
 *                only (sfhk_propagate_many and batches refuse them). The four-wave workgroups cost
 *                about 8% by themselves, so regrouping pays only when many trajectories are
 *                removed (measured on a soft-core hydrogen workload: 22% faster with 86% removed,
 *                14-16% slower with 28% removed). */
typedef struct {
  double gamma;
  double kay_max;
  double overlap_cut;
  double r_fp64;
  int32_t precision;
  int64_t n_out;
  int32_t velocity;
  int32_t pw_mask;
  double pw_radius;
  int32_t compact_every;
} sfhk_params;

typedef struct {
  int64_t n_traj;
  int64_t n_steps;
  int64_t steps_evaluated;   /* (trajectory, t_n) pairs evaluated so far, removal steps included */
  int64_t steps_fp64;        /* of which evaluated after an FP64 step (SFHK_FP32_MIXED) */
  int64_t kay_removed;
  int64_t nonfinite_removed;
  int64_t tiles_total;
  int64_t tiles_done;
  int64_t prims_evaluated;   /* GTO primitives evaluated in the dipole integrand (the rest were
                                skipped by overlap_cut) */
  int64_t integrands_evaluated; /* (trajectory, t_n) pairs whose dipole integrand was evaluated
                                   (not every primitive skipped) */
  int64_t reserved;          /* 0 */
} sfhk_stats;

typedef struct sfhk_ctx sfhk_ctx;
typedef struct sfhk_job sfhk_job;

/* Create a context on HIP device `device` whose jobs may hold at most hbm_budget_bytes of device
 * memory in total (0: no limit). Job buffers come from a stream-ordered memory pool owned by the
 * context, which keeps freed memory cached for later jobs until the context is destroyed (or an
 * allocation would fail, when the cache is returned). Synchronous. */
sfhk_status sfhk_ctx_create(int device, size_t hbm_budget_bytes, sfhk_ctx** out);
/* Waits for all work on the device, then releases the context and its memory pool. Every job of
 * the context must have been destroyed. */
void sfhk_ctx_destroy(sfhk_ctx* ctx);
/* Bytes of device memory held by the context's live jobs (a destroyed job's bytes are counted
 * out at once, while its memory returns to the pool when its last issued work completes). */
size_t sfhk_ctx_bytes_in_use(const sfhk_ctx* ctx);

/* Device bytes a job of this shape will hold (the admission test of a serving loop); velocity as
 * in sfhk_params. */
size_t sfhk_job_footprint(int64_t n_traj, int64_t n_steps, int64_t n_out, int32_t precision,
                          int32_t velocity);

/* Create a job: n_traj trajectories born at times t0[n_traj] with initial phase-space samples
 * q0[3][n_traj], p0[3][n_traj] (SoA, DEVICE) and complex Monte-Carlo/birth weights
 * w[2][n_traj] (re block then im block, DEVICE) or NULL for w_j = exp(i p0.q0)/n_traj (the
 * e^{i p0.q0} factor of the continuum wavefunction at the tunnel exit, App. A).
 * Each trajectory is born on the grid step nearest to t0 (ties to the lower step), with
 * M = I and S = 0. t0 must lie in [t_a, t_a + n_steps h]. Reads t0 synchronously (the host orders
 * trajectories by birth step); the other inputs are read on `stream` before the call returns its
 * status, after which the caller may free all inputs.
 * Errors: SFHK_E_INVALID (NULL pointers; gamma <= 0; kay_max not > 0 (+inf allowed: no
 * removal); overlap_cut not >= 0 (+inf allowed: no skipping); r_fp64 not >= 0 in the mixed form;
 * h <= 0; n_steps not in 1..2^30; n_traj not in 1..2^31; neither e_half nor a pulse; a pulse with
 * a non-finite e0 or cep, or omega or n_cycles not > 0; e_half given with a pulse but more than
 * 1e-9 e0 away from its field; unknown potential kind; r_scr <= 0 for the screened potential; l not
 * 0/1; n_prim not in 1..SFHK_MAX_PRIM or an exponent <= 0; precision unknown; n_out < 0; velocity
 * not 0/1; pw_mask outside [0, 0x1FF] or pw_radius not finite and > 0 with a mask; compact_every
 * not 0 or in [16, 2^24], or given with the mixed form; t0 outside the grid), SFHK_E_BUDGET,
 * SFHK_E_NOMEM, SFHK_E_DEVICE. NaN parameters fail these tests. Non-finite samples are not
 * errors: the trajectory is removed at its birth step and counted in nonfinite_removed. */
sfhk_status sfhk_job_create(sfhk_ctx* ctx, const sfhk_potential* pot, const sfhk_ground* ground,
                            const sfhk_grid* grid, const sfhk_params* params, int64_t n_traj,
                            const double* t0, const double* q0, const double* p0, const double* w,
                            void* stream, sfhk_job** out);
/* Release a job. Does not block: the job's memory is freed in stream order once all work issued
 * on it so far (on any stream) has completed. The caller must not issue further work on the job,
 * nor replay a batch whose staged table still lists it. */
void sfhk_job_destroy(sfhk_job* job);

/* Propagate the job's trajectories (RK4 steps of the 43 ODEs, HK prefactor, Kay removal, dipole
 * integrand, per-step reduction) by at most max_steps steps each (max_steps <= 0: to the end of
 * the grid). Returns SFHK_OK when every trajectory has reached the end of the grid,
 * SFHK_E_NOT_DONE when some have not (call again to continue: state stays in HBM between calls and
 * the result is identical to one uninterrupted call). Asynchronous on `stream`; the completion
 * status is known on the host without waiting for the kernels. */
sfhk_status sfhk_propagate(sfhk_job* job, int64_t max_steps, void* stream);

/* Propagate several jobs of one context with one kernel launch per (precision, potential kind)
 * present (jobs may differ in size, pulse, potential and precision). Same semantics per job as
 * sfhk_propagate; returns SFHK_E_NOT_DONE if any job is unfinished. The jobs must be distinct
 * (SFHK_E_INVALID if one is listed twice). */
sfhk_status sfhk_propagate_many(sfhk_job* const* jobs, int32_t n_jobs, int64_t max_steps,
                                void* stream);

/* Batched, graph-captured propagation. A batch owns a job table of fixed capacity (max_jobs
 * jobs, max_tiles unfinished tiles) at fixed device addresses and a HIP graph captured once at
 * creation: a queue reset followed by one kernel per (precision, potential kind). Each replay
 * (sfhk_batch_run) advances every staged unfinished tile by up to max_steps steps (max_steps <= 0:
 * to the end of its grid), longest tiles first. workers_per_cu > 0: that many single-wave workgroups
 * per compute unit stay resident and pop tiles from a device-side atomic queue (persistent
 * form); 0: one workgroup per tile, dispatched by the hardware. The table is rewritten between
 * replays by sfhk_batch_set_jobs (no re-capture), so jobs can be added and dropped between replays
 * (continuous batching). Results are identical to sfhk_propagate on each job alone.
 * Errors: SFHK_E_INVALID (capacity exceeded, jobs of another context, bad sizes), SFHK_E_NOMEM,
 * SFHK_E_DEVICE. A batch is used from one host thread; the jobs' other calls must be ordered with
 * its replays by the caller (same stream). */
typedef struct sfhk_batch sfhk_batch;
sfhk_status sfhk_batch_create(sfhk_ctx* ctx, int32_t max_jobs, int64_t max_tiles, int64_t max_steps,
                              int32_t workers_per_cu, sfhk_batch** out);
/* Stage the unfinished tiles of jobs[0..n_jobs) (distinct jobs; SFHK_E_INVALID if one is listed
 * twice): the table is written to one of two pinned
 * staging sets, used in turn, and copied asynchronously on `stream`. The call waits only until
 * the replay issued after the previous use of that set has completed, so a caller can stage the
 * next replay while the current one runs (the host stays at most one replay ahead). */
sfhk_status sfhk_batch_set_jobs(sfhk_batch* batch, sfhk_job* const* jobs, int32_t n_jobs, void* stream);
/* One graph replay on `stream`. SFHK_OK when every staged job has finished (at once for an empty
 * table), else SFHK_E_NOT_DONE; SFHK_E_INVALID, with nothing launched, when no table is staged
 * (sfhk_batch_set_jobs not called yet, or its last call failed). */
sfhk_status sfhk_batch_run(sfhk_batch* batch, void* stream);
/* Resident workgroups of the persistent form (0 for hardware dispatch). */
int32_t sfhk_batch_workers(const sfhk_batch* batch);
void sfhk_batch_destroy(sfhk_batch* batch);

/* Round the job's exact per-step sums once into F(t_n) = sum_j f_j(t_n) (every term was added as
 * an integer into fixed-point accumulators, so F is the correctly rounded sum of the step's terms
 * as grouped within each tile, whatever the order of the tiles) and write d_out = -2 Re F (Eq. 2: "+ c.c." with the leading minus) on the job's output grid (n_out points,
 * or n_steps + 1 when n_out = 0). f_out (nullable) receives F on the step grid as
 * [2][n_steps+1] (re block then im block). Requires a finished job (else SFHK_E_NOT_DONE). */
sfhk_status sfhk_dipole(sfhk_job* job, double* d_out, double* f_out, void* stream);

/* The dipole velocity of a job created with velocity = 1 (App. C.2): the exact per-step sum
 * V(t_n) = sum_j w_j C_j(t_n) <psi0|k_z|p_t,q_t,gamma> e^{i(S_j - Ip t_n)} over the same
 * trajectories, steps and removal rule as F, and v_out = -2 Re V on the job's output grid
 * (as d_out of sfhk_dipole); vf_out (nullable) receives V as [2][n_steps+1]. The velocity element
 * is the printed s-/p-wave form in the scale of the dipole element: for an s-wave ground state
 * -2 i a sum_j alpha_j N_j E_j, for a p-wave one 2 i sum_j N_j E_j (2 gamma (gamma + alpha_j)
 * - alpha_j a^2), with a = 2 gamma q_z + i p_z and N_j E_j the dipole element's primitive terms;
 * that is, the printed forms times 2 (s) and 4 i gamma (p), the ratio of the two elements'
 * written-out constants, so that both forms keep their relative phase. Requires a finished job
 * (SFHK_E_NOT_DONE) created with velocity = 1 (else SFHK_E_INVALID). DEVICE pointers. */
sfhk_status sfhk_velocity(sfhk_job* job, double* v_out, double* vf_out, void* stream);

/* 1 once every trajectory of the job has been propagated to the end of the grid by the calls
 * issued so far (host-side bookkeeping: no synchronisation; the device work completes in stream
 * order), else 0. */
int32_t sfhk_job_is_done(const sfhk_job* job);

/* Number of points sfhk_dipole writes to d_out. */
int64_t sfhk_job_n_out(const sfhk_job* job);

/* Checkpoint and restore of a job's propagation state, for suspending a job (for instance to free
 * its HBM) and resuming it later: the trajectory state, removal steps, per-tile progress, partial
 * rows, counters and the number of steps requested so far.
 * sfhk_job_checkpoint_bytes: size of a checkpoint of this job.
 * sfhk_job_checkpoint: writes it to dst (DEVICE, checkpoint_bytes, caller-owned) on `stream` and
 *   returns once the copies have completed. Errors: SFHK_E_INVALID (NULL), SFHK_E_DEVICE.
 * sfhk_job_restore: loads a checkpoint into `job`, which must have been created from the same
 *   inputs and not propagated; propagation then continues exactly as the checkpointed job would
 *   have (bit for bit). The checkpoint records the job's shape and a fingerprint of its potential,
 *   ground state, grid (t_a, h) and sfhk_params, and a job that differs in any of them is refused
 *   (the field table's values are not compared). Reads the header synchronously, copies the state
 *   asynchronously on `stream`. Errors: SFHK_E_INVALID (NULL, not a checkpoint, another job's
 *   shape or parameters, a job already propagated), SFHK_E_DEVICE. */
int64_t sfhk_job_checkpoint_bytes(const sfhk_job* job);
sfhk_status sfhk_job_checkpoint(sfhk_job* job, void* dst, void* stream);
sfhk_status sfhk_job_restore(sfhk_job* job, const void* src, void* stream);

/* Hann-windowed Fourier transform (App. D): with t_n = t_first + n dt and d zero-padded to
 * n_fft samples (n_fft = 0: n),
 *   X_k = dt sum_n d_n W_H(t_n) exp(i omega_k t_n),  W_H(t) = (1 + cos(pi t / tau_h)) / 2 for
 *   |t| < tau_h and 0 otherwise,  omega_k = 2 pi k / (n_fft dt),  k = 0..n_fft/2.
 * Writes omega_out[k], power_out[k] = |X_k|^2 and (nullable) x_out[2k], x_out[2k+1] = X_k.
 * Stateless. Errors: SFHK_E_INVALID for n < 1, n_fft < n, n_fft > 2^31, dt <= 0 or tau_h <= 0. */
sfhk_status sfhk_spectrum(const double* d, int64_t n, double t_first, double dt, double tau_h,
                          int64_t n_fft, double* omega_out, double* power_out, double* x_out,
                          void* stream);

/* sfhk_spectrum for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same arguments and the same
 * results, bit for bit, but its working memory (the windowed samples, the twiddle table and the
 * per-span partial sums) is a fixed device array of the library, SFHK_SPECTRUM_NOALLOC_BYTES per
 * GPU, which each GPU the library runs on holds until the process ends; the call allocates and
 * frees nothing and needs no clearing of that array (every byte it reads it has written first).
 * Limit: n_fft <= SFHK_SPECTRUM_NOALLOC_MAX_FFT (n_fft = 0: n); SFHK_E_INVALID beyond, or as
 * sfhk_spectrum. The first call on a device looks up that device's copy of the array
 * (SFHK_E_DEVICE if the lookup fails). Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (on different streams, or from different host threads without ordering)
 * race and give wrong results; order them on one stream. */
#define SFHK_SPECTRUM_NOALLOC_MAX_FFT 65536
#define SFHK_SPECTRUM_NOALLOC_BYTES 35128320
sfhk_status sfhk_spectrum_noalloc(const double* d, int64_t n, double t_first, double dt,
                                  double tau_h, int64_t n_fft, double* omega_out,
                                  double* power_out, double* x_out, void* stream);

/* Counters of the job (synchronises `stream` first). */
sfhk_status sfhk_job_stats(sfhk_job* job, sfhk_stats* out, void* stream);

/* Per-trajectory state in the caller's original trajectory order (for checks and checkpoints):
 * y_out[43][n_traj] = q(3) p(3) M (6 columns of Q(3) P(3)) S at the last step evaluated (the
 * removal step for removed trajectories), c_out[2][n_traj] = HK prefactor C at the last accepted
 * step, death_out[n_traj] = removal step or -1 (int64). Any output may be NULL. DEVICE pointers. */
sfhk_status sfhk_job_trajectories(sfhk_job* job, double* y_out, double* c_out, int64_t* death_out,
                                  void* stream);

/* Text of the most recent error on the calling thread ("" if none). */
const char* sfhk_last_error(void);
const char* sfhk_status_string(sfhk_status s);

/* The two elementary functions of the trajectory arithmetic, exported so their operation
 * sequences can be checked against an independent implementation (DEVICE pointers, y[i] = f(x[i])
 * for i < n, asynchronous on `stream`; SFHK_E_INVALID for NULL pointers or n outside [0, 2^31)).
 *
 * sfhk_traj_exp: exp as evaluated inside the screened potential. Cody-Waite reduction
 * x = k ln2 + r (ln2 split into a 32-significant-bit head and a rounded tail, both applied with
 * fused multiply-adds), the degree-13 Taylor polynomial of exp(r) in Horner form with fused
 * multiply-adds, then scaling by 2^k; 0 for x < -708. Within one ulp of exp.
 *
 * sfhk_traj_rsqrt: 1/sqrt(x) as used for every square root and reciprocal on the trajectory path.
 * Bit-pattern seed (magic constant 0x5FE6EB50C7B537A9), three Newton steps
 * y <- y (3/2 - (x/2) y^2), a final step y + y (1/2 - (x/2) y^2); arguments outside
 * [2^-1000, 2^1000] are first scaled by an even power of two. Within one ulp of 1/sqrt(x);
 * 0 -> +inf, +inf -> 0, negative or NaN -> NaN. */
sfhk_status sfhk_traj_exp(const double* x, double* y, int64_t n, void* stream);
sfhk_status sfhk_traj_rsqrt(const double* x, double* y, int64_t n, void* stream);

/* Gabor time-frequency transform (the emission-time analysis of Sec. III.A) of a real signal d
 * (the dipole or the dipole velocity), n samples at t_n = t_first + n dt:
 *   G(t_c, w_k) = dt sum_n d_n exp(-(t_n - t_c)^2 / (2 sigma^2)) exp(i w_k t_n),
 * t_c = tc_first + c tc_step (c < n_c <= 65535), w_k = k w_step (k < n_w).
 * power_out[n_c][n_w] = |G|^2; g_out (nullable) [n_c][n_w][2] = (Re G, Im G). Samples farther than
 * 9.2 sigma from t_c (window below 4e-19 of its peak) are not summed. DEVICE pointers;
 * asynchronous on `stream`. SFHK_E_INVALID for negative counts, dt or sigma not finite and > 0,
 * non-finite grids, more than 65535 centres or 2^31 outputs, or a NULL array. */
sfhk_status sfhk_gabor(const double* d, int64_t n, double t_first, double dt, double sigma,
                       double tc_first, double tc_step, int64_t n_c, double w_step, int64_t n_w,
                       double* power_out, double* g_out, void* stream);

/* sfhk_traj_sincos: s[i], c[i] = sin(x[i]), cos(x[i]) as evaluated in the SFA birth step's
 * saddle-point solve. Cody-Waite reduction x = k pi/2 + r, k = rint(x 2/pi), with pi/2 split into
 * two 33-significant-bit heads and a rounded tail (applied with fused multiply-adds), Taylor
 * polynomials in r^2 of degree 17 (sine) and 18 (cosine) in Horner form with fused multiply-adds,
 * and the quadrant k mod 4. NaN for |x| >= 2^20 or non-finite x. Within one ulp for |x| <= 64.
 * n must be below 2^31. */
sfhk_status sfhk_traj_sincos(const double* x, double* s, double* c, int64_t n, void* stream);

/* ------------------------------------------------------------------------------------------------
 * SFA birth step (App. A: the continuum wave packet right after tunnelling, the saddle-point
 * equation, the tunnel exit and the action under the barrier; App. B: tunnelling elements).
 *
 * The pulse is the sfhk_pulse of sfhk_grid (the same description a job's field is tabulated
 * from); n_cycles must exceed 1 here.
 */

typedef enum {
  SFHK_BIRTH_GTO = 0,      /* Eq. A.2 with the GTO tunnelling element of App. B.1 */
  SFHK_BIRTH_MODIFIED = 1  /* the modified saddle-point form of App. B.2 */
} sfhk_birth_mode;

/* For every sample j < n, with birth time t0[j] and transverse momentum (kx, ky) =
 * (kperp[j], kperp[n + j]):
 *  - the saddle point t_s = t0 + i t_t of [k + A(t_s) - A(t0)]^2 / 2 + Ip = 0 (Ip = gs->ip) with
 *    k = p0 = (kx, ky, k_z): Im A(t_s) = +-kappa, kappa^2 = 2 Ip + kx^2 + ky^2, fixes t_t > 0 (the
 *    root nearest the real axis) and k_z = A(t0) - Re A(t_s);
 *  - the tunnel exit q0 = (0, 0, Re int_{t_s}^{t0} A(t) dt);
 *  - S_down = Ip t_s - int_{t_s}^{t0} [k + A(t) - A(t0)]^2 / 2 dt and the birth weight
 *      SFHK_BIRTH_GTO:      w = u_j e^{i p0.q0} (-i) sqrt(2 pi i / (E(t_s).k_s)) <k_s| r.E(t_s) |psi0>
 *                               e^{i S_down},  k_s = k + A(t_s) - A(t0),
 *                           <k|z|psi0> = int e^{-i k.r} z psi0(r) d^3r over the GTOs of gs (s-wave:
 *                           -i (pi^{3/2}/2) k_z sum_i c_i a_i^{-5/2} e^{-k^2/(4 a_i)}; p-wave:
 *                           (pi^{3/2}/4) sum_i c_i a_i^{-7/2} (2 a_i - k_z^2) e^{-k^2/(4 a_i)});
 *      SFHK_BIRTH_MODIFIED: w = u_j e^{i p0.q0} e^{i S_down} / (E(t_s).k_s).
 * u[n] are Monte-Carlo weights (NULL: 1/n). Outputs: q0[3][n], p0[3][n], w[2][n] (re block, im
 * block) -- the layout sfhk_job_create takes -- and t_tun[n] = t_t (may be NULL).
 * t_t, k_z and q0 are computed with the trajectory arithmetic (sfhk_traj_sincos, sfhk_traj_exp,
 * sfhk_traj_rsqrt; a march of at most 512 steps of 1/(4 (omega + omega/n_cycles)) to the first
 * |Im A| >= kappa, then 16 bisection steps and 4 Newton steps kept inside the bracket), so they
 * are reproducible bit for bit; the weight uses
 * library functions. A sample with no crossing within the march, or with non-finite inputs, gets
 * NaN outputs (sfhk_job_create then counts it as a removed trajectory). Birth times outside the
 * pulse [-T/2, T/2] are not rejected here (the product-to-sum form of A is continued past the
 * envelope's support); sfhk_job_create rejects them.
 * All arrays are DEVICE pointers owned by the caller; asynchronous on `stream`. SFHK_E_INVALID for a
 * bad pulse, Ip <= 0, l not 0/1, an unknown mode, no or too many GTO primitives (mode GTO), a NULL
 * array, or n outside [0, 2^31). */
sfhk_status sfhk_sfa_birth(const sfhk_pulse* pulse, const sfhk_ground* gs, int32_t mode, int64_t n,
                           const double* t0, const double* kperp, const double* u, double* q0,
                           double* p0, double* w, double* t_tun, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SFHK_H */
