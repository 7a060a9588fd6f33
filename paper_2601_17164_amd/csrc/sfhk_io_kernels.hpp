// sfhk_io_kernels.hpp -- the kernels around the propagation (gfx950): birth steps and initial
// state of a job, the dipole from the per-step exact accumulators, resampling, the
// per-trajectory state in caller order, the Hann-windowed Fourier transform, and the exported
// contract functions. Included by sfhk.hip after sfhk_kernels.hpp (device layout and the
// propagation kernels).
#pragma once
#include "sfhk_kernels.hpp"

namespace {

// ------------------------------------------------------------------------------------------------
// initialisation: gather the sorted samples into the SoA state
// ------------------------------------------------------------------------------------------------
// birth step of sample i: the nearest grid step to t0, ties to the lower one (u = (t0 - t_a)/h,
// n0 = ceil(u - 1/2), clamped to 0..n_steps)
__device__ __forceinline__ int birth_step(double t, double t_a, double h, int n_steps) {
  double nn = ceil((t - t_a) / h - 0.5);
  if (!(nn >= 0.0)) nn = 0.0;
  if (nn > (double)n_steps) nn = (double)n_steps;
  return (int)nn;
}

// Birth steps of the samples in caller order (n_steps + 1 on padding slots), each tile's first
// birth step, and two flags for the host: flags[0] = smallest index whose t0 lies outside
// [t_lo, t_hi] (all ones if none), flags[1] != 0 if the birth steps are not non-decreasing.
__global__ void k_birth(const double* __restrict__ t0, long long n_traj, long long n_pad,
                        double t_a, double h, double t_lo, double t_hi, int n_steps,
                        int* __restrict__ n0, int* __restrict__ tile_n0,
                        unsigned long long* __restrict__ flags) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pad) return;
  int b = n_steps + 1;
  if (i < n_traj) {
    const double t = t0[i];
    if (!(t >= t_lo && t <= t_hi)) atomicMin(&flags[0], (unsigned long long)i);
    b = birth_step(t, t_a, h, n_steps);
    if (i > 0 && birth_step(t0[i - 1], t_a, h, n_steps) > b) atomicOr(&flags[1], 1ull);
  }
  n0[i] = b;
  if ((i % kTile) == 0) tile_n0[i / kTile] = b;
}

// perm == nullptr: slot s holds sample s (samples already in birth order), padding beyond n_traj
__global__ void k_init(JobDev J, const long long* __restrict__ perm, long long n_traj,
                       const double* __restrict__ q0, const double* __restrict__ p0,
                       const double* __restrict__ w) {
  long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= J.n_pad) return;
  long long np = J.n_pad;
  long long o = perm ? perm[s] : (s < n_traj ? s : -1);
  double* y = J.y;
  double q[3] = {0, 0, 0}, p[3] = {0, 0, 0}, wr = 0.0, wi = 0.0;
  if (o >= 0) {
    for (int i = 0; i < 3; ++i) {
      q[i] = q0[i * n_traj + o];
      p[i] = p0[i * n_traj + o];
    }
    if (w) {
      wr = w[o];
      wi = w[n_traj + o];
    } else {  // exp(i p0.q0) / n
      double pq = p[0] * q[0] + p[1] * q[1] + p[2] * q[2];
      double sn, cs;
      sincos(pq, &sn, &cs);
      wr = cs / (double)n_traj;
      wi = sn / (double)n_traj;
    }
  }
  for (int i = 0; i < 3; ++i) {
    y[i * np + s] = q[i];
    y[(3 + i) * np + s] = p[i];
  }
  for (int c = 0; c < 36; ++c) y[(6 + c) * np + s] = (c % 7 == 0) ? 1.0 : 0.0;  // M = I
  y[42 * np + s] = 0.0;
  J.aux[0 * np + s] = 1.0;  // C_prev
  J.aux[1 * np + s] = 0.0;
  J.aux[2 * np + s] = wr;
  J.aux[3 * np + s] = wi;
  J.aux[4 * np + s] = 1.0;  // branch sign
  J.death[s] = (o >= 0) ? -1 : -2;
}

// ------------------------------------------------------------------------------------------------
// the dipole from the per-step exact accumulators
// ------------------------------------------------------------------------------------------------
// F(t_n) = the exact sum of the step's integrands, rounded once to binary64; d = -2 Re F (Eq. 2:
// "+ c.c." with the leading minus); f_out (nullable) = [Re F][Im F] on the step grid
__global__ void k_acc_final(const long long* __restrict__ acc, int n_steps, double* __restrict__ d,
                            double* __restrict__ f_out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n > n_steps) return;
  const int64_t* a = (const int64_t*)acc + (long long)n * (2 * sfhk_exact::kExactWords);
  const double re = sfhk_exact::round_total(a);
  const double im = sfhk_exact::round_total(a + sfhk_exact::kExactWords);
  d[n] = -2.0 * re;
  if (f_out) {
    f_out[n] = re;
    f_out[n_steps + 1 + n] = im;
  }
}

__global__ void k_resample(const double* __restrict__ d, long long n_steps, long long n_out,
                           double* __restrict__ out) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_out) return;
  long long num = k * n_steps;
  long long i = num / n_out;
  long long rem = num - i * n_out;
  double frac = (double)rem / (double)n_out;
  out[k] = (i >= n_steps) ? d[n_steps] : d[i] + frac * (d[i + 1] - d[i]);
}

// ------------------------------------------------------------------------------------------------
// trajectories in the caller's order
// ------------------------------------------------------------------------------------------------
__global__ void k_scatter_traj(JobDev J, const long long* __restrict__ perm, long long n_traj,
                               double* __restrict__ y_out, double* __restrict__ c_out,
                               long long* __restrict__ death_out) {
  long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= J.n_pad) return;
  long long o = perm ? perm[s] : (s < n_traj ? s : -1);
  if (o < 0) return;
  if (y_out)
    for (int c = 0; c < kNY; ++c) y_out[c * n_traj + o] = J.y[c * J.n_pad + s];
  if (c_out) {
    c_out[o] = J.aux[s];
    c_out[n_traj + o] = J.aux[J.n_pad + s];
  }
  if (death_out) death_out[o] = J.death[s];
}

// ------------------------------------------------------------------------------------------------
// spectrum: Hann window and direct Fourier sum with exact index reduction k n mod n_fft
// ------------------------------------------------------------------------------------------------
__global__ void k_window(const double* __restrict__ d, long long n, long long n_fft, double t_first,
                         double dt, double tau_h, double* __restrict__ xw, double2* __restrict__ tw) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_fft) return;
  double v = 0.0;
  if (i < n) {
    double t = t_first + (double)i * dt;
    double win = fabs(t) >= tau_h ? 0.0 : 0.5 * (1.0 + cos(M_PI * t / tau_h));
    v = d[i] * win;
  }
  xw[i] = v;
  double s, c;
  sincospi(2.0 * (double)i / (double)n_fft, &s, &c);
  tw[i] = make_double2(c, s);
}

// Direct DFT, Y_k = sum_n x_n e^{2 pi i k n / n_fft} for k = 0..n_fft/2. Blocks along y take
// consecutive spans of samples; within a span each lane keeps its twiddle by the recurrence
// t <- t e^{2 pi i k / n_fft}, re-anchored from the exact table (index k m mod n_fft) at every
// staged chunk of kDftChunk samples, so the recurrence error stays near kDftChunk ulps. Partial
// sums per span are added in span order by k_dft_final (deterministic).
constexpr int kDftChunk = 1024;
constexpr int kDftMaxSpans = 64;

__global__ __launch_bounds__(256) void k_dft_partial(const double* __restrict__ xw,
                                                     const double2* __restrict__ tw, long long n,
                                                     long long n_fft, long long span,
                                                     double2* __restrict__ part) {
  __shared__ double xs[kDftChunk];
  const long long nk = n_fft / 2 + 1;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long kk = k < nk ? k : 0;
  const long long lo = (long long)blockIdx.y * span;
  const long long hi = min(n, lo + span);
  const double2 step = tw[kk];
  double cr = 0.0, ci = 0.0;
  for (long long base = lo; base < hi; base += kDftChunk) {
    const int cnt = (int)min((long long)kDftChunk, hi - base);
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) xs[i] = xw[base + i];
    __syncthreads();
    double2 t = tw[(kk * base) % n_fft];
    for (int i = 0; i < cnt; ++i) {
      cr = SFHK_FMA(xs[i], t.x, cr);
      ci = SFHK_FMA(xs[i], t.y, ci);
      const double tr = SFHK_FMA(t.x, step.x, -(t.y * step.y));
      t.y = SFHK_FMA(t.x, step.y, t.y * step.x);
      t.x = tr;
    }
  }
  if (k < nk) part[(long long)blockIdx.y * nk + k] = make_double2(cr, ci);
}

__global__ void k_dft_final(const double2* __restrict__ part, int n_spans, long long n_fft,
                            double t_first, double dt, double* __restrict__ omega_out,
                            double* __restrict__ power_out, double* __restrict__ x_out) {
  const long long nk = n_fft / 2 + 1;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  double sr = 0.0, si = 0.0;
  for (int g = 0; g < n_spans; ++g) {
    const double2 v = part[(long long)g * nk + k];
    sr += v.x;
    si += v.y;
  }
  const double omega = 2.0 * M_PI * (double)k / ((double)n_fft * dt);
  double s, c;
  sincos(omega * t_first, &s, &c);
  const double xr = dt * (sr * c - si * s);
  const double xi = dt * (sr * s + si * c);
  if (omega_out) omega_out[k] = omega;
  if (power_out) power_out[k] = xr * xr + xi * xi;
  if (x_out) {
    x_out[2 * k] = xr;
    x_out[2 * k + 1] = xi;
  }
}

__global__ void k_traj_fn(int which, const double* __restrict__ x, double* __restrict__ y,
                          long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = which == 0 ? exp_cw(x[i]) : rsqrt_c(x[i]);
}

}  // namespace
