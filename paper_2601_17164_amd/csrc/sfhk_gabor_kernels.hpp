// sfhk_gabor_kernels.hpp -- Gabor time-frequency transform (the emission-time analysis of
// Sec. III.A):  G(t_c, w_k) = dt sum_n d_n exp(-(t_n - t_c)^2 / (2 sigma^2)) exp(i w_k t_n),
// t_n = t_first + n dt, t_c = tc_first + c tc_step, w_k = k w_step.
//
// One block per (centre c, 256 frequencies), one thread per frequency. The Gaussian window falls
// below exp(-kGaborCut^2 / 2) = 4e-19 of its peak beyond kGaborCut sigma, so only the samples
// within that distance of t_c are summed (the truncated tail is far below rounding). The block
// stages the windowed samples x_n = d_n exp(-(t_n - t_c)^2 / (2 sigma^2)) of each chunk of 1024 in
// LDS (computed once, read by every frequency); each thread sums the chunk as the polynomial
// sum_j x_j z^j in z = e^{i w_k dt} by Horner's rule (four FP64 instructions per sample; with
// |z| = 1 the error stays at about the chunk length in roundings) and adds it times the chunk's
// anchor e^{i w_k t_base}, taken from a library sincos.
#pragma once
#include <hip/hip_runtime.h>

namespace {

constexpr int kGaborThreads = 256;
constexpr int kGaborChunk = 1024;  // samples staged per barrier (kGaborChunk / kGaborThreads each)
constexpr double kGaborCut = 9.2;

__global__ __launch_bounds__(kGaborThreads) void k_gabor(const double* __restrict__ d, long long n,
                                                         double t_first, double dt, double sigma,
                                                         double tc_first, double tc_step, double w_step,
                                                         long long n_w, double* __restrict__ power,
                                                         double2* __restrict__ g) {
  __shared__ double xs[kGaborChunk];
  const int tid = threadIdx.x;
  const long long c = blockIdx.y;
  const long long k = (long long)blockIdx.x * kGaborThreads + tid;
  const double tc = tc_first + (double)c * tc_step;
  // samples within kGaborCut sigma of t_c (block-uniform)
  const double lo_t = (tc - kGaborCut * sigma - t_first) / dt;
  const double hi_t = (tc + kGaborCut * sigma - t_first) / dt;
  // clamped to [0, n] and [-1, n - 1] before the conversion (an empty range when the window
  // misses the record)
  const long long n_lo = (long long)ceil(fmin(fmax(lo_t, 0.0), (double)n));
  const long long n_hi = (long long)floor(fmax(fmin(hi_t, (double)(n - 1)), -1.0));
  const double w = (double)k * w_step;
  double rs, rc;
  ::sincos(w * dt, &rs, &rc);  // rotation per sample
  double ar = 0.0, ai = 0.0;
  const double inv2s2 = 0.5 / (sigma * sigma);
  for (long long base = n_lo; base <= n_hi; base += kGaborChunk) {
#pragma unroll
    for (int s = 0; s < kGaborChunk / kGaborThreads; ++s) {
      const long long m = base + s * kGaborThreads + tid;
      double x = 0.0;
      if (m <= n_hi) {
        const double u = t_first + (double)m * dt - tc;
        x = d[m] * exp(-(u * u) * inv2s2);
      }
      xs[s * kGaborThreads + tid] = x;
    }
    __syncthreads();
    // the chunk's sum as a polynomial in z = e^{i w dt} by Horner's rule (from its last sample
    // down), then one multiplication by the anchor e^{i w t_base}
    const long long len = n_hi - base + 1 < kGaborChunk ? n_hi - base + 1 : kGaborChunk;
    double pr = 0.0, pi = 0.0;
    for (int j = (int)len - 1; j >= 0; --j) {
      const double np = fma(pr, rc, fma(-pi, rs, xs[j]));
      pi = fma(pr, rs, pi * rc);
      pr = np;
    }
    double ts, tcos;
    ::sincos(w * (t_first + (double)base * dt), &ts, &tcos);
    ar = fma(pr, tcos, fma(-pi, ts, ar));
    ai = fma(pr, ts, fma(pi, tcos, ai));
    __syncthreads();
  }
  if (k < n_w) {
    const double gr = ar * dt, gi = ai * dt;
    const long long o = c * n_w + k;
    power[o] = gr * gr + gi * gi;
    if (g) g[o] = make_double2(gr, gi);
  }
}

}  // namespace
