// sfhk_gabor_kernels.hpp -- Gabor time-frequency transform (the emission-time analysis of
// Sec. III.A):  G(t_c, w_k) = dt sum_n d_n exp(-(t_n - t_c)^2 / (2 sigma^2)) exp(i w_k t_n),
// t_n = t_first + n dt, t_c = tc_first + c tc_step, w_k = k w_step.
//
// One block per (centre c, 512 frequencies), each thread two frequencies k and k + 256 (two
// independent chains sharing every staged sample). The Gaussian window falls
// below exp(-kGaborCut^2 / 2) = 4e-19 of its peak beyond kGaborCut sigma, so only the samples
// within that distance of t_c are summed (the truncated tail is far below rounding). The block
// stages the windowed samples x_n = d_n exp(-(t_n - t_c)^2 / (2 sigma^2)) of each chunk of 1024 in
// LDS (computed once, read by every frequency); each chain sums the chunk as the polynomial
// sum_j x_j z^j in z = e^{i w_k dt} by Horner's rule (four FP64 instructions per sample; with
// |z| = 1 the error stays at about the chunk length in roundings) and adds it times the chunk's
// anchor e^{i w_k t_base}, taken from a library sincos.
#pragma once
#include <hip/hip_runtime.h>

namespace {

constexpr int kGaborThreads = 256;
constexpr int kGaborChunk = 1024;  // samples staged per barrier (kGaborChunk / kGaborThreads each)
constexpr double kGaborCut = 9.2;

constexpr int kGaborFreqPerBlock = 2 * kGaborThreads;

__global__ __launch_bounds__(kGaborThreads) void k_gabor(const double* __restrict__ d, long long n,
                                                         double t_first, double dt, double sigma,
                                                         double tc_first, double tc_step, double w_step,
                                                         long long n_w, double* __restrict__ power,
                                                         double2* __restrict__ g) {
  __shared__ double xs[kGaborChunk];
  const int tid = threadIdx.x;
  const long long c = blockIdx.y;
  const long long k0 = (long long)blockIdx.x * kGaborFreqPerBlock + tid;
  const long long k1 = k0 + kGaborThreads;
  const double tc = tc_first + (double)c * tc_step;
  // samples within kGaborCut sigma of t_c (block-uniform)
  const double lo_t = (tc - kGaborCut * sigma - t_first) / dt;
  const double hi_t = (tc + kGaborCut * sigma - t_first) / dt;
  // clamped to [0, n] and [-1, n - 1] before the conversion (an empty range when the window
  // misses the record)
  const long long n_lo = (long long)ceil(fmin(fmax(lo_t, 0.0), (double)n));
  const long long n_hi = (long long)floor(fmax(fmin(hi_t, (double)(n - 1)), -1.0));
  const double w0 = (double)k0 * w_step, w1 = (double)k1 * w_step;
  double rs0, rc0, rs1, rc1;
  ::sincos(w0 * dt, &rs0, &rc0);  // rotation per sample
  ::sincos(w1 * dt, &rs1, &rc1);
  double ar0 = 0.0, ai0 = 0.0, ar1 = 0.0, ai1 = 0.0;
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
    double pr0 = 0.0, pi0 = 0.0, pr1 = 0.0, pi1 = 0.0;
#pragma unroll 4
    for (int j = (int)len - 1; j >= 0; --j) {
      const double x = xs[j];
      const double np0 = fma(pr0, rc0, fma(-pi0, rs0, x));
      pi0 = fma(pr0, rs0, pi0 * rc0);
      pr0 = np0;
      const double np1 = fma(pr1, rc1, fma(-pi1, rs1, x));
      pi1 = fma(pr1, rs1, pi1 * rc1);
      pr1 = np1;
    }
    const double tb = t_first + (double)base * dt;
    double ts, tcos;
    ::sincos(w0 * tb, &ts, &tcos);
    ar0 = fma(pr0, tcos, fma(-pi0, ts, ar0));
    ai0 = fma(pr0, ts, fma(pi0, tcos, ai0));
    ::sincos(w1 * tb, &ts, &tcos);
    ar1 = fma(pr1, tcos, fma(-pi1, ts, ar1));
    ai1 = fma(pr1, ts, fma(pi1, tcos, ai1));
    __syncthreads();
  }
  if (k0 < n_w) {
    const double gr = ar0 * dt, gi = ai0 * dt;
    const long long o = c * n_w + k0;
    power[o] = gr * gr + gi * gi;
    if (g) g[o] = make_double2(gr, gi);
  }
  if (k1 < n_w) {
    const double gr = ar1 * dt, gi = ai1 * dt;
    const long long o = c * n_w + k1;
    power[o] = gr * gr + gi * gi;
    if (g) g[o] = make_double2(gr, gi);
  }
}

}  // namespace
