/* The hot path through the C ABI from plain C (no Python, no C++): reads an instance written by
 * tests/test_gpu_c_api.py, uploads it with the HIP runtime API, creates a context and a job whose
 * field the library tabulates from the pulse, propagates it in chunks, and writes F (step grid,
 * re block then im block), d (step grid) and the power spectrum to the output file.
 *   usage: c_api_driver <instance file> <output file>
 * Instance file (little-endian): int64 n_traj, n_steps, n_prim, l, pot_kind, chunk; double t_a, h,
 * e0, omega, n_cycles, cep, gamma, kay_max, overlap_cut, ip, z_inf, z_in, r_scr, soft2, omega_ho;
 * double alpha[n_prim], coef[n_prim], t0[n], q0[3][n], p0[3][n]. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "sfhk.h"

#define CHECK_HIP(x)                                                          \
  do {                                                                        \
    hipError_t e_ = (x);                                                      \
    if (e_ != hipSuccess) {                                                   \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                 \
      return 2;                                                               \
    }                                                                         \
  } while (0)
#define CHECK_SFHK(x)                                                         \
  do {                                                                        \
    sfhk_status s_ = (x);                                                     \
    if (s_ != SFHK_OK) {                                                      \
      fprintf(stderr, "%s: %s (%s)\n", #x, sfhk_status_string(s_), sfhk_last_error()); \
      return 3;                                                               \
    }                                                                         \
  } while (0)

static int read_all(FILE* f, void* p, size_t bytes) { return fread(p, 1, bytes, f) == bytes; }

int main(int argc, char** argv) {
  if (argc != 3) return 1;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 1;
  int64_t hdr[6];
  double par[15];
  if (!read_all(f, hdr, sizeof hdr) || !read_all(f, par, sizeof par)) return 1;
  const int64_t n = hdr[0], ns = hdr[1], np = hdr[2], chunk = hdr[5];
  if (n < 1 || ns < 1 || np < 1 || np > SFHK_MAX_PRIM) return 1;
  double* alpha = malloc(np * sizeof(double));
  double* coef = malloc(np * sizeof(double));
  double* host = malloc((size_t)7 * n * sizeof(double));  /* t0, q0[3], p0[3] */
  if (!alpha || !coef || !host) return 1;
  if (!read_all(f, alpha, np * sizeof(double)) || !read_all(f, coef, np * sizeof(double)) ||
      !read_all(f, host, (size_t)7 * n * sizeof(double)))
    return 1;
  fclose(f);

  double* dev = NULL; /* t0 | q0 | p0 */
  CHECK_HIP(hipMalloc((void**)&dev, (size_t)7 * n * sizeof(double)));
  CHECK_HIP(hipMemcpy(dev, host, (size_t)7 * n * sizeof(double), hipMemcpyHostToDevice));

  sfhk_ctx* ctx = NULL;
  CHECK_SFHK(sfhk_ctx_create(0, 0, &ctx));
  const sfhk_potential pot = {(int32_t)hdr[4], par[10], par[11], par[12], par[13], par[14]};
  const sfhk_ground gs = {(int32_t)hdr[3], (int32_t)np, alpha, coef, par[9]};
  const sfhk_pulse pulse = {par[2], par[3], par[4], par[5]};
  const sfhk_grid grid = {par[0], par[1], ns, NULL, &pulse};
  sfhk_params prm = {0};
  prm.gamma = par[6];
  prm.kay_max = par[7];
  prm.overlap_cut = par[8];
  prm.r_fp64 = 2.0;
  prm.precision = SFHK_FP64;
  sfhk_job* job = NULL;
  CHECK_SFHK(sfhk_job_create(ctx, &pot, &gs, &grid, &prm, n, dev, dev + n, dev + 4 * n, NULL, NULL,
                             &job));
  sfhk_status st;
  int launches = 0;
  while ((st = sfhk_propagate(job, chunk, NULL)) == SFHK_E_NOT_DONE) ++launches;
  CHECK_SFHK(st);

  const int64_t m = ns + 1, nk = m / 2 + 1;
  double *d = NULL, *fr = NULL, *om = NULL, *pw = NULL;
  CHECK_HIP(hipMalloc((void**)&d, m * sizeof(double)));
  CHECK_HIP(hipMalloc((void**)&fr, 2 * m * sizeof(double)));
  CHECK_HIP(hipMalloc((void**)&om, nk * sizeof(double)));
  CHECK_HIP(hipMalloc((void**)&pw, nk * sizeof(double)));
  CHECK_SFHK(sfhk_dipole(job, d, fr, NULL));
  CHECK_SFHK(sfhk_spectrum(d, m, par[0], par[1], 0.5 * par[1] * (double)ns, 0, om, pw, NULL, NULL));
  CHECK_HIP(hipDeviceSynchronize());

  double* out = malloc((size_t)(3 * m + nk) * sizeof(double));
  if (!out) return 1;
  CHECK_HIP(hipMemcpy(out, fr, 2 * m * sizeof(double), hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(out + 2 * m, d, m * sizeof(double), hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(out + 3 * m, pw, nk * sizeof(double), hipMemcpyDeviceToHost));
  FILE* g = fopen(argv[2], "wb");
  if (!g || fwrite(out, sizeof(double), (size_t)(3 * m + nk), g) != (size_t)(3 * m + nk)) return 1;
  fclose(g);
  printf("c_api_driver: %lld trajectories, %lld steps, %d chunked calls\n", (long long)n,
         (long long)ns, launches + 1);

  sfhk_job_destroy(job);
  sfhk_ctx_destroy(ctx);
  CHECK_HIP(hipFree(d));
  CHECK_HIP(hipFree(fr));
  CHECK_HIP(hipFree(om));
  CHECK_HIP(hipFree(pw));
  CHECK_HIP(hipFree(dev));
  free(out);
  free(host);
  free(alpha);
  free(coef);
  return 0;
}
