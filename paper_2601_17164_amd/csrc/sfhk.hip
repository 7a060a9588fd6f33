// sfhk.hip -- host runtime of the SFHK hot path (gfx950) behind include/sfhk.h: contexts, jobs,
// launches, batches (graph capture), dipole and spectrum calls. The propagation kernels and the
// device data layout are in sfhk_kernels.hpp, the kernels around them in sfhk_io_kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/sfhk.h"
#include "sfhk_kernels.hpp"
#include "sfhk_io_kernels.hpp"
#include "sfhk_sfa_kernels.hpp"
#include "sfhk_gabor_kernels.hpp"
#include "sfhk_host.hpp"

namespace {

thread_local std::string g_err;

sfhk_status fail(sfhk_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? SFHK_E_NOMEM : SFHK_E_DEVICE,            \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

// a roctx range around a host API call (visible with rocprofv3 --marker-trace; a few nanoseconds
// when no profiler is attached)
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace

// ================================================================================================
// host runtime
// ================================================================================================
struct sfhk_ctx {
  int device;
  size_t budget;
  size_t in_use = 0;
  std::mutex mu;
  // job buffers come from a stream-ordered pool of this context that keeps freed memory for
  // reuse; sfhk_job_destroy frees them on free_stream once the job's last issued work is done
  hipMemPool_t pool = nullptr;
  hipStream_t free_stream = nullptr;
  // staging of sfhk_propagate_many: job descriptors and the combined work list
  JobDev* many_desc = nullptr;
  WorkItem* many_work = nullptr;
  JobDev* many_desc_host = nullptr;  // pinned
  WorkItem* many_work_host = nullptr;
  size_t many_desc_cap = 0, many_work_cap = 0;
};

struct sfhk_job {
  sfhk_ctx* ctx = nullptr;
  JobDev host{};               // host copy of the device descriptor
  JobDev* dev = nullptr;       // device copy
  int kind = 0;
  int precision = 0;
  long long n_traj = 0;
  long long n_out = 0;
  long long* perm = nullptr;   // [n_pad] sorted slot -> original index (-1: padding)
  WorkItem* work = nullptr;    // [n_tiles] (0, t): this job's tiles, longest first
  double* dbuf = nullptr;      // [n_steps+1] dipole on the step grid
  size_t bytes = 0;
  std::vector<void*> allocs;
  hipEvent_t last_use = nullptr;  // recorded after every piece of work issued on the job
  std::vector<int> tile_n0_host;
  long long steps_done = 0;    // steps requested so far (uniform across tiles)
  long long acc_words = 0;     // 64-bit words of the exact accumulators (dipole and velocity)
  uint64_t fingerprint = 0;    // of the inputs that define the propagation (checkpoint matching)
  bool done = false;
  bool regroup = false;  // live trajectories regrouped every compact_every steps (k_propagate_rg)
};

struct sfhk_batch {
  sfhk_ctx* ctx = nullptr;
  int max_jobs = 0;
  long long max_items = 0;
  int64_t max_steps = 0;
  int workers_per_cu = 0;
  int n_workers = 0;
  hipStream_t cap_stream = nullptr;   // private stream used for the capture
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  JobDev* desc = nullptr;             // device, [max_jobs]
  WorkItem* work = nullptr;           // device, [max_items]
  BatchDev* bdev = nullptr;           // device
  // two pinned staging sets, used in turn: set s is refilled only after the replay that followed
  // its last copies has completed (event done[s]), so the host runs at most one replay ahead and
  // never waits for the replay in flight
  JobDev* desc_host[2] = {nullptr, nullptr};
  WorkItem* work_host[2] = {nullptr, nullptr};
  BatchDev* bdev_host[2] = {nullptr, nullptr};
  hipEvent_t done[2] = {nullptr, nullptr};
  bool done_recorded[2] = {false, false};
  int cur = 0;  // set of the latest staging
  std::vector<sfhk_job*> jobs;
  bool staged = false;
  // hardware-dispatch form: the graph's kernel node of each segment, whose grid is resized to the
  // segment's staged tile count before each replay (grid_update), so that no replay dispatches
  // the workgroups of the batch's whole capacity for a segment that holds few tiles or none
  bool grid_update = false;
  hipGraphNode_t seg_node[kSegs] = {};
  const void* seg_fn[kSegs] = {};
  const JobDev* arg_desc = nullptr;
  const WorkItem* arg_work = nullptr;
  const BatchDev* arg_bdev = nullptr;
  int arg_ms = 0;
};

namespace {

// 64-bit words of a job's exact accumulators: two per step (Re, Im) for the dipole, two more for
// the dipole velocity
long long accumulator_words(long long n_steps, int velocity) {
  return (n_steps + 1) * 2 * sfhk_exact::kExactWords * (velocity ? 2 : 1);
}

size_t footprint_bytes(long long n_traj, long long n_steps, int velocity) {
  const long long n_pad = (n_traj + kTile - 1) / kTile * kTile;
  const long long n_tiles = n_pad / kTile;
  size_t b = 0;
  b += (size_t)n_pad * kNY * 8 + (size_t)n_pad * 5 * 8 + (size_t)n_pad * 8 * 2;  // y, aux, n0+death, perm
  b += (size_t)n_tiles * (4 * 3 + sizeof(WorkItem));                             // tile arrays, work list
  b += (size_t)accumulator_words(n_steps, velocity) * 8;
  b += (size_t)(2 * n_steps + 1) * 8;  // field table
  b += (size_t)(n_steps + 1) * 8;      // dipole on the step grid
  b += 64;
  return b;
}

template <typename T>
sfhk_status job_alloc(sfhk_job* j, T** p, size_t count, hipStream_t st) {
  void* q = nullptr;
  const size_t bytes = count * sizeof(T) + 16;
  hipError_t e = hipMallocFromPoolAsync(&q, bytes, j->ctx->pool, st);
  if (e == hipErrorOutOfMemory) {
    // memory freed by destroyed jobs may still wait on the free stream, or sit cached in the
    // pool in blocks too small: let the frees complete, return the cache, try once more
    (void)hipGetLastError();
    (void)hipStreamSynchronize(j->ctx->free_stream);
    (void)hipMemPoolTrimTo(j->ctx->pool, 0);
    e = hipMallocFromPoolAsync(&q, bytes, j->ctx->pool, st);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(SFHK_E_NOMEM, "device allocation failed for a job buffer");
  }
  j->allocs.push_back(q);
  *p = (T*)q;
  return SFHK_OK;
}

// frees the job's buffers in stream order after all work issued on it so far; does not block
void job_free(sfhk_job* j) {
  hipStream_t fs = j->ctx->free_stream;
  if (j->last_use) (void)hipStreamWaitEvent(fs, j->last_use, 0);
  for (void* p : j->allocs) (void)hipFreeAsync(p, fs);
  j->allocs.clear();
}

// records that work touching the job has been issued on `st`
sfhk_status mark_use(sfhk_job* j, hipStream_t st) {
  HIP_TRY(hipEventRecord(j->last_use, st));
  return SFHK_OK;
}

int blocks_for(long long n, int t) { return (int)((n + t - 1) / t); }

// launch the (precision, kind) instance of the propagate kernel
sfhk_status launch_propagate(int precision, int kind, const JobDev* descs, const WorkItem* work,
                             int n_items, int max_steps, hipStream_t st) {
  if (n_items <= 0) return SFHK_OK;
  const dim3 g(n_items), b(kTile);
#define SFHK_LAUNCH(K)                                                                             \
  if (precision == SFHK_FP32_MIXED)                                                                \
    hipLaunchKernelGGL(k_propagate_mixed<K>, g, b, 0, st, descs, work, max_steps);                 \
  else                                                                                             \
    hipLaunchKernelGGL(k_propagate_fp64<K>, g, b, 0, st, descs, work, max_steps);
  switch (kind) {
    case SFHK_POT_SOFTCORE: SFHK_LAUNCH(POT_SOFTCORE) break;
    case SFHK_POT_SCREENED: SFHK_LAUNCH(POT_SCREENED) break;
    case SFHK_POT_HARMONIC: SFHK_LAUNCH(POT_HARMONIC) break;
    default: SFHK_LAUNCH(POT_NONE) break;
  }
#undef SFHK_LAUNCH
  HIP_TRY(hipGetLastError());
  return SFHK_OK;
}

// a job listed twice would have its tiles queued twice: two workgroups racing on one tile's state
bool has_duplicates(sfhk_job* const* jobs, int n_jobs) {
  return sfhk_host::has_duplicates((const void* const*)jobs, n_jobs);
}

int segment_of(int precision, int kind) { return (precision == SFHK_FP32_MIXED ? kKinds : 0) + kind; }

// the regrouping launch of one FP64 job: one workgroup of kRgWaves waves per kRgWaves work items
sfhk_status launch_regroup(sfhk_job* job, int n_items, int max_steps, hipStream_t st) {
  if (n_items <= 0) return SFHK_OK;
  const dim3 g(blocks_for(n_items, kRgWaves)), b(kRgWaves * kTile);
  const JobDev* D = job->dev;
  const WorkItem* W = job->work;
  switch (job->kind) {
    case SFHK_POT_SOFTCORE: hipLaunchKernelGGL(k_propagate_rg<POT_SOFTCORE>, g, b, 0, st, D, W, n_items, max_steps); break;
    case SFHK_POT_SCREENED: hipLaunchKernelGGL(k_propagate_rg<POT_SCREENED>, g, b, 0, st, D, W, n_items, max_steps); break;
    case SFHK_POT_HARMONIC: hipLaunchKernelGGL(k_propagate_rg<POT_HARMONIC>, g, b, 0, st, D, W, n_items, max_steps); break;
    default: hipLaunchKernelGGL(k_propagate_rg<POT_NONE>, g, b, 0, st, D, W, n_items, max_steps); break;
  }
  HIP_TRY(hipGetLastError());
  return SFHK_OK;
}

}  // namespace

namespace {

using sfhk_host::CkptHeader;
using sfhk_host::kCkptAlign;
using sfhk_host::kCkptMagic;

// (device pointer of the job, bytes) of every section after the header, in checkpoint order
std::vector<std::pair<void*, size_t>> ckpt_sections(sfhk_job* j) {
  const JobDev& H = j->host;
  const size_t np = (size_t)H.n_pad, nt = (size_t)H.n_tiles;
  std::vector<std::pair<void*, size_t>> v = {{H.y, np * kNY * sizeof(double)},
                                              {H.aux, np * 5 * sizeof(double)},
                                              {H.death, np * sizeof(int)},
                                              {H.tile_next, nt * sizeof(int)},
                                              {H.tile_last, nt * sizeof(int)},
                                              {H.counters, 8 * sizeof(unsigned long long)},
                                              {H.acc, (size_t)j->acc_words * sizeof(long long)}};
  if (j->regroup) {  // regrouping moves trajectories between slots and tiles
    v.push_back({H.n0, np * sizeof(int)});
    v.push_back({H.perm, np * sizeof(long long)});
  }
  return v;
}

// offsets of the sections in a checkpoint; returns its size
size_t ckpt_offsets(sfhk_job* j, std::vector<std::pair<void*, size_t>>& secs, std::vector<size_t>& off) {
  secs = ckpt_sections(j);
  std::vector<size_t> bytes(secs.size());
  for (size_t i = 0; i < secs.size(); ++i) bytes[i] = secs[i].second;
  return sfhk_host::ckpt_layout(bytes, off);
}

size_t ckpt_bytes(sfhk_job* j) {
  std::vector<std::pair<void*, size_t>> secs;
  std::vector<size_t> off;
  return ckpt_offsets(j, secs, off);
}

// the header a checkpoint of this job carries
CkptHeader ckpt_header(const sfhk_job* job) {
  CkptHeader h{};
  h.magic = kCkptMagic;
  h.n_traj = job->n_traj;
  h.n_pad = job->host.n_pad;
  h.n_tiles = job->host.n_tiles;
  h.n_steps = job->host.n_steps;
  h.acc_words = job->acc_words;
  h.steps_done = job->steps_done;
  h.kind = job->kind;
  h.precision = job->precision;
  h.done = job->done ? 1 : 0;
  h.fingerprint = job->fingerprint;
  return h;
}

}  // namespace

extern "C" {

const char* sfhk_last_error(void) { return g_err.c_str(); }

const char* sfhk_status_string(sfhk_status s) {
  switch (s) {
    case SFHK_OK: return "ok";
    case SFHK_E_INVALID: return "invalid argument";
    case SFHK_E_NOMEM: return "out of device memory";
    case SFHK_E_DEVICE: return "HIP runtime error";
    case SFHK_E_NOT_DONE: return "not done";
    case SFHK_E_BUDGET: return "HBM budget exceeded";
  }
  return "unknown status";
}

sfhk_status sfhk_ctx_create(int device, size_t hbm_budget_bytes, sfhk_ctx** out) {
  if (!out) return fail(SFHK_E_INVALID, "out is NULL");
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(SFHK_E_INVALID, "device index out of range");
  HIP_TRY(hipSetDevice(device));
  sfhk_ctx* c = new sfhk_ctx();
  c->device = device;
  c->budget = hbm_budget_bytes;
  hipMemPoolProps props = {};
  props.allocType = hipMemAllocationTypePinned;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = device;
  hipError_t e = hipMemPoolCreate(&c->pool, &props);
  if (e == hipSuccess) {
    uint64_t keep = UINT64_MAX;  // keep freed memory cached for the next jobs
    e = hipMemPoolSetAttribute(c->pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  if (e == hipSuccess) {
    int no = 0;  // never make an allocating stream wait for another stream's frees
    e = hipMemPoolSetAttribute(c->pool, hipMemPoolReuseAllowInternalDependencies, &no);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->free_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    if (c->free_stream) (void)hipStreamDestroy(c->free_stream);
    if (c->pool) (void)hipMemPoolDestroy(c->pool);
    delete c;
    return fail(SFHK_E_DEVICE, std::string("context set-up: ") + hipGetErrorString(e));
  }
  *out = c;
  return SFHK_OK;
}

void sfhk_ctx_destroy(sfhk_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(ctx->many_desc);
  (void)hipFree(ctx->many_work);
  (void)hipHostFree(ctx->many_desc_host);
  (void)hipHostFree(ctx->many_work_host);
  if (ctx->free_stream) (void)hipStreamDestroy(ctx->free_stream);
  if (ctx->pool) (void)hipMemPoolDestroy(ctx->pool);
  delete ctx;
}

size_t sfhk_ctx_bytes_in_use(const sfhk_ctx* ctx) { return ctx ? ctx->in_use : 0; }

size_t sfhk_job_footprint(int64_t n_traj, int64_t n_steps, int64_t n_out, int32_t precision,
                          int32_t velocity) {
  (void)precision;
  if (n_traj < 1 || n_steps < 1) return 0;
  (void)n_out;
  return footprint_bytes(n_traj, n_steps, velocity != 0);
}

int64_t sfhk_job_n_out(const sfhk_job* job) {
  if (!job) return 0;
  return job->n_out > 0 ? job->n_out : (int64_t)job->host.n_steps + 1;
}

sfhk_status sfhk_job_create(sfhk_ctx* ctx, const sfhk_potential* pot, const sfhk_ground* ground,
                            const sfhk_grid* grid, const sfhk_params* params, int64_t n_traj,
                            const double* t0, const double* q0, const double* p0, const double* w,
                            void* stream, sfhk_job** out) {
  TraceRange trace_("sfhk_job_create");
  if (!ctx || !pot || !ground || !grid || !params || !t0 || !q0 || !p0 || !out)
    return fail(SFHK_E_INVALID, "NULL argument");
  if (!(params->gamma > 0.0)) return fail(SFHK_E_INVALID, "gamma must be > 0");
  if (!(params->kay_max > 0.0)) return fail(SFHK_E_INVALID, "kay_max must be > 0 (+inf: no Kay removal)");
  if (!(params->overlap_cut >= 0.0))
    return fail(SFHK_E_INVALID, "overlap_cut must be >= 0 (+inf: no primitive skipped)");
  if (params->precision == SFHK_FP32_MIXED && !(params->r_fp64 >= 0.0))
    return fail(SFHK_E_INVALID, "r_fp64 must be >= 0");
  if (!(grid->h > 0.0)) return fail(SFHK_E_INVALID, "h must be > 0");
  if (grid->n_steps < 1 || grid->n_steps > (1LL << 30)) return fail(SFHK_E_INVALID, "n_steps out of range");
  if (!grid->e_half && !grid->pulse) return fail(SFHK_E_INVALID, "the grid needs e_half or a pulse");
  if (const sfhk_pulse* pl = grid->pulse)
    if (!(std::isfinite(pl->e0) && pl->omega > 0.0 && std::isfinite(pl->omega) && pl->n_cycles > 0.0 &&
          std::isfinite(pl->n_cycles) && std::isfinite(pl->cep)))
      return fail(SFHK_E_INVALID, "pulse: need finite e0 and cep, omega > 0, n_cycles > 0");
  if (n_traj < 1 || n_traj > (1LL << 31)) return fail(SFHK_E_INVALID, "n_traj out of range");
  if (ground->l != 0 && ground->l != 1) return fail(SFHK_E_INVALID, "ground-state l must be 0 or 1");
  if (ground->n_prim < 1 || ground->n_prim > SFHK_MAX_PRIM || !ground->alpha || !ground->coef)
    return fail(SFHK_E_INVALID, "n_prim must be in 1..SFHK_MAX_PRIM with alpha/coef given");
  if (pot->kind < SFHK_POT_NONE || pot->kind > SFHK_POT_HARMONIC)
    return fail(SFHK_E_INVALID, "unknown potential kind");
  if (pot->kind == SFHK_POT_SCREENED && !(pot->r_scr > 0.0))
    return fail(SFHK_E_INVALID, "r_scr must be > 0");
  if (params->precision != SFHK_FP64 && params->precision != SFHK_FP32_MIXED)
    return fail(SFHK_E_INVALID, "unknown precision");
  if (params->n_out < 0) return fail(SFHK_E_INVALID, "n_out must be >= 0");
  if (params->velocity != 0 && params->velocity != 1) return fail(SFHK_E_INVALID, "velocity must be 0 or 1");
  if (params->pw_mask < 0 || params->pw_mask > 0x1FF) return fail(SFHK_E_INVALID, "pw_mask must be in [0, 0x1FF]");
  if (params->pw_mask && !(params->pw_radius > 0.0 && std::isfinite(params->pw_radius)))
    return fail(SFHK_E_INVALID, "pw_radius must be finite and > 0");
  if (params->compact_every != 0 && (params->compact_every < 16 || params->compact_every > (1 << 24)))
    return fail(SFHK_E_INVALID, "compact_every must be 0 or in [16, 2^24]");
  if (params->compact_every != 0 && params->precision != SFHK_FP64)
    return fail(SFHK_E_INVALID, "compact_every: regrouping runs in the FP64 form only");
  for (int j = 0; j < ground->n_prim; ++j)
    if (!(ground->alpha[j] > 0.0)) return fail(SFHK_E_INVALID, "GTO exponents must be > 0");

  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const long long N = n_traj;
  const int NS = (int)grid->n_steps;

  const long long n_pad = (N + kTile - 1) / kTile * kTile;
  const int n_tiles = (int)(n_pad / kTile);
  const double t_b = grid->t_a + (double)NS * grid->h;

  sfhk_job* j = new sfhk_job();
  j->ctx = ctx;
  if (hipEventCreateWithFlags(&j->last_use, hipEventDisableTiming) != hipSuccess) {
    delete j;
    return fail(SFHK_E_DEVICE, "hipEventCreateWithFlags failed");
  }
  size_t bytes = 0;  // counted against the budget once known
  auto cleanup = [&](sfhk_status s) {
    (void)hipEventRecord(j->last_use, st);  // work already issued on st finishes before the frees
    job_free(j);
    (void)hipEventDestroy(j->last_use);
    if (bytes) {
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->in_use -= bytes;
    }
    delete j;
    return s;
  };
#define TRY_C(expr)                                                              \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) return cleanup(fail(SFHK_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_))); \
  } while (0)
  JobDev& H = j->host;
  sfhk_status rc;

  // birth steps on the device (k_birth); the host reads back only each tile's first birth step and
  // two flags unless the samples are not in birth order
  unsigned long long* flags = nullptr;
  if ((rc = job_alloc(j, &H.n0, (size_t)n_pad, st)) || (rc = job_alloc(j, &H.tile_n0, (size_t)n_tiles, st)) ||
      (rc = job_alloc(j, &flags, 2, st)))
    return cleanup(rc);
  TRY_C(hipMemsetAsync(flags, 0xFF, sizeof(unsigned long long), st));
  TRY_C(hipMemsetAsync(flags + 1, 0, sizeof(unsigned long long), st));
  hipLaunchKernelGGL(k_birth, dim3(blocks_for(n_pad, 256)), dim3(256), 0, st, t0, N, n_pad,
                     grid->t_a, grid->h, grid->t_a - 0.5 * grid->h, t_b + 0.5 * grid->h, NS, H.n0,
                     H.tile_n0, flags);
  TRY_C(hipGetLastError());
  unsigned long long fl[2] = {0, 0};
  std::vector<int> tile_n0(n_tiles);
  TRY_C(hipMemcpyAsync(fl, flags, sizeof(fl), hipMemcpyDeviceToHost, st));
  TRY_C(hipMemcpyAsync(tile_n0.data(), H.tile_n0, n_tiles * sizeof(int), hipMemcpyDeviceToHost, st));
  TRY_C(hipStreamSynchronize(st));
  if (fl[0] != ~0ull)
    return cleanup(fail(SFHK_E_INVALID, "t0[" + std::to_string(fl[0]) + "] outside the time grid"));
  // stable order by birth step: the identity when the samples already come in birth order (the
  // usual layout), else a counting sort over the grid steps 0..NS on the host
  const bool in_order = fl[1] == 0;
  std::vector<long long> perm;
  std::vector<int> n0s;
  if (!in_order) {
    std::vector<int> n0h(N);
    TRY_C(hipMemcpyAsync(n0h.data(), H.n0, N * sizeof(int), hipMemcpyDeviceToHost, st));
    TRY_C(hipStreamSynchronize(st));
    if (!sfhk_host::birth_sort(n0h.data(), N, NS, n_pad, perm, n0s))
      return cleanup(fail(SFHK_E_DEVICE, "birth steps out of range"));
    sfhk_host::tile_first_steps(n0s, kTile, tile_n0);
  }
  std::vector<int> tile_next, tile_last;
  sfhk_host::tile_progress(tile_n0, tile_next, tile_last);
  const long long acc_words = accumulator_words(NS, params->velocity != 0);
  const size_t need = footprint_bytes(N, NS, params->velocity != 0);
  bool over = false;
  size_t left = 0;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->budget && ctx->in_use + need > ctx->budget) {
      over = true;
      left = ctx->budget - ctx->in_use;
    } else {
      ctx->in_use += need;
    }
  }
  if (over)
    return cleanup(fail(SFHK_E_BUDGET, "job needs " + std::to_string(need) + " bytes; budget left " +
                                           std::to_string(left)));
  bytes = need;

  j->kind = pot->kind;
  j->precision = params->precision;
  j->n_traj = N;
  j->n_out = params->n_out;
  j->bytes = bytes;
  j->tile_n0_host = tile_n0;
  j->acc_words = acc_words;
  // fast range of the screened potential: 2^-1000 <= r^2 <= 2^999 and 0 <= a <= 2^999 keep r^2
  // and r^2 + a within the square root's core range
  const double r2_fast = (pot->kind == SFHK_POT_SCREENED && pot->soft2 >= 0.0 && pot->soft2 <= 0x1p999)
                             ? 0x1p999 : -1.0;
  H.pot = {pot->z_inf, pot->z_in, pot->r_scr, pot->soft2, pot->omega_ho,
           pot->kind == SFHK_POT_SCREENED ? 1.0 / pot->r_scr : 0.0, r2_fast};
  const double g = params->gamma;
  H.gto.l = ground->l;
  H.gto.n_prim = ground->n_prim;
  for (int k = 0; k < ground->n_prim; ++k) {
    const double a = ground->alpha[k];
    const double ga = g + a;
    H.gto.A[k] = 1.0 / (4.0 * ga);
    H.gto.B[k] = a * g / ga;
    H.gto.D[k] = a / ga;
    H.gto.N[k] = ground->coef[k] * std::pow(ga, ground->l == 0 ? -2.5 : -3.5);
    H.gto.G2[k] = 2.0 * ga;
    H.gto.Va[k] = a;
    H.gto.Vg[k] = 2.0 * g * ga;
  }
  H.gto.vel = params->velocity;
  H.pw_mask = params->pw_mask;
  H.pw_r2 = params->pw_mask ? params->pw_radius * params->pw_radius : 0.0;
  H.gto.two_gamma = 2.0 * g;
  H.gto.ip = ground->ip;
  H.gto.Amin = H.gto.A[0];
  H.gto.Bmin = H.gto.B[0];
  for (int k = 1; k < ground->n_prim; ++k) {
    H.gto.Amin = std::min(H.gto.Amin, H.gto.A[k]);
    H.gto.Bmin = std::min(H.gto.Bmin, H.gto.B[k]);
  }
  H.gto.cut_hi = params->overlap_cut * (1.0 + 1e-12);
  H.kind = pot->kind;
  H.gamma = g;
  H.inv4g = 1.0 / (4.0 * g);
  H.kay2 = params->kay_max * params->kay_max;
  H.cut = params->overlap_cut;
  H.r64sq = params->r_fp64 * params->r_fp64;
  H.t_a = grid->t_a;
  H.h = grid->h;
  H.h2 = 0.5 * grid->h;
  H.h6 = grid->h / 6.0;
  H.n_steps = NS;
  H.n_tiles = n_tiles;
  H.n_pad = n_pad;
  {
    // FNV-1a over the parameters that define the propagation (not the field table's values)
    uint64_t fp = 1469598103934665603ULL;
    auto mix = [&fp](const void* p, size_t n) {
      const unsigned char* b = (const unsigned char*)p;
      for (size_t i = 0; i < n; ++i) fp = (fp ^ b[i]) * 1099511628211ULL;
    };
    mix(pot, sizeof(*pot));
    mix(&ground->l, sizeof(ground->l));
    mix(&ground->ip, sizeof(ground->ip));
    mix(ground->alpha, sizeof(double) * (size_t)ground->n_prim);
    mix(ground->coef, sizeof(double) * (size_t)ground->n_prim);
    mix(&grid->t_a, sizeof(grid->t_a));
    mix(&grid->h, sizeof(grid->h));
    if (grid->pulse) mix(grid->pulse, sizeof(*grid->pulse));
    const double pv[5] = {params->gamma, params->kay_max, params->overlap_cut, params->r_fp64,
                          params->pw_mask ? params->pw_radius : 0.0};
    const int64_t iv[5] = {params->precision, params->n_out, params->velocity, params->pw_mask,
                           params->compact_every};
    mix(pv, sizeof(pv));
    mix(iv, sizeof(iv));
    j->fingerprint = fp;
  }

  double* e_half = nullptr;
  if ((rc = job_alloc(j, &e_half, 2 * (size_t)NS + 1, st)) || (rc = job_alloc(j, &H.y, (size_t)n_pad * kNY, st)) ||
      (rc = job_alloc(j, &H.aux, (size_t)n_pad * 5, st)) || (rc = job_alloc(j, &H.death, (size_t)n_pad, st)) ||
      (rc = job_alloc(j, &H.tile_next, (size_t)n_tiles, st)) || (rc = job_alloc(j, &H.tile_last, (size_t)n_tiles, st)) ||
      (rc = job_alloc(j, &H.acc, (size_t)acc_words, st)) ||
      (rc = job_alloc(j, &H.counters, 8, st)) || (rc = job_alloc(j, &j->work, (size_t)n_tiles, st)) ||
      (rc = job_alloc(j, &j->dbuf, (size_t)NS + 1, st)) || (rc = job_alloc(j, &j->dev, 1, st)))
    return cleanup(rc);
  const bool regroup = params->compact_every > 0;
  if ((!in_order || regroup) && (rc = job_alloc(j, &j->perm, (size_t)n_pad, st))) return cleanup(rc);
  j->regroup = regroup;
  H.compact_every = params->compact_every;
  H.perm = j->perm;
  H.e_half = e_half;
  H.acc_v = params->velocity ? H.acc + acc_words / 2 : nullptr;
  if (grid->e_half)
    TRY_C(hipMemcpyAsync(e_half, grid->e_half, (2 * (size_t)NS + 1) * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (const sfhk_pulse* pl = grid->pulse) {
    // tabulate the pulse's field, or check the given table against it (flags[0] = mismatch)
    TRY_C(hipMemsetAsync(flags, 0, sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_field_table, dim3(blocks_for(2 * (long long)NS + 1, 256)), dim3(256), 0, st,
                       pl->e0, pl->omega, pl->n_cycles, pl->cep, grid->t_a, grid->h, (long long)NS,
                       grid->e_half ? nullptr : e_half, grid->e_half ? e_half : nullptr, flags,
                       1e-9 * std::fabs(pl->e0));
    TRY_C(hipGetLastError());
    if (grid->e_half) {
      unsigned long long mismatch = 0;
      TRY_C(hipMemcpyAsync(&mismatch, flags, sizeof(mismatch), hipMemcpyDeviceToHost, st));
      TRY_C(hipStreamSynchronize(st));
      if (mismatch)
        return cleanup(fail(SFHK_E_INVALID, "e_half differs from the pulse's field by more than 1e-9 e0"));
    }
  }
  if (regroup && in_order) {  // slots hold the samples in caller order; regrouping moves them
    perm.resize(n_pad);
    for (long long i = 0; i < n_pad; ++i) perm[i] = i < N ? i : -1;
  }
  if (regroup || !in_order)
    TRY_C(hipMemcpyAsync(j->perm, perm.data(), n_pad * sizeof(long long), hipMemcpyHostToDevice, st));
  if (!in_order) {  // the sorted order replaces the caller order k_birth wrote
    TRY_C(hipMemcpyAsync(H.n0, n0s.data(), n_pad * sizeof(int), hipMemcpyHostToDevice, st));
    TRY_C(hipMemcpyAsync(H.tile_n0, tile_n0.data(), n_tiles * sizeof(int), hipMemcpyHostToDevice, st));
  }
  TRY_C(hipMemcpyAsync(H.tile_next, tile_next.data(), n_tiles * sizeof(int), hipMemcpyHostToDevice, st));
  TRY_C(hipMemcpyAsync(H.tile_last, tile_last.data(), n_tiles * sizeof(int), hipMemcpyHostToDevice, st));
  std::vector<WorkItem> work(n_tiles);
  for (int t = 0; t < n_tiles; ++t) work[t] = {0, t};
  TRY_C(hipMemcpyAsync(j->work, work.data(), n_tiles * sizeof(WorkItem), hipMemcpyHostToDevice, st));
  TRY_C(hipMemsetAsync(H.counters, 0, 8 * sizeof(unsigned long long), st));
  TRY_C(hipMemsetAsync(H.acc, 0, (size_t)acc_words * sizeof(long long), st));  // exact sums start at 0
  TRY_C(hipMemcpyAsync(j->dev, &H, sizeof(JobDev), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_init, dim3(blocks_for(n_pad, 256)), dim3(256), 0, st, H, j->perm, N, q0, p0, w);
  TRY_C(hipGetLastError());
  TRY_C(hipEventRecord(j->last_use, st));
  // the host vectors above are about to go out of scope: finish the copies before returning
  TRY_C(hipStreamSynchronize(st));
#undef TRY_C
  *out = j;
  return SFHK_OK;
}

void sfhk_job_destroy(sfhk_job* job) {
  if (!job) return;
  (void)hipSetDevice(job->ctx->device);
  job_free(job);
  if (job->last_use) (void)hipEventDestroy(job->last_use);
  {
    std::lock_guard<std::mutex> lk(job->ctx->mu);
    job->ctx->in_use -= job->bytes;
  }
  delete job;
}

// number of tiles that still have steps left after `done` steps have been requested
static int unfinished_tiles(const sfhk_job* j, long long done) {
  return sfhk_host::unfinished_tiles(j->tile_n0_host, j->host.n_steps, done);
}

// the longest-first work list over the unfinished tiles of the jobs, grouped by kernel segment
static std::vector<sfhk_host::Item> work_items(sfhk_job* const* jobs, int n_jobs) {
  std::vector<sfhk_host::JobProgress> jp((size_t)n_jobs);
  for (int i = 0; i < n_jobs; ++i)
    jp[(size_t)i] = {&jobs[i]->tile_n0_host, jobs[i]->host.n_steps, jobs[i]->steps_done,
                     jobs[i]->done, segment_of(jobs[i]->precision, jobs[i]->kind)};
  return sfhk_host::work_items(jp);
}

sfhk_status sfhk_propagate(sfhk_job* job, int64_t max_steps, void* stream) {
  TraceRange trace_("sfhk_propagate");
  if (!job) return fail(SFHK_E_INVALID, "job is NULL");
  if (job->done) return SFHK_OK;
  HIP_TRY(hipSetDevice(job->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int NS = job->host.n_steps;
  const int nt = unfinished_tiles(job, job->steps_done);
  if (nt > 0) {
    int ms = (max_steps <= 0 || max_steps > NS + 1) ? 0 : (int)max_steps;
    sfhk_status rc = job->regroup
                         ? launch_regroup(job, nt, ms, st)
                         : launch_propagate(job->precision, job->kind, job->dev, job->work, nt, ms, st);
    if (rc) return rc;
    if ((rc = mark_use(job, st))) return rc;
  }
  job->steps_done += (max_steps <= 0) ? (long long)NS + 1 : max_steps;
  if (unfinished_tiles(job, job->steps_done) == 0) {
    job->done = true;
    return SFHK_OK;
  }
  return SFHK_E_NOT_DONE;
}

sfhk_status sfhk_propagate_many(sfhk_job* const* jobs, int32_t n_jobs, int64_t max_steps, void* stream) {
  TraceRange trace_("sfhk_propagate_many");
  if (!jobs || n_jobs < 0) return fail(SFHK_E_INVALID, "bad job list");
  if (n_jobs == 0) return SFHK_OK;
  sfhk_ctx* ctx = jobs[0] ? jobs[0]->ctx : nullptr;
  for (int i = 0; i < n_jobs; ++i)
    if (!jobs[i] || jobs[i]->ctx != ctx) return fail(SFHK_E_INVALID, "jobs must be non-NULL and share one context");
  if (has_duplicates(jobs, n_jobs)) return fail(SFHK_E_INVALID, "a job is listed more than once");
  for (int i = 0; i < n_jobs; ++i)
    if (jobs[i]->regroup) return fail(SFHK_E_INVALID, "a job created with compact_every runs through sfhk_propagate only");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  // one launch per (precision, potential kind) kernel over the unfinished tiles of every job,
  // each ordered by steps left (longest first)
  const std::vector<sfhk_host::Item> items = work_items(jobs, n_jobs);
  if (!items.empty()) {
    HIP_TRY(hipStreamSynchronize(st));  // the staging buffers of the previous call are free
    if (ctx->many_desc_cap < (size_t)n_jobs) {
      (void)hipFree(ctx->many_desc);
      (void)hipHostFree(ctx->many_desc_host);
      ctx->many_desc = nullptr;
      ctx->many_desc_host = nullptr;
      ctx->many_desc_cap = 0;
      HIP_TRY(hipMalloc(&ctx->many_desc, n_jobs * sizeof(JobDev)));
      HIP_TRY(hipHostMalloc(&ctx->many_desc_host, n_jobs * sizeof(JobDev), hipHostMallocDefault));
      ctx->many_desc_cap = n_jobs;
    }
    if (ctx->many_work_cap < items.size()) {
      (void)hipFree(ctx->many_work);
      (void)hipHostFree(ctx->many_work_host);
      ctx->many_work = nullptr;
      ctx->many_work_host = nullptr;
      ctx->many_work_cap = 0;
      HIP_TRY(hipMalloc(&ctx->many_work, items.size() * sizeof(WorkItem)));
      HIP_TRY(hipHostMalloc(&ctx->many_work_host, items.size() * sizeof(WorkItem), hipHostMallocDefault));
      ctx->many_work_cap = items.size();
    }
    for (int i = 0; i < n_jobs; ++i) ctx->many_desc_host[i] = jobs[i]->host;
    for (size_t k = 0; k < items.size(); ++k) ctx->many_work_host[k] = {items[k].job, items[k].tile};
    HIP_TRY(hipMemcpyAsync(ctx->many_desc, ctx->many_desc_host, n_jobs * sizeof(JobDev), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(ctx->many_work, ctx->many_work_host, items.size() * sizeof(WorkItem), hipMemcpyHostToDevice, st));
    int ms = (max_steps <= 0 || max_steps > INT32_MAX / 2) ? 0 : (int)max_steps;
    size_t a = 0;
    while (a < items.size()) {
      size_t b = a;
      while (b < items.size() && items[b].seg == items[a].seg) ++b;
      const int sg = items[a].seg;
      sfhk_status rc = launch_propagate(sg >= kKinds ? SFHK_FP32_MIXED : SFHK_FP64, sg % kKinds,
                                        ctx->many_desc, ctx->many_work + a, (int)(b - a), ms, st);
      if (rc) return rc;
      a = b;
    }
    for (int i = 0; i < n_jobs; ++i)
      if (!jobs[i]->done) HIP_TRY(hipEventRecord(jobs[i]->last_use, st));
  }
  sfhk_status agg = SFHK_OK;
  for (int i = 0; i < n_jobs; ++i) {
    sfhk_job* j = jobs[i];
    if (j->done) continue;
    const int NS = j->host.n_steps;
    j->steps_done += (max_steps <= 0) ? (long long)NS + 1 : max_steps;
    if (unfinished_tiles(j, j->steps_done) == 0)
      j->done = true;
    else
      agg = SFHK_E_NOT_DONE;
  }
  return agg;
}

// ------------------------------------------------------------------------------------------------
// batched, graph-captured propagation
// ------------------------------------------------------------------------------------------------
void sfhk_batch_destroy(sfhk_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->ctx->device);
  (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  (void)hipFree(b->desc);
  (void)hipFree(b->work);
  (void)hipFree(b->bdev);
  for (int s = 0; s < 2; ++s) {
    (void)hipHostFree(b->desc_host[s]);
    (void)hipHostFree(b->work_host[s]);
    (void)hipHostFree(b->bdev_host[s]);
    if (b->done[s]) (void)hipEventDestroy(b->done[s]);
  }
  delete b;
}

sfhk_status sfhk_batch_create(sfhk_ctx* ctx, int32_t max_jobs, int64_t max_tiles, int64_t max_steps,
                              int32_t workers_per_cu, sfhk_batch** out) {
  if (!ctx || !out) return fail(SFHK_E_INVALID, "NULL argument");
  if (max_jobs < 1 || max_tiles < 1 || max_tiles > INT32_MAX)
    return fail(SFHK_E_INVALID, "max_jobs and max_tiles must be >= 1 (max_tiles < 2^31)");
  if (workers_per_cu < 0 || workers_per_cu > 64) return fail(SFHK_E_INVALID, "workers_per_cu must be in 0..64");
  HIP_TRY(hipSetDevice(ctx->device));
  int cus = 0;
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
  sfhk_batch* b = new sfhk_batch();
  b->ctx = ctx;
  b->max_jobs = max_jobs;
  b->max_items = max_tiles;
  b->max_steps = max_steps;
  b->workers_per_cu = workers_per_cu;
  b->n_workers = workers_per_cu * cus;
  auto bail = [&](sfhk_status st) {
    sfhk_batch_destroy(b);
    return st;
  };
#define TRY_B(expr)                                                                               \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess)                                                                         \
      return bail(fail(e_ == hipErrorOutOfMemory ? SFHK_E_NOMEM : SFHK_E_DEVICE,                  \
                       std::string(#expr) + ": " + hipGetErrorString(e_)));                       \
  } while (0)
  TRY_B(hipMalloc(&b->desc, (size_t)max_jobs * sizeof(JobDev)));
  TRY_B(hipMalloc(&b->work, (size_t)max_tiles * sizeof(WorkItem)));
  TRY_B(hipMalloc(&b->bdev, sizeof(BatchDev)));
  for (int s = 0; s < 2; ++s) {
    TRY_B(hipHostMalloc(&b->desc_host[s], (size_t)max_jobs * sizeof(JobDev), hipHostMallocDefault));
    TRY_B(hipHostMalloc(&b->work_host[s], (size_t)max_tiles * sizeof(WorkItem), hipHostMallocDefault));
    TRY_B(hipHostMalloc(&b->bdev_host[s], sizeof(BatchDev), hipHostMallocDefault));
    TRY_B(hipEventCreateWithFlags(&b->done[s], hipEventDisableTiming));
  }
  TRY_B(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  std::memset(b->bdev_host[0], 0, sizeof(BatchDev));
  TRY_B(hipMemcpyAsync(b->bdev, b->bdev_host[0], sizeof(BatchDev), hipMemcpyHostToDevice, b->cap_stream));
  TRY_B(hipStreamSynchronize(b->cap_stream));
  const int ms = (max_steps <= 0 || max_steps > INT32_MAX / 2) ? 0 : (int)max_steps;
  // capture: reset the queue heads with a kernel (no memset node), then one kernel per precision
  TRY_B(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, b->cap_stream, b->bdev);
  {
    const JobDev* D = b->desc;
    const WorkItem* W = b->work;
    BatchDev* BD = b->bdev;
    const dim3 gq(b->n_workers), gg((unsigned)max_tiles), bl(kTile);
    hipStream_t cs = b->cap_stream;
#define SFHK_CAPTURE(K)                                                                            \
    if (workers_per_cu > 0) {                                                                      \
      hipLaunchKernelGGL(k_queue_fp64<K>, gq, bl, 0, cs, D, W, BD, ms);                             \
      hipLaunchKernelGGL(k_queue_mixed<K>, gq, bl, 0, cs, D, W, BD, ms);                            \
    } else {                                                                                       \
      hipLaunchKernelGGL(k_grid_fp64<K>, gg, bl, 0, cs, D, W, (const BatchDev*)BD, ms);            \
      hipLaunchKernelGGL(k_grid_mixed<K>, gg, bl, 0, cs, D, W, (const BatchDev*)BD, ms);           \
    }
    SFHK_CAPTURE(POT_NONE)
    SFHK_CAPTURE(POT_SOFTCORE)
    SFHK_CAPTURE(POT_SCREENED)
    SFHK_CAPTURE(POT_HARMONIC)
#undef SFHK_CAPTURE
  }
  hipError_t le = hipGetLastError();
  hipGraph_t g = nullptr;
  hipError_t ce = hipStreamEndCapture(b->cap_stream, &g);
  b->graph = g;
  TRY_B(le);
  TRY_B(ce);
  TRY_B(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  if (workers_per_cu == 0) {  // find each segment's kernel node (else the grids stay at capacity)
    const void* fns[kSegs] = {
        (const void*)k_grid_fp64<POT_NONE>,      (const void*)k_grid_fp64<POT_SOFTCORE>,
        (const void*)k_grid_fp64<POT_SCREENED>,  (const void*)k_grid_fp64<POT_HARMONIC>,
        (const void*)k_grid_mixed<POT_NONE>,     (const void*)k_grid_mixed<POT_SOFTCORE>,
        (const void*)k_grid_mixed<POT_SCREENED>, (const void*)k_grid_mixed<POT_HARMONIC>};
    static_assert(POT_NONE == 0 && POT_SOFTCORE == 1 && POT_SCREENED == 2 && POT_HARMONIC == 3 &&
                      kSegs == 8, "segment order");
    size_t nn = 0;
    int found = 0;
    if (hipGraphGetNodes(b->graph, nullptr, &nn) == hipSuccess && nn > 0) {
      std::vector<hipGraphNode_t> nodes(nn);
      if (hipGraphGetNodes(b->graph, nodes.data(), &nn) == hipSuccess) {
        for (hipGraphNode_t nd : nodes) {
          hipGraphNodeType ty;
          hipKernelNodeParams kp{};
          if (hipGraphNodeGetType(nd, &ty) != hipSuccess || ty != hipGraphNodeTypeKernel ||
              hipGraphKernelNodeGetParams(nd, &kp) != hipSuccess)
            continue;
          for (int g = 0; g < kSegs; ++g)
            if (kp.func == fns[g] && !b->seg_node[g]) {
              b->seg_node[g] = nd;
              b->seg_fn[g] = fns[g];
              ++found;
            }
        }
      }
    }
    b->arg_desc = b->desc;
    b->arg_work = b->work;
    b->arg_bdev = b->bdev;
    b->arg_ms = ms;
    b->grid_update = found == kSegs;
    (void)hipGetLastError();  // a failed lookup only keeps the grids at capacity
  }
#undef TRY_B
  *out = b;
  return SFHK_OK;
}

sfhk_status sfhk_batch_set_jobs(sfhk_batch* b, sfhk_job* const* jobs, int32_t n_jobs, void* stream) {
  TraceRange trace_("sfhk_batch_set_jobs");
  if (!b || (!jobs && n_jobs > 0) || n_jobs < 0) return fail(SFHK_E_INVALID, "bad batch or job list");
  if (n_jobs > b->max_jobs) return fail(SFHK_E_INVALID, "more jobs than the batch was created for");
  for (int i = 0; i < n_jobs; ++i)
    if (!jobs[i] || jobs[i]->ctx != b->ctx) return fail(SFHK_E_INVALID, "jobs must be non-NULL and share the batch's context");
  if (has_duplicates(jobs, n_jobs)) return fail(SFHK_E_INVALID, "a job is listed more than once");
  for (int i = 0; i < n_jobs; ++i)
    if (jobs[i]->regroup) return fail(SFHK_E_INVALID, "a job created with compact_every runs through sfhk_propagate only");
  HIP_TRY(hipSetDevice(b->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const std::vector<sfhk_host::Item> items = work_items(jobs, n_jobs);
  if ((long long)items.size() > b->max_items) return fail(SFHK_E_INVALID, "more unfinished tiles than the batch was created for");
  // the other staging set than the latest one; its copies were followed by a replay (or by
  // nothing) recorded in done[s]
  const int s = b->cur ^ 1;
  if (b->done_recorded[s]) HIP_TRY(hipEventSynchronize(b->done[s]));
  BatchDev bd{};
  sfhk_host::segment_table(items, kSegs, bd.n_items, bd.offset);
  if (b->grid_update) {
    // the next replay dispatches exactly each segment's tiles (one workgroup when it has none:
    // the kernel's own bound check ends it); replays already launched keep their grids
    void* args[4] = {(void*)&b->arg_desc, (void*)&b->arg_work, (void*)&b->arg_bdev, (void*)&b->arg_ms};
    for (int g = 0; g < kSegs; ++g) {
      hipKernelNodeParams kp{};
      kp.func = const_cast<void*>(b->seg_fn[g]);
      kp.gridDim = dim3((unsigned)std::max(1, bd.n_items[g]));
      kp.blockDim = dim3(kTile);
      kp.sharedMemBytes = 0;
      kp.kernelParams = args;
      kp.extra = nullptr;
      const hipError_t e = hipGraphExecKernelNodeSetParams(b->exec, b->seg_node[g], &kp);
      if (e != hipSuccess) {  // grids of mixed sizes: nothing may run until a staging succeeds
        b->staged = false;
        return fail(SFHK_E_DEVICE, std::string("hipGraphExecKernelNodeSetParams: ") + hipGetErrorString(e));
      }
    }
  }
  for (int i = 0; i < n_jobs; ++i) b->desc_host[s][i] = jobs[i]->host;
  for (size_t k = 0; k < items.size(); ++k) b->work_host[s][k] = {items[k].job, items[k].tile};
  *b->bdev_host[s] = bd;
  if (n_jobs) HIP_TRY(hipMemcpyAsync(b->desc, b->desc_host[s], n_jobs * sizeof(JobDev), hipMemcpyHostToDevice, st));
  if (!items.empty())
    HIP_TRY(hipMemcpyAsync(b->work, b->work_host[s], items.size() * sizeof(WorkItem), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(b->bdev, b->bdev_host[s], sizeof(BatchDev), hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(b->done[s], st));
  b->done_recorded[s] = true;
  b->cur = s;
  b->jobs.assign(jobs, jobs + n_jobs);
  b->staged = true;
  return SFHK_OK;
}

sfhk_status sfhk_batch_run(sfhk_batch* b, void* stream) {
  TraceRange trace_("sfhk_batch_run");
  if (!b) return fail(SFHK_E_INVALID, "batch is NULL");
  if (!b->staged)
    return fail(SFHK_E_INVALID, "no job table is staged (sfhk_batch_set_jobs has not been called, "
                                "or its last call failed)");
  if (b->jobs.empty()) return SFHK_OK;
  HIP_TRY(hipSetDevice(b->ctx->device));
  HIP_TRY(hipGraphLaunch(b->exec, (hipStream_t)stream));
  for (sfhk_job* j : b->jobs) HIP_TRY(hipEventRecord(j->last_use, (hipStream_t)stream));
  // the latest staging set is refilled only after this replay: at most one replay ahead
  HIP_TRY(hipEventRecord(b->done[b->cur], (hipStream_t)stream));
  sfhk_status agg = SFHK_OK;
  for (sfhk_job* j : b->jobs) {
    if (j->done) continue;
    const int NS = j->host.n_steps;
    j->steps_done += (b->max_steps <= 0) ? (long long)NS + 1 : b->max_steps;
    if (unfinished_tiles(j, j->steps_done) == 0)
      j->done = true;
    else
      agg = SFHK_E_NOT_DONE;
  }
  return agg;
}

int32_t sfhk_batch_workers(const sfhk_batch* b) { return b ? b->n_workers : 0; }

int32_t sfhk_job_is_done(const sfhk_job* job) { return job && job->done ? 1 : 0; }

// the dipole (or the dipole velocity) from the job's exact per-step accumulators
static sfhk_status reduce_rows(sfhk_job* job, bool velocity, double* d_out, double* f_out, void* stream) {
  if (!job || !d_out) return fail(SFHK_E_INVALID, "NULL argument");
  if (!job->done) return fail(SFHK_E_NOT_DONE, "job is not finished");
  if (velocity && !job->host.acc_v) return fail(SFHK_E_INVALID, "job was created without velocity");
  HIP_TRY(hipSetDevice(job->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const JobDev& H = job->host;
  double* d_step = job->n_out > 0 ? job->dbuf : d_out;
  hipLaunchKernelGGL(k_acc_final, dim3(blocks_for(H.n_steps + 1, 256)), dim3(256), 0, st,
                     (const long long*)(velocity ? H.acc_v : H.acc), H.n_steps, d_step, f_out);
  HIP_TRY(hipGetLastError());
  if (job->n_out > 0) {
    hipLaunchKernelGGL(k_resample, dim3(blocks_for(job->n_out, 256)), dim3(256), 0, st,
                       (const double*)job->dbuf, (long long)H.n_steps, (long long)job->n_out, d_out);
    HIP_TRY(hipGetLastError());
  }
  return mark_use(job, st);
}

sfhk_status sfhk_dipole(sfhk_job* job, double* d_out, double* f_out, void* stream) {
  TraceRange trace_("sfhk_dipole");
  return reduce_rows(job, false, d_out, f_out, stream);
}

sfhk_status sfhk_velocity(sfhk_job* job, double* v_out, double* vf_out, void* stream) {
  TraceRange trace_("sfhk_velocity");
  return reduce_rows(job, true, v_out, vf_out, stream);
}

}  // extern "C"

namespace {

// The spectrum's working memory for n samples zero-padded to n_fft: windowed samples xw[n_fft],
// twiddles tw[n_fft], and one row of partial sums per span of samples, part[n_spans][n_fft/2+1].
// Spans are whole chunks of kDftChunk samples, at most kDftMaxSpans of them.
using sfhk_host::SpectrumPlan;
static_assert(sizeof(double2) == 2 * sizeof(double), "complex layout of the workspace");

SpectrumPlan spectrum_plan(long long n, long long n_fft) {
  return sfhk_host::spectrum_plan(n, n_fft, kDftChunk, kDftMaxSpans);
}

sfhk_status spectrum_check(const double* d, int64_t n, int64_t n_fft, double dt, double tau_h) {
  if (!d || n < 1 || n_fft < n || n_fft > (1LL << 31) || !(dt > 0.0) || !(tau_h > 0.0))
    return fail(SFHK_E_INVALID, "spectrum: need d, 1 <= n <= n_fft <= 2^31, dt > 0, tau_h > 0");
  return SFHK_OK;
}

// the window, the partial transforms and their fixed-order sum, in the workspace `ws`
sfhk_status spectrum_launch(const double* d, long long n, double t_first, double dt, double tau_h,
                            long long n_fft, double* omega_out, double* power_out, double* x_out,
                            hipStream_t st, const SpectrumPlan& P, char* ws) {
  double* xw = (double*)(ws + P.xw_off);
  double2* tw = (double2*)(ws + P.tw_off);
  double2* part = (double2*)(ws + P.part_off);
  hipLaunchKernelGGL(k_window, dim3(blocks_for(n_fft, 256)), dim3(256), 0, st, d, n, n_fft,
                     t_first, dt, tau_h, xw, tw);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_dft_partial, dim3(blocks_for(P.nk, 256), P.n_spans), dim3(256), 0, st,
                     (const double*)xw, (const double2*)tw, n, n_fft, P.span, part);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_dft_final, dim3(blocks_for(P.nk, 256)), dim3(256), 0, st,
                     (const double2*)part, P.n_spans, n_fft, t_first, dt, omega_out, power_out,
                     x_out);
  HIP_TRY(hipGetLastError());
  return SFHK_OK;
}

// Working memory of sfhk_spectrum_noalloc: one copy per GPU, held until the process ends. In host
// code `scratch` only names the symbol; its device address on each GPU comes from
// hipGetSymbolAddress (scratch_ptr below), and only that address is passed to kernels.
constexpr size_t kNoAllocBytes = SFHK_SPECTRUM_NOALLOC_BYTES;
static __device__ __align__(256) char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
std::vector<char*> g_scratch_ptr;  // per device, nullptr until looked up

// the current device's address of `scratch` (looked up once per device, with it current)
sfhk_status scratch_ptr(char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SFHK_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return SFHK_OK;
}

}  // namespace

static_assert(SFHK_SPECTRUM_NOALLOC_MAX_FFT % 2 == 0, "max n_fft");

extern "C" {

sfhk_status sfhk_spectrum(const double* d, int64_t n, double t_first, double dt, double tau_h,
                          int64_t n_fft, double* omega_out, double* power_out, double* x_out,
                          void* stream) {
  TraceRange trace_("sfhk_spectrum");
  if (n_fft == 0) n_fft = n;
  sfhk_status rc = spectrum_check(d, n, n_fft, dt, tau_h);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const SpectrumPlan P = spectrum_plan(n, n_fft);
  char* ws = nullptr;
  HIP_TRY(hipMallocAsync((void**)&ws, P.bytes, st));
  rc = spectrum_launch(d, n, t_first, dt, tau_h, n_fft, omega_out, power_out, x_out, st, P, ws);
  hipError_t fe = hipFreeAsync(ws, st);
  if (rc) return rc;
  HIP_TRY(fe);
  return SFHK_OK;
}

sfhk_status sfhk_spectrum_noalloc(const double* d, int64_t n, double t_first, double dt,
                                  double tau_h, int64_t n_fft, double* omega_out,
                                  double* power_out, double* x_out, void* stream) {
  TraceRange trace_("sfhk_spectrum_noalloc");
  if (n_fft == 0) n_fft = n;
  sfhk_status rc = spectrum_check(d, n, n_fft, dt, tau_h);
  if (rc) return rc;
  if (n_fft > SFHK_SPECTRUM_NOALLOC_MAX_FFT)
    return fail(SFHK_E_INVALID, "spectrum_noalloc: n_fft above SFHK_SPECTRUM_NOALLOC_MAX_FFT");
  const SpectrumPlan P = spectrum_plan(n, n_fft);
  if (P.bytes > kNoAllocBytes)  // cannot happen for n <= n_fft <= the maximum; kept as a guard
    return fail(SFHK_E_INVALID, "spectrum_noalloc: working memory above its fixed size");
  char* ws = nullptr;
  if ((rc = scratch_ptr(&ws))) return rc;
  return spectrum_launch(d, n, t_first, dt, tau_h, n_fft, omega_out, power_out, x_out,
                         (hipStream_t)stream, P, ws);
}

sfhk_status sfhk_job_stats(sfhk_job* job, sfhk_stats* out, void* stream) {
  if (!job || !out) return fail(SFHK_E_INVALID, "NULL argument");
  HIP_TRY(hipSetDevice(job->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  unsigned long long c[8] = {0};
  HIP_TRY(hipMemcpyAsync(c, job->host.counters, sizeof(c), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  out->n_traj = job->n_traj;
  out->n_steps = job->host.n_steps;
  out->steps_evaluated = (int64_t)c[0];
  out->kay_removed = (int64_t)c[1];
  out->nonfinite_removed = (int64_t)c[2];
  out->steps_fp64 = (int64_t)c[3];
  out->prims_evaluated = (int64_t)c[4];
  out->integrands_evaluated = (int64_t)c[5];
  out->reserved = 0;
  out->tiles_total = job->host.n_tiles;
  out->tiles_done = job->host.n_tiles - unfinished_tiles(job, job->steps_done);
  return SFHK_OK;
}

sfhk_status sfhk_job_trajectories(sfhk_job* job, double* y_out, double* c_out, int64_t* death_out,
                                  void* stream) {
  if (!job) return fail(SFHK_E_INVALID, "job is NULL");
  HIP_TRY(hipSetDevice(job->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_scatter_traj, dim3(blocks_for(job->host.n_pad, 256)), dim3(256), 0, st,
                     job->host, (const long long*)job->perm, (long long)job->n_traj, y_out, c_out,
                     (long long*)death_out);
  HIP_TRY(hipGetLastError());
  return mark_use(job, st);
}

// ------------------------------------------------------------------------------------------------
// checkpoint / restore of a job's propagation state
// ------------------------------------------------------------------------------------------------

int64_t sfhk_job_checkpoint_bytes(const sfhk_job* job) {
  return job ? (int64_t)ckpt_bytes(const_cast<sfhk_job*>(job)) : 0;
}

sfhk_status sfhk_job_checkpoint(sfhk_job* job, void* dst, void* stream) {
  if (!job || !dst) return fail(SFHK_E_INVALID, "NULL argument");
  HIP_TRY(hipSetDevice(job->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const CkptHeader h = ckpt_header(job);
  char* out = (char*)dst;
  HIP_TRY(hipMemcpyAsync(out, &h, sizeof(h), hipMemcpyHostToDevice, st));
  std::vector<std::pair<void*, size_t>> secs;
  std::vector<size_t> off;
  ckpt_offsets(job, secs, off);
  for (size_t i = 0; i < secs.size(); ++i)
    HIP_TRY(hipMemcpyAsync(out + off[i], secs[i].first, secs[i].second, hipMemcpyDeviceToDevice, st));
  sfhk_status rc = mark_use(job, st);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(st));  // the header above lives on this call's stack
  return SFHK_OK;
}

sfhk_status sfhk_job_restore(sfhk_job* job, const void* src, void* stream) {
  if (!job || !src) return fail(SFHK_E_INVALID, "NULL argument");
  if (job->steps_done != 0) return fail(SFHK_E_INVALID, "restore needs a job that has not been propagated");
  HIP_TRY(hipSetDevice(job->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  CkptHeader h{};
  const char* in = (const char*)src;
  HIP_TRY(hipMemcpyAsync(&h, in, sizeof(h), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (!sfhk_host::ckpt_matches(h, ckpt_header(job)))
    return fail(SFHK_E_INVALID, "checkpoint does not match this job (other inputs or not a checkpoint)");
  std::vector<std::pair<void*, size_t>> secs;
  std::vector<size_t> off;
  ckpt_offsets(job, secs, off);
  for (size_t i = 0; i < secs.size(); ++i)
    HIP_TRY(hipMemcpyAsync(secs[i].first, in + off[i], secs[i].second, hipMemcpyDeviceToDevice, st));
  sfhk_status rc = mark_use(job, st);
  if (rc) return rc;
  job->steps_done = h.steps_done;
  job->done = h.done != 0;
  return SFHK_OK;
}

static sfhk_status traj_fn(int which, const double* x, double* y, int64_t n, void* stream) {
  if (!x || !y || n < 0 || n > INT32_MAX) return fail(SFHK_E_INVALID, "NULL pointer or bad count");
  if (n == 0) return SFHK_OK;
  hipLaunchKernelGGL(k_traj_fn, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, which, x,
                     y, (long long)n);
  HIP_TRY(hipGetLastError());
  return SFHK_OK;
}

sfhk_status sfhk_traj_exp(const double* x, double* y, int64_t n, void* stream) {
  return traj_fn(0, x, y, n, stream);
}

sfhk_status sfhk_traj_rsqrt(const double* x, double* y, int64_t n, void* stream) {
  return traj_fn(1, x, y, n, stream);
}

sfhk_status sfhk_gabor(const double* d, int64_t n, double t_first, double dt, double sigma,
                       double tc_first, double tc_step, int64_t n_c, double w_step, int64_t n_w,
                       double* power_out, double* g_out, void* stream) {
  TraceRange trace_("sfhk_gabor");
  if (n < 0 || n_c < 0 || n_w < 0) return fail(SFHK_E_INVALID, "negative count");
  if (!(dt > 0.0) || !(sigma > 0.0) || !std::isfinite(dt) || !std::isfinite(sigma) ||
      !std::isfinite(t_first) || !std::isfinite(tc_first) || !std::isfinite(tc_step) ||
      !std::isfinite(w_step))
    return fail(SFHK_E_INVALID, "dt and sigma must be finite and > 0, the grids finite");
  if (n_c > 65535) return fail(SFHK_E_INVALID, "at most 65535 centre times per call");
  if (n_w > INT32_MAX || n_c * n_w > INT32_MAX) return fail(SFHK_E_INVALID, "output grid too large");
  if (n_c == 0 || n_w == 0) return SFHK_OK;
  if (!power_out || (n > 0 && !d)) return fail(SFHK_E_INVALID, "NULL array");
  dim3 grid((unsigned)((n_w + kGaborFreqPerBlock - 1) / kGaborFreqPerBlock), (unsigned)n_c);
  hipLaunchKernelGGL(k_gabor, grid, dim3(kGaborThreads), 0, (hipStream_t)stream, d, (long long)n, t_first,
                     dt, sigma, tc_first, tc_step, w_step, (long long)n_w, power_out, (double2*)g_out);
  HIP_TRY(hipGetLastError());
  return SFHK_OK;
}

sfhk_status sfhk_traj_sincos(const double* x, double* s, double* c, int64_t n, void* stream) {
  if (!x || !s || !c || n < 0 || n > INT32_MAX) return fail(SFHK_E_INVALID, "NULL pointer or bad count");
  if (n == 0) return SFHK_OK;
  hipLaunchKernelGGL(k_traj_sincos, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, x, s,
                     c, (long long)n);
  HIP_TRY(hipGetLastError());
  return SFHK_OK;
}

sfhk_status sfhk_sfa_birth(const sfhk_pulse* pulse, const sfhk_ground* gs, int32_t mode, int64_t n,
                           const double* t0, const double* kperp, const double* u, double* q0,
                           double* p0, double* w, double* t_tun, void* stream) {
  TraceRange trace_("sfhk_sfa_birth");
  if (!pulse || !gs) return fail(SFHK_E_INVALID, "NULL pulse or ground state");
  if (!(pulse->e0 > 0.0) || !(pulse->omega > 0.0) || !(pulse->n_cycles > 1.0) ||
      !std::isfinite(pulse->e0) || !std::isfinite(pulse->omega) || !std::isfinite(pulse->n_cycles) ||
      !std::isfinite(pulse->cep))
    return fail(SFHK_E_INVALID, "pulse needs finite e0 > 0, omega > 0, n_cycles > 1 and cep");
  if (!(gs->ip > 0.0) || !std::isfinite(gs->ip)) return fail(SFHK_E_INVALID, "ip must be finite and > 0");
  if (gs->l != 0 && gs->l != 1) return fail(SFHK_E_INVALID, "ground state l must be 0 or 1");
  if (mode != SFHK_BIRTH_GTO && mode != SFHK_BIRTH_MODIFIED) return fail(SFHK_E_INVALID, "unknown birth mode");
  if (mode == SFHK_BIRTH_GTO && (gs->n_prim < 1 || gs->n_prim > SFHK_MAX_PRIM || !gs->alpha || !gs->coef))
    return fail(SFHK_E_INVALID, "ground state needs 1..SFHK_MAX_PRIM primitives");
  if (n < 0 || n > INT32_MAX) return fail(SFHK_E_INVALID, "n must be in [0, 2^31)");
  if (n == 0) return SFHK_OK;
  if (!t0 || !kperp || !q0 || !p0 || !w) return fail(SFHK_E_INVALID, "NULL sample or output array");
  SfaParams P{};
  P.e0 = pulse->e0;
  P.omega = pulse->omega;
  P.n_cycles = pulse->n_cycles;
  P.cep = pulse->cep;
  P.ip = gs->ip;
  P.mode = mode;
  P.l = gs->l;
  P.n_prim = mode == SFHK_BIRTH_GTO ? gs->n_prim : 0;
  for (int i = 0; i < P.n_prim; ++i) {
    if (!(gs->alpha[i] > 0.0)) return fail(SFHK_E_INVALID, "GTO exponents must be > 0");
    P.alpha[i] = gs->alpha[i];
    P.coef[i] = gs->coef[i];
    P.cnorm[i] = gs->coef[i] * std::pow(gs->alpha[i], gs->l == 0 ? -2.5 : -3.5);
  }
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_sfa_saddle, dim3(blocks_for(n, 256)), dim3(256), 0, st, P, (long long)n, t0, kperp,
                     q0, p0, w, t_tun);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_sfa_weight, dim3(blocks_for(n, 256)), dim3(256), 0, st, P, (long long)n, t0, kperp, u,
                     q0, p0, w, t_tun);
  HIP_TRY(hipGetLastError());
  return SFHK_OK;
}

}  // extern "C"
