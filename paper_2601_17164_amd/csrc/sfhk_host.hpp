// sfhk_host.hpp -- the host runtime's pure logic, free of HIP so that it also builds with a plain
// C++ compiler (and runs under the address and undefined-behaviour sanitizers in the test suite):
// the birth-step order of a job's samples and its tiles, the longest-first work list over the
// unfinished tiles of several jobs with its per-kernel segments, the checkpoint layout and header
// check, the spectrum's work plan, and the duplicate-handle test.
#pragma once
#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace sfhk_host {

// ------------------------------------------------------------------------------------------------
// birth order
// ------------------------------------------------------------------------------------------------
// Stable order of n samples by birth step (each in 0..n_steps): perm[s] = the sample in slot s
// (slots n..n_pad-1: -1), n0s[s] = its birth step (n_steps + 1 on padding). A counting sort over
// the grid steps: O(n + n_steps). Returns false (outputs untouched) if a birth step is out of range.
inline bool birth_sort(const int* n0, long long n, int n_steps, long long n_pad,
                       std::vector<long long>& perm, std::vector<int>& n0s) {
  if (n < 0 || n_pad < n || n_steps < 0) return false;
  for (long long i = 0; i < n; ++i)
    if (n0[i] < 0 || n0[i] > n_steps) return false;
  std::vector<long long> next((size_t)n_steps + 2, 0);
  for (long long i = 0; i < n; ++i) ++next[(size_t)n0[i] + 1];
  for (int k = 0; k <= n_steps; ++k) next[(size_t)k + 1] += next[(size_t)k];
  perm.assign((size_t)n_pad, -1);
  for (long long i = 0; i < n; ++i) perm[(size_t)next[(size_t)n0[i]]++] = i;
  n0s.assign((size_t)n_pad, n_steps + 1);
  for (long long s = 0; s < n; ++s) n0s[(size_t)s] = n0[perm[(size_t)s]];
  return true;
}

// each tile's first birth step (the birth step of its first slot); tiles of `tile` slots
inline void tile_first_steps(const std::vector<int>& n0s, int tile, std::vector<int>& tile_n0) {
  const size_t nt = n0s.size() / (size_t)tile;
  tile_n0.resize(nt);
  for (size_t t = 0; t < nt; ++t) tile_n0[t] = n0s[t * (size_t)tile];
}

// a fresh job's per-tile progress: the next step to propagate and the last step propagated
inline void tile_progress(const std::vector<int>& tile_n0, std::vector<int>& next,
                          std::vector<int>& last) {
  next.assign(tile_n0.begin(), tile_n0.end());
  last.resize(tile_n0.size());
  for (size_t t = 0; t < tile_n0.size(); ++t) last[t] = tile_n0[t] - 1;
}

// Tiles that still have steps left after `done` steps have been requested. Tiles are in birth
// order (first birth steps non-decreasing), so they are a prefix: tile t is finished once
// tile_n0[t] + done > n_steps.
inline int unfinished_tiles(const std::vector<int>& tile_n0, int n_steps, long long done) {
  int lo = 0, hi = (int)tile_n0.size();
  while (lo < hi) {
    const int mid = lo + (hi - lo) / 2;
    if ((long long)tile_n0[(size_t)mid] + done <= n_steps) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// ------------------------------------------------------------------------------------------------
// work list of several jobs
// ------------------------------------------------------------------------------------------------
struct JobProgress {
  const std::vector<int>* tile_n0;  // the job's tiles' first birth steps (birth order)
  int n_steps;
  long long steps_done;
  bool done;
  int seg;  // the kernel segment that runs the job (precision and potential kind)
};

struct Item {
  long long left;  // steps the tile still has
  int job, tile, seg;
};

// Every unfinished tile of every job that is not done, grouped by segment (ascending) and, inside
// a segment, longest first; ties keep job order, then tile order (stable).
inline std::vector<Item> work_items(const std::vector<JobProgress>& jobs) {
  std::vector<Item> items;
  for (size_t i = 0; i < jobs.size(); ++i) {
    const JobProgress& j = jobs[i];
    if (j.done) continue;
    const int nt = unfinished_tiles(*j.tile_n0, j.n_steps, j.steps_done);
    for (int t = 0; t < nt; ++t)
      items.push_back({(long long)j.n_steps + 1 - ((long long)(*j.tile_n0)[(size_t)t] + j.steps_done),
                       (int)i, t, j.seg});
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) {
    return a.seg != b.seg ? a.seg < b.seg : a.left > b.left;
  });
  return items;
}

// items per segment and the first item of each segment (n_segs entries each)
inline void segment_table(const std::vector<Item>& items, int n_segs, int* n_items, int* offset) {
  for (int g = 0; g < n_segs; ++g) n_items[g] = 0;
  for (const Item& it : items)
    if (it.seg >= 0 && it.seg < n_segs) n_items[it.seg]++;
  offset[0] = 0;
  for (int g = 1; g < n_segs; ++g) offset[g] = offset[g - 1] + n_items[g - 1];
}

// a handle listed twice would have its tiles queued twice
inline bool has_duplicates(const void* const* p, int n) {
  if (n < 2) return false;
  std::vector<const void*> v(p, p + n);
  std::sort(v.begin(), v.end());
  return std::adjacent_find(v.begin(), v.end()) != v.end();
}

// ------------------------------------------------------------------------------------------------
// checkpoints
// ------------------------------------------------------------------------------------------------
constexpr uint64_t kCkptMagic = 0x54504b434b484653ull;  // "SFHKCKPT"
constexpr size_t kCkptAlign = 256;

struct CkptHeader {
  uint64_t magic;
  int64_t n_traj, n_pad, n_tiles, n_steps, acc_words, steps_done;
  int32_t kind, precision, done, reserved;
  uint64_t fingerprint;  // of the job's potential, ground state, grid and method parameters
};
static_assert(sizeof(CkptHeader) <= kCkptAlign, "checkpoint header");

inline size_t ckpt_round(size_t b) { return (b + kCkptAlign - 1) / kCkptAlign * kCkptAlign; }

// byte offset of every section after the header (in order) and the total size
inline size_t ckpt_layout(const std::vector<size_t>& section_bytes, std::vector<size_t>& offsets) {
  offsets.resize(section_bytes.size());
  size_t off = kCkptAlign;
  for (size_t i = 0; i < section_bytes.size(); ++i) {
    offsets[i] = off;
    off += ckpt_round(section_bytes[i]);
  }
  return off;
}

// a checkpoint restores into a job only if it was taken of a job made from the same inputs
inline bool ckpt_matches(const CkptHeader& h, const CkptHeader& job) {
  return h.magic == kCkptMagic && h.n_traj == job.n_traj && h.n_pad == job.n_pad &&
         h.n_tiles == job.n_tiles && h.n_steps == job.n_steps && h.acc_words == job.acc_words &&
         h.kind == job.kind && h.precision == job.precision && h.fingerprint == job.fingerprint &&
         h.steps_done >= 0 && (h.done == 0 || h.done == 1);
}

// ------------------------------------------------------------------------------------------------
// spectrum work plan
// ------------------------------------------------------------------------------------------------
// n samples zero-padded to n_fft: nk = n_fft/2 + 1 frequencies; the samples in at most max_spans
// spans of whole chunks of `chunk` samples; one workspace holding the windowed samples
// (n_fft doubles), the twiddles (n_fft complex doubles) and the per-span partial sums
// (n_spans x nk complex doubles), each part 256-byte aligned.
struct SpectrumPlan {
  long long nk, span;
  int n_spans;
  size_t xw_off, tw_off, part_off, bytes;
};

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

inline SpectrumPlan spectrum_plan(long long n, long long n_fft, int chunk, int max_spans) {
  SpectrumPlan P{};
  P.nk = n_fft / 2 + 1;
  const long long chunks = (n + chunk - 1) / chunk;
  const long long per = (chunks + max_spans - 1) / max_spans;
  P.span = per * chunk;
  P.n_spans = (int)((n + P.span - 1) / P.span);
  P.xw_off = 0;
  P.tw_off = align256((size_t)n_fft * sizeof(double));
  P.part_off = P.tw_off + align256((size_t)n_fft * 2 * sizeof(double));
  P.bytes = P.part_off + align256((size_t)P.n_spans * (size_t)P.nk * 2 * sizeof(double));
  return P;
}

}  // namespace sfhk_host
