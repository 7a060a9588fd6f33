// Host driver for the runtime's pure logic (paper_2601_17164_amd/csrc/sfhk_host.hpp), built with
// g++ under AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_host_logic.py. Reads
// commands from stdin, one per line, and prints one result line per command:
//   sort N NS NPAD TILE n0_0 .. n0_{N-1}
//       -> "ok" perm[0..NPAD) "|" n0s[0..NPAD) "|" tile_n0 "|" tile_next "|" tile_last, or "bad"
//   unfinished NS DONE NT tile_n0_0 ..      -> count
//   work NJOBS NSEGS, then per job: NS DONE_STEPS DONE SEG NT tile_n0_0 ..
//       -> "items" (left job tile seg)... "|" n_items... "|" offsets...
//   dup N v_0 .. v_{N-1}                    -> 0 or 1 (the values stand for handles)
//   ckpt NSEC bytes_0 .. | header fields (a) | header fields (b)
//       -> offsets... total "|" match(a as checkpoint, b as job)
//   plan N NFFT CHUNK MAXSPANS              -> nk span n_spans xw_off tw_off part_off bytes
#include <cstdint>
#include <cstdio>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "../../paper_2601_17164_amd/csrc/sfhk_host.hpp"

using namespace sfhk_host;

static void print_vec(const std::vector<long long>& v) {
  for (long long x : v) std::printf(" %lld", x);
}
static void print_vec(const std::vector<int>& v) {
  for (int x : v) std::printf(" %d", x);
}

static CkptHeader read_header(std::istringstream& in) {
  CkptHeader h{};
  long long m;
  in >> m >> h.n_traj >> h.n_pad >> h.n_tiles >> h.n_steps >> h.acc_words >> h.steps_done >> h.kind >>
      h.precision >> h.done >> h.fingerprint;
  h.magic = m ? kCkptMagic : 0;
  return h;
}

int main() {
  std::string line;
  while (std::getline(std::cin, line)) {
    std::istringstream in(line);
    std::string cmd;
    in >> cmd;
    if (cmd == "sort") {
      long long n, npad;
      int ns, tile;
      in >> n >> ns >> npad >> tile;
      std::vector<int> n0((size_t)n);
      for (auto& x : n0) in >> x;
      std::vector<long long> perm;
      std::vector<int> n0s, tn0, next, last;
      if (!birth_sort(n0.data(), n, ns, npad, perm, n0s)) {
        std::printf("bad\n");
        continue;
      }
      tile_first_steps(n0s, tile, tn0);
      tile_progress(tn0, next, last);
      std::printf("ok");
      print_vec(perm);
      std::printf(" |");
      print_vec(n0s);
      std::printf(" |");
      print_vec(tn0);
      std::printf(" |");
      print_vec(next);
      std::printf(" |");
      print_vec(last);
      std::printf("\n");
    } else if (cmd == "unfinished") {
      int ns, nt;
      long long done;
      in >> ns >> done >> nt;
      std::vector<int> tn0((size_t)nt);
      for (auto& x : tn0) in >> x;
      std::printf("%d\n", unfinished_tiles(tn0, ns, done));
    } else if (cmd == "work") {
      int nj, nsegs;
      in >> nj >> nsegs;
      std::vector<std::vector<int>> tiles((size_t)nj);
      std::vector<JobProgress> jobs((size_t)nj);
      for (int i = 0; i < nj; ++i) {
        int ns, done, seg, nt;
        long long steps_done;
        in >> ns >> steps_done >> done >> seg >> nt;
        tiles[(size_t)i].resize((size_t)nt);
        for (auto& x : tiles[(size_t)i]) in >> x;
        jobs[(size_t)i] = {&tiles[(size_t)i], ns, steps_done, done != 0, seg};
      }
      const std::vector<Item> items = work_items(jobs);
      std::vector<int> n_items((size_t)nsegs), offset((size_t)nsegs);
      segment_table(items, nsegs, n_items.data(), offset.data());
      std::printf("items");
      for (const Item& it : items) std::printf(" %lld %d %d %d", it.left, it.job, it.tile, it.seg);
      std::printf(" |");
      print_vec(n_items);
      std::printf(" |");
      print_vec(offset);
      std::printf("\n");
    } else if (cmd == "dup") {
      int n;
      in >> n;
      std::vector<uintptr_t> v((size_t)n);
      for (auto& x : v) in >> x;
      std::vector<const void*> p((size_t)n);
      for (int i = 0; i < n; ++i) p[(size_t)i] = (const void*)(v[(size_t)i] * 64);
      std::printf("%d\n", has_duplicates(p.data(), n) ? 1 : 0);
    } else if (cmd == "ckpt") {
      int nsec;
      in >> nsec;
      std::vector<size_t> bytes((size_t)nsec);
      for (auto& b : bytes) in >> b;
      std::string bar;
      in >> bar;
      const CkptHeader a = read_header(in);
      in >> bar;
      const CkptHeader b = read_header(in);
      std::vector<size_t> off;
      const size_t total = ckpt_layout(bytes, off);
      for (size_t o : off) std::printf("%zu ", o);
      std::printf("%zu | %d\n", total, ckpt_matches(a, b) ? 1 : 0);
    } else if (cmd == "plan") {
      long long n, nfft;
      int chunk, maxspans;
      in >> n >> nfft >> chunk >> maxspans;
      const SpectrumPlan P = spectrum_plan(n, nfft, chunk, maxspans);
      std::printf("%lld %lld %d %zu %zu %zu %zu\n", P.nk, P.span, P.n_spans, P.xw_off, P.tw_off,
                  P.part_off, P.bytes);
    } else if (!cmd.empty()) {
      std::printf("unknown\n");
    }
    std::fflush(stdout);
  }
  return 0;
}
