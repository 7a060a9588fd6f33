// Host driver for the exact per-step accumulator (sfhk_exact_sum.hpp): reads groups of binary64
// values (as 16-digit hex bit patterns) from stdin, one group per line, accumulates each group in
// its own accumulator and prints the rounded total's bits, one line per group.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "../../paper_2601_17164_amd/csrc/sfhk_exact_sum.hpp"

int main() {
  std::string line;
  while (std::getline(std::cin, line)) {
    std::istringstream in(line);
    std::vector<int64_t> acc(sfhk_exact::kExactWords, 0);
    std::string tok;
    while (in >> tok) {
      uint64_t u = std::stoull(tok, nullptr, 16);
      double v;
      std::memcpy(&v, &u, sizeof v);
      sfhk_exact::add_host(acc.data(), v);
    }
    double r = sfhk_exact::round_total(acc.data());
    uint64_t u;
    std::memcpy(&u, &r, sizeof u);
    std::printf("%016llx\n", (unsigned long long)u);
  }
  return 0;
}
