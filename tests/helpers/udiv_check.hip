// Host-side check of the library's division by a 64-bit reciprocal
// (udiv_magic): compares it with the plain quotient on edge and random cases.
// Prints "tests <n> bad <m>" and exits nonzero on any mismatch.
#include <cstdio>
#include <random>

#include "../../paper_2110_15425_amd/csrc/internal.hpp"

int main() {
  std::mt19937_64 g(1);
  unsigned long long bad = 0, n_tests = 0;
  auto chk = [&](uint32_t n, uint32_t d) {
    ++n_tests;
    if (cm::udiv_magic(n, cm::udiv_magic_for(d)) != n / d && bad++ < 5) printf("bad %u / %u\n", n, d);
  };
  const uint32_t ds[] = {1, 2, 3, 7, 9, 100, 1000, 3000, 10000, 65536, 65537,
                         1u << 31, (1u << 31) + 1, 0xFFFFFFFEu, 0xFFFFFFFFu};
  for (uint32_t d : ds) {
    for (uint32_t k = 0; k < 20000; ++k) {
      chk(k, d);
      chk(0xFFFFFFFFu - k, d);
    }
    for (uint64_t m = 1; m < 20000 && m * d < (1ull << 32); ++m) {
      chk((uint32_t)(m * d), d);  // exact multiples and their predecessors
      chk((uint32_t)(m * d - 1), d);
    }
    for (int k = 0; k < 100000; ++k) chk((uint32_t)g(), d);
  }
  for (int k = 0; k < 2000000; ++k) {
    uint32_t d = (uint32_t)g() >> (g() % 32);
    chk((uint32_t)g() >> (g() % 32), d ? d : 1u);
  }
  printf("tests %llu bad %llu\n", n_tests, bad);
  return bad != 0;
}
