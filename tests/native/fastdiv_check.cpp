// Check of the division by invariant integers used for tile positions (FastDiv in lbm_device.hpp):
// fast_div(n, make_fast_div(d)) == n / d for every divisor up to 70 000, for powers of two and their
// neighbours, for random divisors up to 2^32 - 1, each against numerators at and around multiples of
// the divisor, random ones and the extremes.  Prints the number of checks; exit status 1 on a
// mismatch.
#include <cstdio>
#include <random>

#include "lbm_device.hpp"

int main() {
  std::mt19937_64 rng(7);
  unsigned long long checks = 0, bad = 0;
  auto check_d = [&](unsigned d) {
    const lbm::FastDiv f = lbm::make_fast_div(d);
    auto one = [&](unsigned n) {
      ++checks;
      if (lbm::fast_div(n, f) != n / d) {
        if (bad < 10) std::fprintf(stderr, "mismatch: %u / %u\n", n, d);
        ++bad;
      }
    };
    for (unsigned n : {0u, 1u, 2u, d - 1, d, d + 1, 0x7fffffffu, 0x80000000u, 0xfffffffeu, 0xffffffffu}) one(n);
    for (unsigned long long k = 2; k < 40; ++k) {
      const unsigned long long m = k * d;
      if (m > 0xffffffffull) break;
      one((unsigned)m);
      one((unsigned)(m - 1));
      if (m < 0xffffffffull) one((unsigned)(m + 1));
    }
    const unsigned long long top = 0xffffffffull / d * d;  // the largest multiple
    one((unsigned)top);
    if (top > 0) one((unsigned)(top - 1));
    for (int r = 0; r < 8; ++r) one((unsigned)rng());
  };
  for (unsigned d = 1; d <= 70000; ++d) check_d(d);
  for (int b = 1; b < 32; ++b) {
    const unsigned p = 1u << b;
    check_d(p - 1);
    check_d(p);
    check_d(p + 1);
  }
  check_d(0xffffffffu);
  for (int r = 0; r < 20000; ++r) {
    const unsigned d = (unsigned)rng();
    if (d) check_d(d);
  }
  std::printf("checks %llu mismatches %llu\n", checks, bad);
  return bad ? 1 : 0;
}
