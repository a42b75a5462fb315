// Host check of the invariant-divisor quotient used for the sweep tile
// order: udiv(n, make_udiv(d)) == n / d for divisors 1 .. 4096 and large
// ones, at edge dividends, random dividends and a dense sweep of the 32-bit
// range for a few divisors.  Prints the number of mismatches; exit status 1
// if any.
#include "hlbm_internal.h"

#include <cstdio>
#include <cstdint>

using hlbm::make_udiv;
using hlbm::udiv;

int main() {
  uint64_t state = 0x9e3779b97f4a7c15ull;
  auto next = [&]() {  // xorshift64
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return uint32_t(state >> 16);
  };
  long checked = 0, bad = 0;
  auto check = [&](uint32_t d, uint32_t n) {
    ++checked;
    if (udiv(n, make_udiv(d)) != n / d && bad++ < 5) printf("mismatch d=%u n=%u\n", d, n);
  };
  for (uint32_t d = 1; d <= 4096; ++d) {
    const uint32_t edges[] = {0u, 1u, d - 1, d, d + 1, 2 * d - 1, 2 * d, 0x7fffffffu, 0x80000000u, 0xfffffffeu, 0xffffffffu};
    for (uint32_t n : edges) check(d, n);
    for (int k = 0; k < 200; ++k) {
      const uint32_t n = next();
      check(d, n);
      const uint32_t q = n / d * d;  // multiples and their predecessors
      check(d, q);
      if (q) check(d, q - 1);
    }
  }
  const uint32_t big[] = {65536u * 3, 1u << 20, 123456789u, 0x7fffffffu, 0x80000000u, 0x80000001u, 3000000000u, 0xfffffffeu, 0xffffffffu};
  for (uint32_t d : big)
    for (int k = 0; k < 100000; ++k) check(d, next());
  for (uint32_t d : {3u, 24u, 96u, 98304u})
    for (uint64_t n = 0; n <= 0xffffffffull; n += 977) check(d, uint32_t(n));
  printf("checked %ld, mismatches %ld\n", checked, bad);
  return bad != 0;
}
