// Host check of the fixed-point summation the adjoint uses for the scattered
// probe-velocity adjoints (fix_split / fix_merge of the library's internal
// header): the sum of the pieces of n values, merged, must not depend on the
// order of the terms (bit for bit), must equal the exact sum of the rounded
// terms (128-bit integers) to one rounding, must lie within n 2^-65 of the
// sum of the unrounded terms (long double, up to its own rounding), and
// values beyond 2^40 or not
// finite must be refused.  Prints the number of failures; exit status 1 if any.
#include "hlbm_internal.h"

#include <cmath>
#include <cstdio>
#include <cstdint>
#include <random>
#include <algorithm>

using hlbm::fix_merge;
using hlbm::fix_split;

int main() {
  std::mt19937_64 g(20240611);
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  long failures = 0, cases = 0;
  double worst = 0.0;
  for (int trial = 0; trial < 40000; ++trial) {
    const int n = 1 + trial % 64;
    const double scale = std::ldexp(1.0, (trial % 100) - 70);  // 2^-70 .. 2^29
    double v[64];
    for (int k = 0; k < n; ++k) v[k] = u(g) * scale * (k % 7 == 3 ? 1e-6 : 1.0);
    long long a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    long double ref = 0.0L, mag = 0.0L;
    __int128 exact = 0;
    for (int k = 0; k < n; ++k) {
      long long p[3];
      if (!fix_split(v[k], p)) { ++failures; continue; }
      for (int j = 0; j < 3; ++j) a[j] = (long long)((unsigned long long)a[j] + (unsigned long long)p[j]);
      exact += ((__int128)p[0] << 64) + ((__int128)p[1] << 32) + (__int128)p[2];
      ref += (long double)v[k];
      mag += std::fabs((long double)v[k]);
    }
    std::shuffle(v, v + n, g);
    for (int k = 0; k < n; ++k) {
      long long p[3];
      fix_split(v[k], p);
      for (int j = 0; j < 3; ++j) b[j] = (long long)((unsigned long long)b[j] + (unsigned long long)p[j]);
    }
    const double sa = fix_merge(a[0], a[1], a[2]), sb = fix_merge(b[0], b[1], b[2]);
    ++cases;
    if (!(sa == sb)) { ++failures; continue; }
    // the exact sum of the rounded terms, converted once
    const double ex = (double)((long double)exact / 18446744073709551616.0L);
    if (std::fabs(sa - ex) > std::ldexp(std::fabs(ex), -52)) ++failures;
    const double err = std::fabs(sa - (double)ref);
    // rounding of each term to 2^-64, of the result, and of the long double sum itself
    const double bound = n * std::ldexp(1.0, -65) + std::ldexp(std::fabs((double)ref), -52) +
                         n * std::ldexp((double)mag, -63);
    if (err > bound) ++failures;
    worst = std::max(worst, err / bound);
  }
  // out of range and non-finite values are refused
  long long p[3] = {7, 7, 7};
  const double bad[4] = {std::ldexp(1.0, 40), -std::ldexp(1.0, 41), NAN, INFINITY};
  for (double x : bad)
    if (fix_split(x, p) || p[0] != 7) ++failures;
  if (!fix_split(std::ldexp(1.0, 40) * 0.999, p)) ++failures;
  std::printf("cases %ld failures %ld worst error / bound %.3f\n", cases, failures, worst);
  return failures ? 1 : 0;
}
