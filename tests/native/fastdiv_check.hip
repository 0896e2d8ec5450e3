// Host-only check of the multiply-and-shift division (FastDiv in tiles.hpp)
// against integer division: every divisor up to 70000 at the boundary
// indices and 64 random ones, and large divisors at 200000 random indices.
#include "tiles.hpp"
#include <cstdio>
#include <random>
using namespace pmsz;
int main() {
  std::mt19937_64 rng(1);
  long long bad = 0, tests = 0;
  auto check = [&](int64_t d, int32_t n) {
    FastDiv f = make_div(d);
    int32_t q = fdiv(n, f);
    ++tests;
    if (q != (int32_t)(n / d)) { if (bad < 10) printf("bad d=%lld n=%d q=%d\n", (long long)d, n, q); ++bad; }
  };
  for (int64_t d = 1; d <= 70000; ++d) {
    const int32_t ns[] = {0, 1, (int32_t)d - 1, (int32_t)d, (int32_t)d + 1, 2147483647, 2147483646, (int32_t)(2147483647 / d * d), (int32_t)(2147483647 / d * d - 1)};
    for (int32_t n : ns) if (n >= 0) check(d, n);
    for (int k = 0; k < 64; ++k) check(d, (int32_t)(rng() & 0x7fffffff));
  }
  const int64_t big[] = {134217728, 268435456, 1073741824, 2147483647, 1048576, 786432, 805306368, 1 << 24, 12345678, 99999989};
  for (int64_t d : big) for (int k = 0; k < 200000; ++k) check(d, (int32_t)(rng() & 0x7fffffff));
  printf("tests %lld bad %lld\n", tests, bad);
  return bad != 0;
}
