// Host check of the invariant-divisor division used by the kernels' index
// maps: udiv(n, udiv_make(d)) == n / d for edge and random n and d.
#include "gw_kernels.h"
#include <cstdio>
#include <cstdint>
int main() {
  unsigned long long bad = 0, n_checked = 0;
  uint64_t x = 88172645463325252ull;
  auto rnd = [&]() { x ^= x << 13; x ^= x >> 7; x ^= x << 17; return (unsigned)x; };
  auto check = [&](unsigned d) {
    const Udiv u = udiv_make(d);
    const unsigned edge[] = {0u, 1u, d - 1, d, d + 1, 2 * d - 1, 2 * d, 0x7fffffffu, 0x80000000u, 0xfffffffeu, 0xffffffffu};
    for (unsigned n : edge) { ++n_checked; if (udiv(n, u) != n / d) ++bad; }
    for (int i = 0; i < 2000; ++i) { unsigned n = rnd(); ++n_checked; if (udiv(n, u) != n / d) ++bad;
      unsigned m = n % (64u * d + 1u); ++n_checked; if (udiv(m, u) != m / d) ++bad; }
  };
  for (unsigned d = 1; d <= 5000; ++d) check(d);
  for (int i = 0; i < 5000; ++i) { unsigned d = rnd() >> (rnd() % 32); if (d) check(d); }
  check(0x7fffffffu); check(0x80000000u); check(0xffffffffu);
  printf("checked %llu bad %llu\n", n_checked, bad);
  return bad != 0;
}
