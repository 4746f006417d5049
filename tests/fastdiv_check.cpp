// Host check of the kernels' division by a fixed divisor (wd_fastdiv.h)
// against exact integer division: every divisor up to 4096 with the dividends
// where an error would show first (multiples of d and their neighbours, up to
// the 2^30 bound) and random ones, then large and power-of-two divisors.
// Prints "ok <count>" and exits 0, or prints the first mismatch and exits 1.
#include <stdint.h>
#include <stdio.h>

#define WD_HD inline
#include "wd_fastdiv.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t next_u32() {  // xorshift64*
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (uint32_t)((rng_state * 0x2545F4914F6CDD1Dull) >> 32);
}

static long long checked = 0;
static bool check(long long n, int d, const wd::FastDiv& f) {
  if (n < 0 || n >= (1ll << 30)) return true;
  ++checked;
  const int q = wd::fdiv((int)n, f);
  if (q != (int)(n / d)) {
    printf("mismatch: n=%lld d=%d got %d want %lld (m=%u s=%u)\n", n, d, q, n / d, f.m, f.s);
    return false;
  }
  return true;
}

static bool check_divisor(int d, int nrandom) {
  const wd::FastDiv f = wd::make_fastdiv(d);
  if (f.m <= (1u << 30) || f.m > (1u << 31)) {
    printf("multiplier out of range: d=%d m=%u\n", d, f.m);
    return false;
  }
  const long long top = (1ll << 30) - 1, dd = d;
  const long long small = 4 * dd + 8 < 65536 ? 4 * dd + 8 : 65536;
  for (long long n = 0; n < small; ++n)
    if (!check(n, d, f)) return false;
  for (long long k = top / dd - 3; k <= top / dd + 1; ++k)
    for (long long r = -1; r <= 1; ++r)
      if (!check(k * dd + r, d, f) || !check(k * dd + dd - 1 + r, d, f)) return false;
  if (!check(top, d, f)) return false;
  for (int i = 0; i < nrandom; ++i) {
    const long long n = next_u32() >> 2;
    const long long k = n / dd;
    if (!check(n, d, f) || !check(k * dd, d, f) || !check(k * dd - 1, d, f) || !check(k * dd + dd - 1, d, f))
      return false;
  }
  return true;
}

int main() {
  for (int d = 1; d <= 4096; ++d)
    if (!check_divisor(d, 2000)) return 1;
  for (int e = 12; e < 30; ++e) {
    const int p = 1 << e;
    if (!check_divisor(p - 1, 200) || !check_divisor(p, 200) || !check_divisor(p + 1, 200)) return 1;
  }
  for (int i = 0; i < 2000; ++i) {
    const int d = 1 + (int)(next_u32() >> 3);
    if (!check_divisor(d, 20)) return 1;
  }
  printf("ok %lld\n", checked);
  return 0;
}
