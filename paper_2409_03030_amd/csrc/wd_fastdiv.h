// Division by a divisor fixed when a launch is set up, for the kernels' site
// and block index arithmetic (a runtime integer division compiles to about 20
// vector instructions on the GPU; this takes a multiply and a shift).
//
// For a divisor d >= 1 let l = floor(log2 d), s = 31 + l and m = ceil(2^s / d).
// Then floor(n / d) = floor(n m / 2^s) for every 0 <= n < 2^30: write
// m d = 2^s + e with 0 <= e < d < 2^(l+1) and n = q d + r with 0 <= r < d;
// n m / 2^s = q + (r + n e / 2^s) / d, and n e < 2^30 2^(l+1) = 2^s, so the
// fraction stays below 1.  m itself lies in (2^30, 2^31], so it fits 32 bits.
// This is the round-up reciprocal of Granlund and Montgomery (PLDI 1994).
//
// The includer defines WD_HD (the function qualifiers of the kernels' helpers).
#pragma once

#include <stdint.h>

namespace wd {

struct FastDiv {
  uint32_t m;  // ceil(2^s / d)
  uint32_t s;  // 31 + floor(log2 d)
};

// Host: the multiplier and shift of a divisor d >= 1 (d < 1 is taken as 1).
inline FastDiv make_fastdiv(int d) {
  const uint64_t dd = d < 1 ? 1u : (uint64_t)d;
  uint32_t l = 0;
  while ((dd >> (l + 1)) != 0) ++l;
  const uint32_t s = 31 + l;
  const uint64_t m = ((1ull << s) + dd - 1) / dd;
  return FastDiv{(uint32_t)m, s};
}

// floor(n / d) for 0 <= n < 2^30.
WD_HD int fdiv(int n, FastDiv f) { return (int)(((uint64_t)(uint32_t)n * f.m) >> f.s); }

}  // namespace wd
