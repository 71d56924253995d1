// Division of wave-uniform 31-bit values by a divisor fixed per launch,
// as one multiply-high and a shift (Granlund and Montgomery, "Division by
// invariant integers using multiplication", 1994): with l = ceil(log2 d)
// and m = ceil(2^(31+l) / d) < 2^32, floor(n/d) = floor(n*m / 2^(31+l)) for
// every n < 2^31, because m*d - 2^(31+l) < d <= 2^l.  On the device the
// multiply-high of uniform operands is a scalar instruction, so a kernel
// decodes its tile index with no vector division.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace heconv {

struct UDiv {
  uint32_t d, m, s;  // divisor, magic, shift (l - 1); d = 1 divides by itself
};

inline UDiv udiv_make(uint32_t d) {
  if (d <= 1) return UDiv{1, 0, 0};
  uint32_t l = 0;
  while ((1ull << l) < d) l++;
  const uint64_t m = (((uint64_t)1 << (31 + l)) + d - 1) / d;
  return UDiv{d, (uint32_t)m, l - 1};
}

__host__ __device__ __forceinline__ uint32_t udiv(uint32_t n, const UDiv& v) {
  return v.d == 1 ? n : __umulhi(n, v.m) >> v.s;
}

}  // namespace heconv
