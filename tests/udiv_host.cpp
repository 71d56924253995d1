// Host check of udiv.h: floor(n/d) by multiply-high and shift equals the
// quotient for every divisor given and numerators spread over [0, 2^31)
// (all of them below 2^16, the largest ones, multiples of d and their
// neighbours, and a pseudo-random sample).  Usage: udiv_host <d>...;
// prints "ok" or the first mismatch and exits 1.
#include <cstdio>
#include <cstdlib>

#include "udiv.h"

int main(int argc, char** argv) {
  uint64_t st = 0x5eed;
  for (int a = 1; a < argc; a++) {
    const uint32_t d = (uint32_t)strtoul(argv[a], 0, 10);
    const heconv::UDiv v = heconv::udiv_make(d);
    auto check = [&](uint32_t n) {
      if (n >= (1u << 31)) return true;
      if (heconv::udiv(n, v) != n / d) {
        std::printf("d=%u n=%u got %u want %u\n", d, n, heconv::udiv(n, v), n / d);
        return false;
      }
      return true;
    };
    for (uint32_t n = 0; n < (1u << 16); n++)
      if (!check(n)) return 1;
    for (uint32_t k = 0; k < (1u << 16); k++)
      if (!check((1u << 31) - 1 - k)) return 1;
    for (uint64_t k = 1; k * d < (1ull << 31) && k < (1u << 20); k++)
      if (!check((uint32_t)(k * d - 1)) || !check((uint32_t)(k * d)) || !check((uint32_t)(k * d + 1))) return 1;
    for (int k = 0; k < 1000000; k++) {
      st = st * 6364136223846793005ull + 1442695040888963407ull;
      if (!check((uint32_t)(st >> 33))) return 1;
    }
  }
  std::printf("ok\n");
  return 0;
}
