// Host check of the MAC's accumulator folds (modarith.h) against exact
// 128-bit arithmetic: fold30_pm and fold3_pm (primes 2^60 - delta,
// delta < 2^20; four and three accumulators).  Accumulators are built as the MAC builds
// them: up to 16 channel blocks of products of 30-bit halves of residues
// below q, plus the residue carried from the previous 16 blocks (its low 30
// bits in a00, its high bits in a01), with random and extreme operands.
// Usage: fold_host <q> <delta or 0> <trials>; prints "ok <n>" or the first
// mismatch and exits 1.
#include <cstdio>
#include <cstdlib>

#include "modarith.h"

using heconv::Half30;
using heconv::split30;
typedef unsigned __int128 u128;

static uint64_t sm_state = 0x1234567;
static uint64_t splitmix() {
  uint64_t z = (sm_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int main(int argc, char** argv) {
  if (argc < 4) return 2;
  const uint64_t q = strtoull(argv[1], 0, 10);
  const uint32_t delta = (uint32_t)strtoul(argv[2], 0, 10);
  const long trials = strtol(argv[3], 0, 10);
  for (long n = 0; n < trials; n++) {
    // 0 random, 1 all q-1, 2 mixed extremes, 3 few blocks, 4 every accumulator
    // at its bound, 5 accumulators uniform below their bounds
    const int mode = (int)(n % 6);
    const int blocks = mode == 3 ? 1 + (int)(splitmix() % 16) : 16;
    const uint64_t carry = mode == 1 ? q - 1 : splitmix() % q;
    uint64_t a00 = carry & ((1ull << 30) - 1), a01 = carry >> 30, a10 = 0, a11 = 0;
    for (int b = 0; b < blocks; b++) {
      uint64_t x = splitmix() % q, w = splitmix() % q;
      if (mode == 1) x = w = q - 1;
      if (mode == 2) {
        x = (b & 1) ? q - 1 : x;
        w = (b & 2) ? q - 1 : (b & 4 ? (1ull << 30) - 1 : w);
      }
      const Half30 xs = split30(x), ws = split30(w);
      a00 += (uint64_t)xs.lo * ws.lo;
      a01 += (uint64_t)xs.lo * ws.hi;
      a10 += (uint64_t)xs.hi * ws.lo;
      a11 += (uint64_t)xs.hi * ws.hi;
    }
    const uint64_t pmax = 16 * ((1ull << 30) - 1) * ((1ull << 30) - 1);  // 16 blocks at the largest halves
    if (mode == 4) a00 = pmax + ((1ull << 30) - 1), a01 = pmax + ((q - 1) >> 30), a10 = pmax, a11 = pmax;
    if (mode == 5) {
      a00 = splitmix() % (pmax + (1ull << 30));
      a01 = splitmix() % (pmax + ((q - 1) >> 30) + 1);
      a10 = splitmix() % (pmax + 1);
      a11 = splitmix() % (pmax + 1);
    }
    const u128 T = (u128)a00 + (((u128)a01 + a10) << 30) + ((u128)a11 << 60);
    const uint64_t want = (uint64_t)(T % q);
    uint64_t got = 0;
    if (delta) {
      got = heconv::fold30_pm(a00, a01, a10, a11, delta, 1u << 30);
    } else {
      std::printf("fold30 needs device constants; only fold30_pm is checked here\n");
      return 2;
    }
    if (got != want) {
      std::printf("mismatch q=%llu n=%ld a=%llu %llu %llu %llu got %llu want %llu\n", (unsigned long long)q, n,
                  (unsigned long long)a00, (unsigned long long)a01, (unsigned long long)a10,
                  (unsigned long long)a11, (unsigned long long)got, (unsigned long long)want);
      return 1;
    }
  }
  // three accumulators, eight blocks per fold: a00 and a11 take one product
  // of halves per block, am two; the carried value is fold3_pm's unreduced X
  // (below 2^60 + 2^45), which seeds a00 as the MAC seeds it.  Checked: the
  // carried X is congruent to the sum and below its bound, the final value
  // canonical.
  for (long n = 0; n < trials; n++) {
    const int mode = (int)(n % 5);
    const uint64_t m30 = (1ull << 30) - 1, xmax = (1ull << 60) + (1ull << 45);
    uint64_t carry = mode == 1 ? xmax - 1 : (mode == 2 ? q - 1 : splitmix() % xmax);
    if (mode == 3) carry = 0;
    for (int round = 0; round < 3; round++) {
      const int blocks = mode == 3 ? 1 + (int)(splitmix() % 8) : 8;
      uint64_t a00 = carry, am = 0, a11 = 0;
      for (int b = 0; b < blocks; b++) {
        uint64_t x = splitmix() % q, w = splitmix() % q;
        if (mode == 1 || (mode == 4 && (b & 1))) x = w = q - 1;
        const Half30 xs = split30(x), ws = split30(w);
        a00 += (uint64_t)xs.lo * ws.lo;
        am += (uint64_t)xs.lo * ws.hi;
        am += (uint64_t)xs.hi * ws.lo;
        a11 += (uint64_t)xs.hi * ws.hi;
      }
      if (mode == 1 && round == 2) {  // every accumulator at its bound
        const uint64_t p8 = 8 * m30 * m30;
        a00 = p8 + xmax - 1, am = 2 * p8, a11 = p8;
      }
      const u128 T = (u128)a00 + ((u128)am << 30) + ((u128)a11 << 60);
      const uint64_t want = (uint64_t)(T % q);
      const uint64_t X = heconv::fold3_pm<false>(a00, am, a11, delta, 1u << 30);
      const uint64_t r = heconv::fold3_pm<true>(a00, am, a11, delta, 1u << 30);
      if (X >= xmax || X % q != want || r != want) {
        std::printf("fold3 mismatch q=%llu n=%ld a=%llu %llu %llu X %llu r %llu want %llu\n", (unsigned long long)q, n,
                    (unsigned long long)a00, (unsigned long long)am, (unsigned long long)a11,
                    (unsigned long long)X, (unsigned long long)r, (unsigned long long)want);
        return 1;
      }
      carry = X;
    }
  }
  std::printf("ok %ld\n", trials);
  return 0;
}
