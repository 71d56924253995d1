// Host check of the transforms' twiddle product and lazy bounds
// (modarith.h): mul_shoup_2q(x, w, wsh, 2^64 - 2q) with wsh = floor(w*2^63/q)
// equals x*w mod q and stays below 2.75q for every x < 6q; the inverse
// butterfly (X + Y brought below 3q, (X - Y + 3q)*w) keeps every value below
// 3q stage after stage; the forward butterfly (x0 brought below 3q, then
// X +- x1*w with 3q added to the difference) keeps every value below 6q, and
// canon_below6q brings such a value to [0, q).  Random and extreme operands, against exact 128-bit
// arithmetic.  Usage: shoup_host <q> <trials>; prints "ok <n>" or the first
// failure and exits 1.
#include <cstdio>
#include <cstdlib>

#include "modarith.h"

typedef unsigned __int128 u128;

static uint64_t sm_state = 0x9abcdef;
static uint64_t splitmix() {
  uint64_t z = (sm_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  const uint64_t q = strtoull(argv[1], 0, 10);
  const long trials = strtol(argv[2], 0, 10);
  const uint64_t neg2q = 0 - 2 * q, neg3q = 0 - 3 * q, q3 = 3 * q;
  const u128 bound = (u128)q * 11 / 4;  // 2.75q
  for (long n = 0; n < trials; n++) {
    const int mode = (int)(n % 4);
    uint64_t w = splitmix() % q;
    uint64_t x = splitmix() % (6 * q);
    if (mode == 1) x = 6 * q - 1;
    if (mode == 2) w = q - 1;
    if (mode == 3) x = 6 * q - 1 - (splitmix() & 0xffff), w = q - 1 - (splitmix() & 0xff);
    const uint64_t wsh = (uint64_t)(((u128)w << 63) / q);
    const uint64_t r = heconv::mul_shoup_2q(x, w, wsh, neg2q);
    if ((u128)r >= bound || r % q != (uint64_t)((u128)x * w % q)) {
      std::printf("mul_shoup_2q q=%llu x=%llu w=%llu r=%llu\n", (unsigned long long)q, (unsigned long long)x,
                  (unsigned long long)w, (unsigned long long)r);
      return 1;
    }
  }
  // thirteen butterfly stages on values that start below q (or at the bound)
  for (long n = 0; n < trials / 16; n++) {
    uint64_t X = n % 3 == 0 ? 3 * q - 1 : splitmix() % q, Y = n % 3 == 1 ? 3 * q - 1 : splitmix() % q;
    uint64_t ex = X % q, ey = Y % q;
    for (int st = 0; st < 13; st++) {
      const uint64_t w = n % 5 == 0 ? q - 1 : splitmix() % q, wsh = (uint64_t)(((u128)w << 63) / q);
      const uint64_t nx = heconv::csub_neg(X + Y, neg3q);
      const uint64_t ny = heconv::mul_shoup_2q(X - Y + q3, w, wsh, neg2q);
      const uint64_t fx = (ex + ey) % q, fy = (uint64_t)((u128)((ex + q - ey) % q) * w % q);
      if (nx >= q3 || ny >= q3 || nx % q != fx || ny % q != fy) {
        std::printf("butterfly q=%llu n=%ld stage %d\n", (unsigned long long)q, n, st);
        return 1;
      }
      X = (st & 1) ? ny : nx, Y = (st & 1) ? nx : ny;
      ex = (st & 1) ? fy : fx, ey = (st & 1) ? fx : fy;
    }
  }
  // thirteen forward stages (X = x0 below 3q, T = mul_shoup_2q(x1), X + T
  // and X - T + 3q, every value below 6q), then the canonical step
  for (long n = 0; n < trials / 16; n++) {
    uint64_t X = n % 3 == 0 ? 6 * q - 1 : splitmix() % q, Y = n % 3 == 1 ? 6 * q - 1 : splitmix() % q;
    uint64_t ex = X % q, ey = Y % q;
    for (int st = 0; st < 13; st++) {
      const uint64_t w = n % 5 == 0 ? q - 1 : splitmix() % q, wsh = (uint64_t)(((u128)w << 63) / q);
      const uint64_t A = heconv::csub_neg(X, neg3q);
      const uint64_t T = heconv::mul_shoup_2q(Y, w, wsh, neg2q);
      const uint64_t nx = A + T, ny = A - T + q3;
      const uint64_t t = (uint64_t)((u128)ey * w % q), fx = (ex + t) % q, fy = (ex + q - t) % q;
      if (A >= q3 || nx >= 6 * q || ny >= 6 * q || nx % q != fx || ny % q != fy) {
        std::printf("forward butterfly q=%llu n=%ld stage %d\n", (unsigned long long)q, n, st);
        return 1;
      }
      X = (st & 1) ? ny : nx, Y = (st & 1) ? nx : ny;
      ex = (st & 1) ? fy : fx, ey = (st & 1) ? fx : fy;
    }
    const uint64_t negq = 0 - q;
    if (heconv::canon_below6q(X, neg3q, neg2q, negq) != ex || heconv::canon_below6q(Y, neg3q, neg2q, negq) != ey) {
      std::printf("canonical step q=%llu n=%ld\n", (unsigned long long)q, n);
      return 1;
    }
  }
  for (uint64_t x = 0; x < 6 * q; x += q / 7 + 1)
    for (uint64_t d = 0; d < 3; d++) {
      const uint64_t v = x + d < 6 * q ? x + d : 6 * q - 1;
      if (heconv::canon_below6q(v, neg3q, neg2q, 0 - q) != v % q) {
        std::printf("canon_below6q q=%llu x=%llu\n", (unsigned long long)q, (unsigned long long)v);
        return 1;
      }
    }
  std::printf("ok %ld\n", trials);
  return 0;
}
