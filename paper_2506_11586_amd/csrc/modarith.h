// Device-side 64-bit modular arithmetic for primes q < 2^60 (gfx950).
//
// Shoup multiplication by a fixed operand: for w < q and w' = floor(w*2^64/q),
// any x < 2^64 gives r = x*w - umulhi(x, w')*q (mod 2^64) with r in [0, 2q)
// (Harvey, "Faster arithmetic for number-theoretic transforms", 2014).  Only
// the high half of x*w' and the low halves of x*w and hi*q are needed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace heconv {

// Per-limb constants kept on the device.
struct LimbConst {
  uint64_t q, two_q;
  uint64_t ninv, ninv_sh;      // N^-1 mod q and its Shoup quotient
  uint64_t ninv_w, ninv_w_sh;  // N^-1 * (last inverse twiddle) and quotient
  uint64_t r64, r64_sh;        // 2^64 mod q and its Shoup quotient
  uint64_t mu64;               // floor(2^64 / q): Shoup quotient of w = 1
  uint64_t c30, c30_sh;        // 2^30 mod q and its Shoup quotient
  uint64_t c60, c60_sh;        // 2^60 mod q and its Shoup quotient
  uint64_t delta, delta_sh;    // floor(Q/t) mod q and its Shoup quotient (0 if t is unusable)
  uint64_t negq, neg2q;        // 2^64 - q and 2^64 - 2q
  uint64_t r64_sh63;           // Shoup quotient of 2^64 mod q at scale 2^63
  uint64_t pmd;                // delta when q = 2^60 - delta with delta < 2^20, else 0
  uint64_t three_q, neg3q;     // 3q and 2^64 - 3q (the inverse transform's lazy bound)
};

// Device buffers are passed to the transform and MAC bodies as pointers in
// the global address space: a pointer loaded from memory (a job table) is
// otherwise generic to the compiler, whose loads and stores would then be
// flat ones with 64-bit per-lane addresses.
typedef __attribute__((address_space(1))) uint64_t gword;
typedef const __attribute__((address_space(1))) uint64_t cgword;

template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* as_global(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// A twiddle with its Shoup quotient at scale 2^63, wsh = floor(w*2^63/q),
// stored side by side (one 16-byte load).  See mul_shoup63.
struct Tw {
  uint64_t w, wsh;
};

__device__ __forceinline__ uint64_t mul_shoup_lazy(uint64_t x, uint64_t w, uint64_t wsh, uint64_t q) {
  uint64_t hi = __umul64hi(x, wsh);
  return x * w - hi * q;  // in [0, 2q)
}

__device__ __forceinline__ uint64_t csub(uint64_t x, uint64_t m) { return x >= m ? x - m : x; }

// The same two operations for the transforms' hot loops, written with the
// negated modulus (negq = 2^64 - q, a value loaded from memory, so the
// compiler keeps the additions): x*w + hi*negq is one multiply-add chain
// with no 64-bit subtract, and the conditional subtract selects on the sign
// of x - m, which holds for x, m < 2^63 (every value here is below 8q < 2^63).
__device__ __forceinline__ uint64_t mul_shoup_neg(uint64_t x, uint64_t w, uint64_t wsh, uint64_t negq) {
  return x * w + __umul64hi(x, wsh) * negq;  // in [0, 2q)
}

// Shoup multiplication at scale 2^63 for x < 2^62 and wsh = floor(w*2^63/q)
// (so wsh < 2^63): hi = floor(x*wsh / 2^63) = floor((2x)*wsh / 2^64), and
// with both 2x and wsh below 2^63 the two 32x32 cross products plus the
// carry word sum to less than 2^64, so the high word needs three
// multiply-adds and no carry handling.  Result in [0, 2q) (the Shoup bound
// holds for any x < 2^63 at this scale).
__device__ __forceinline__ uint64_t mul_shoup63(uint64_t x, uint64_t w, uint64_t wsh, uint64_t negq) {
  const uint64_t x2 = x << 1;
  const uint32_t a0 = (uint32_t)x2, a1 = (uint32_t)(x2 >> 32);
  const uint32_t b0 = (uint32_t)wsh, b1 = (uint32_t)(wsh >> 32);
  uint64_t s = (uint64_t)a1 * b0 + __umulhi(a0, b0);
  s += (uint64_t)a0 * b1;  // < 2^64: a1, b1 < 2^31
  const uint64_t hi = (uint64_t)a1 * b1 + (s >> 32);
  return x * w + hi * negq;
}

// The same quotient word without doubling x: top = floor(x*wsh / 2^64)
// (x < 6q < 2^62.6 and wsh < 2^63 keep the three partial products' sum
// below 2^64) approximates x*w/(2q) from below by less than 1 + x/2^64, so
// r = x*w - top*2q lies in [0, 2q(1 + 6q/2^64)) within [0, 2.75q).  Two
// instructions fewer than mul_shoup63 (no doubling of x), for callers whose
// lazy bound allows 2.75q.  neg2q = 2^64 - 2q.
__host__ __device__ __forceinline__ uint64_t mul_shoup_2q(uint64_t x, uint64_t w, uint64_t wsh, uint64_t neg2q) {
  const uint32_t a0 = (uint32_t)x, a1 = (uint32_t)(x >> 32);
  const uint32_t b0 = (uint32_t)wsh, b1 = (uint32_t)(wsh >> 32);
  uint64_t s = (uint64_t)a1 * b0 + __umulhi(a0, b0);
#ifdef __HIP_DEVICE_COMPILE__
  __asm__("" : "+v"(s));  // keeps the three multiply-adds in this order (no re-association)
#endif
  s += (uint64_t)a0 * b1;
  const uint64_t top = (uint64_t)a1 * b1 + (s >> 32);
  return x * w + top * neg2q;
}

__host__ __device__ __forceinline__ uint64_t csub_neg(uint64_t x, uint64_t negm) {
  const uint64_t d = x + negm;
  return (int64_t)d < 0 ? x : d;
}

// x < 6q brought to [0, q) by three conditional subtractions (3q, 2q, q);
// neg3q = 2^64 - 3q, and so on.
__host__ __device__ __forceinline__ uint64_t canon_below6q(uint64_t x, uint64_t neg3q, uint64_t neg2q,
                                                           uint64_t negq) {
  return csub_neg(csub_neg(csub_neg(x, neg3q), neg2q), negq);
}

// x < 2^64 reduced into [0, 2q) (Shoup with w = 1).
__device__ __forceinline__ uint64_t reduce64_lazy(uint64_t x, uint64_t mu64, uint64_t q) {
  return x - __umul64hi(x, mu64) * q;
}

// Full 64 x 64 -> 128-bit product as (hi, lo).
__device__ __forceinline__ void mul_wide(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
  lo = a * b;
  hi = __umul64hi(a, b);
}

// 128-bit value (hi, lo) reduced mod q into [0, q): hi*2^64 = hi*(2^64 mod q).
__device__ __forceinline__ uint64_t reduce128(uint64_t hi, uint64_t lo, const LimbConst& c) {
  uint64_t a = mul_shoup_lazy(hi, c.r64, c.r64_sh, c.q);  // [0, 2q)
  uint64_t b = reduce64_lazy(lo, c.mu64, c.q);            // [0, 2q)
  uint64_t s = a + b;                                     // [0, 4q) < 2^63
  s = csub(s, c.two_q);
  return csub(s, c.q);
}

// Residues below 2^60 split into 30-bit halves: x = hi*2^30 + lo.  Products
// of halves are below 2^60, so 16 of them fit one 64-bit accumulator and
// v_mad_u64_u32 accumulates them with no carry handling.
struct Half30 {
  uint32_t lo, hi;
};

__device__ __forceinline__ Half30 split30(uint64_t x) {
  return Half30{(uint32_t)x & 0x3fffffffu, (uint32_t)(x >> 30)};
}

// Bits [s, s+32) of the 64-bit value hi:lo (one v_alignbit_b32).
__host__ __device__ __forceinline__ uint32_t funnel32(uint32_t hi, uint32_t lo, int s) {
  return (uint32_t)((((uint64_t)hi << 32) | lo) >> s);
}

// Fold for a prime q = 2^60 - delta with delta < 2^20 (the largest primes
// below 2^60 are of this form): 2^60 = delta mod q, so a value lo + hi*2^60
// is congruent to lo + hi*delta.  With B = a01 + a10 (65 bits) the sum is
//   T = L + V*2^60,  L = (a00 mod 2^60) + (B mod 2^30)*2^30 < 2^61,
//                    V = a11 + (B >> 30) + (a00 >> 60) < 2^64,
// so T = W = L + V*delta (< 2^85) mod q, then W = X = (W mod 2^60) +
// (W >> 60)*delta < 2^60 + 2^45 < 2q, and X >= q exactly when X + delta
// carries into bit 60, where X - q = (X + delta) mod 2^60.  Every product
// is a 32 x 32 multiply-add; the only carry chain is that of B.  two30 is
// 2^30, passed in (from the limb constants) so that (B mod 2^30)*2^30 + ...
// stays one multiply-add instead of a 64-bit shift, a mask and an add.
// Exact for every a00, a01, a10, a11 < 2^64 with
// a11 + (a01 + a10) / 2^30 + a00 / 2^60 < 2^64, which sixteen blocks of
// 30-bit products (each below (2^30-1)^2) plus a carried residue below 2^60
// satisfy.
__host__ __device__ __forceinline__ uint64_t fold30_pm(uint64_t a00, uint64_t a01, uint64_t a10, uint64_t a11,
                                                       uint32_t delta, uint32_t two30) {
  constexpr uint32_t M28 = (1u << 28) - 1, M30 = (1u << 30) - 1;
  const uint64_t b = a01 + a10;
  const uint32_t bc4 = b < a01 ? 4u : 0u;  // bit 64 of B, as bit 34 of B >> 30
  const uint32_t b_lo = (uint32_t)b, b_hi = (uint32_t)(b >> 32);
  const uint32_t a_lo = (uint32_t)a00, a_hi = (uint32_t)(a00 >> 32);
  const uint64_t a60 = ((uint64_t)(a_hi & M28) << 32) | a_lo;
  const uint64_t Lv = (uint64_t)(b_lo & M30) * two30 + a60;                          // < 2^61
  const uint64_t b30 = ((uint64_t)(b_hi >> 30) << 32) | funnel32(b_hi, b_lo, 30);    // (B mod 2^64) >> 30
  const uint64_t V = a11 + b30 + (((uint64_t)bc4 << 32) | (a_hi >> 28));
  const uint64_t W1 = (uint64_t)(uint32_t)V * delta + Lv;                           // < 2^62
  const uint64_t P = (uint64_t)(uint32_t)(V >> 32) * delta + (uint32_t)(W1 >> 32);  // W >> 32, < 2^53
  const uint32_t wh = funnel32((uint32_t)(P >> 32), (uint32_t)P, 28);               // W >> 60, < 2^25
  const uint64_t wl = ((uint64_t)((uint32_t)P & M28) << 32) | (uint32_t)W1;          // W mod 2^60
  const uint64_t X = (uint64_t)wh * delta + wl;                                     // < 2^60 + 2^45
  const uint32_t ge = (uint32_t)((X + delta) >> 60);                                // X >= q
  const uint64_t Z = (uint64_t)ge * delta + X;
  return Z & ((1ull << 60) - 1);
}

// The same fold for three accumulators, T = a00 + am*2^30 + a11*2^60 (am
// takes both cross products of 30-bit halves): exact for a00, am < 2^64 and
// a11 < 2^63, which eight blocks of products (a00, a11 one per block, am
// two) on top of a carried value below 2^60 + 2^45 in a00 satisfy.  CANON:
// the result in [0, q); else X in [0, 2^60 + 2^45), congruent to T, which
// is all a carried value needs.
template <bool CANON>
__host__ __device__ __forceinline__ uint64_t fold3_pm(uint64_t a00, uint64_t am, uint64_t a11, uint32_t delta,
                                                      uint32_t two30) {
  constexpr uint32_t M28 = (1u << 28) - 1, M30 = (1u << 30) - 1;
  const uint32_t a_lo = (uint32_t)a00, a_hi = (uint32_t)(a00 >> 32);
  const uint64_t a60 = ((uint64_t)(a_hi & M28) << 32) | a_lo;
  const uint64_t Lv = (uint64_t)((uint32_t)am & M30) * two30 + a60;                 // < 2^61
  const uint64_t V = a11 + (am >> 30) + (a_hi >> 28);                               // < 2^64
  const uint64_t W1 = (uint64_t)(uint32_t)V * delta + Lv;                           // < 2^62
  const uint64_t P = (uint64_t)(uint32_t)(V >> 32) * delta + (uint32_t)(W1 >> 32);  // W >> 32, < 2^53
  const uint32_t wh = funnel32((uint32_t)(P >> 32), (uint32_t)P, 28);               // W >> 60, < 2^25
  const uint64_t wl = ((uint64_t)((uint32_t)P & M28) << 32) | (uint32_t)W1;          // W mod 2^60
  const uint64_t X = (uint64_t)wh * delta + wl;                                     // < 2^60 + 2^45
  if (!CANON) return X;
  const uint32_t ge = (uint32_t)((X + delta) >> 60);                                // X >= q
  const uint64_t Z = (uint64_t)ge * delta + X;
  return Z & ((1ull << 60) - 1);
}

// Exact sum of products in four accumulators: a00 + (a01 + a10)*2^30 +
// a11*2^60, reduced into [0, q).
__device__ __forceinline__ uint64_t fold30(uint64_t a00, uint64_t a01, uint64_t a10, uint64_t a11,
                                           const LimbConst& c) {
  // T = a00 + (a01 + a10)*2^30 + a11*2^60 < 2^125 as (hi, t), hi < 2^61 (q > 2^30,
  // so 2^30 needs no reduction); then T mod q = hi*(2^64 mod q) + t mod q:
  // one scale-2^63 Shoup product and one Shoup reduction of a word.
  const uint64_t s = a01 + a10;
  const uint64_t sc = s < a01;  // bit 64 of a01 + a10
  const uint64_t lo = a00 + (s << 30);
  const uint64_t c1 = lo < a00;
  const uint64_t t = lo + (a11 << 60);
  const uint64_t c2 = t < lo;
  const uint64_t hi = (s >> 34) + (sc << 30) + (a11 >> 4) + c1 + c2;
  uint64_t r = mul_shoup63(hi, c.r64, c.r64_sh63, c.negq) + reduce64_lazy(t, c.mu64, c.q);  // [0, 4q)
  r = csub(r, c.two_q);
  return csub(r, c.q);
}

}  // namespace heconv
