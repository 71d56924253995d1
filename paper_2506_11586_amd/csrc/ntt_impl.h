// Fused negacyclic NTT / inverse NTT for gfx950: one workgroup per limb
// polynomial, E = 2^LOGE coefficients per thread in registers, radix-E
// passes (LOGE butterfly stages each) with an LDS transpose between passes.
//
// Forward (Cooley-Tukey, natural order in, bit-reversed order out): the
// butterfly on bit b pairs j and j + 2^b with twiddle psi^brv(2^(n-1-b) +
// (j >> (b+1))), n = log2 N; stages run from bit n-1 down to bit 0.  The
// inverse (Gentleman-Sande) uses the same index with psi^-1 and runs from
// bit 0 up; its last stage also applies N^-1.  Lazy reduction after Harvey,
// with the twiddle products by mul_shoup_2q (inputs below 6q, results below
// 2.75q): forward values stay in [0, 6q) (X = x0 brought below 3q by one
// conditional subtraction, T = mul_shoup_2q(x1), outputs X + T < 5.75q and
// X - T + 3q < 6q), inverse values in [0, 3q) (the sum brought below 3q by
// one conditional subtraction, the difference X - Y + 3q, below 6q, through
// mul_shoup_2q).  Every stored word is canonical (fwd_canon, or the last
// inverse stage).
//
// Thread/element mapping of a pass over bits [lo, lo+LOGE): register k of
// thread t holds element j = (t mod 2^lo) | k << lo | (t >> lo) << (lo+LOGE).
// The top pass (lo = n-LOGE) is j = t + k*N/E: global loads and stores use
// it, so every wave access is a contiguous 512-byte run.  The forward
// transform ends on lo = 0 and goes through LDS once more to store in the
// top mapping; the inverse loads in the top mapping and goes through LDS to
// start at lo = 0.  When n is not a multiple of LOGE the leftover bits are
// done by a partial pass at lo = 0.
#pragma once
#include "modarith.h"


namespace heconv {

__device__ __forceinline__ int lds_pad(int j) { return j + (j >> 4); }

template <int LOGE, int LO>
__device__ __forceinline__ int elem_index(int tid, int k) {
  const int low = tid & ((1 << LO) - 1);
  const int high = tid >> LO;
  return low | (k << LO) | (high << (LO + LOGE));
}

// tid >> LO, the index of the thread's block of 2^LO elements.  From LO = 6
// up every lane of a wave has the same value (tid = 64w + i gives
// w >> (LO - 6)); it is then read from the first lane, so the twiddle index
// is uniform and its loads are scalar loads shared by the wave.
template <int LO>
__device__ __forceinline__ int block_of(int tid) {
  if constexpr (LO >= 6)
    return __builtin_amdgcn_readfirstlane(tid >> LO);
  else
    return tid >> LO;
}

// A forward value (below 6q) brought to [0, q).
__device__ __forceinline__ uint64_t fwd_canon(uint64_t x, const LimbConst& c) {
  return canon_below6q(x, c.neg3q, c.neg2q, c.negq);
}

// Forward stages u in [U0, LOGE) of the pass at bit offset LO.  jb: index
// of the workgroup's first element when it transforms a block of a longer
// polynomial (the stages on bits below the block size only; jb a multiple of
// the block size), else 0.
template <int LOGN, int LOGE, int LO, int U0>
__device__ __forceinline__ void fwd_pass(uint64_t (&x)[1 << LOGE], int tid, const Tw* __restrict__ tw,
                                         const LimbConst& c, uint32_t jb = 0) {
  const int high = block_of<LO>(tid);
  const uint64_t q3 = c.three_q;
#pragma unroll
  for (int u = U0; u < LOGE; u++) {
    const int s = LOGN - LOGE - LO + u;  // stage index: butterflies on bit LO+LOGE-1-u
    const int half = 1 << (LOGE - 1 - u);
#pragma unroll
    for (int g = 0; g < (1 << u); g++) {
      const Tw t = tw[(1 << s) + (jb >> (LO + LOGE - u)) + (high << u) + g];
#pragma unroll
      for (int e = 0; e < half; e++) {
        const int k0 = g * 2 * half + e, k1 = k0 + half;
        const uint64_t X = csub_neg(x[k0], c.neg3q);
        const uint64_t T = mul_shoup_2q(x[k1], t.w, t.wsh, c.neg2q);
        x[k0] = X + T;
        x[k1] = X - T + q3;
      }
    }
  }
}

// Inverse stages u from LOGE-1 down to U0 of the pass at LO.  With LAST, the
// stage on the top bit (u = 0 of the pass at n-LOGE) also applies N^-1 and
// leaves canonical values.  jb as in fwd_pass (a block's first element, for
// the stages on bits below the block size; never with LAST).
template <int LOGN, int LOGE, int LO, int U0, bool LAST>
__device__ __forceinline__ void inv_pass(uint64_t (&x)[1 << LOGE], int tid, const Tw* __restrict__ tw,
                                         const LimbConst& c, uint32_t jb = 0) {
  const int high = block_of<LO>(tid);
  const uint64_t q3 = c.three_q;
#pragma unroll
  for (int u = LOGE - 1; u >= U0; u--) {
    const int s = LOGN - LOGE - LO + u;
    const int half = 1 << (LOGE - 1 - u);
    if (LAST && u == 0) {
#pragma unroll
      for (int e = 0; e < half; e++) {
        const int k0 = e, k1 = e + half;
        uint64_t X = x[k0], Y = x[k1];
        x[k0] = csub_neg(mul_shoup_neg(X + Y, c.ninv, c.ninv_sh, c.negq), c.negq);
        x[k1] = csub_neg(mul_shoup_neg(X - Y + q3, c.ninv_w, c.ninv_w_sh, c.negq), c.negq);
      }
      continue;
    }
#pragma unroll
    for (int g = 0; g < (1 << u); g++) {
      const Tw t = tw[(1 << s) + (jb >> (LO + LOGE - u)) + (high << u) + g];
#pragma unroll
      for (int e = 0; e < half; e++) {
        const int k0 = g * 2 * half + e, k1 = k0 + half;
        uint64_t X = x[k0], Y = x[k1];
        x[k0] = csub_neg(X + Y, c.neg3q);
        x[k1] = mul_shoup_2q(X - Y + q3, t.w, t.wsh, c.neg2q);
      }
    }
  }
}

// Move the thread's registers from the mapping at FROM to the mapping at TO
// through LDS.  The leading barrier keeps the previous exchange's readers
// ahead of this exchange's writers.
//
// Wave-local form.  In a mapping with LO <= 6 the 64 threads of wave w
// (tid = 64w + i) hold exactly the elements whose index bits from 6+LOGE up
// equal w: the low LO bits come from i, and tid >> LO = w*2^(6-LO) + (i >> LO).
// When FROM and TO both satisfy this, each wave writes and reads only its
// own aligned block of 2^(6+LOGE) elements (a disjoint range of LDS after
// padding), so no other wave is involved and no workgroup barrier is needed.
// The LDS operations of one wave are performed in issue order, and the
// empty asm statements with a memory clobber keep the compiler from moving
// a read above a write (for one lane the addresses differ, so it otherwise
// could).  The exchange before a wave-local one either is wave-local too or
// ends with every wave reading its own block, so the leading barrier can go
// as well.  A cross-wave exchange keeps both barriers, which also order it
// after any wave-local one.
template <int LOGE, int FROM, int TO>
__device__ __forceinline__ void exchange(uint64_t* lds, uint64_t (&x)[1 << LOGE], int tid) {
  constexpr bool WAVE = FROM <= 6 && TO <= 6;
  if constexpr (WAVE)
    asm volatile("" ::: "memory");
  else
    __syncthreads();
#pragma unroll
  for (int k = 0; k < (1 << LOGE); k++) lds[lds_pad(elem_index<LOGE, FROM>(tid, k))] = x[k];
  if constexpr (WAVE)
    asm volatile("" ::: "memory");
  else
    __syncthreads();
#pragma unroll
  for (int k = 0; k < (1 << LOGE); k++) x[k] = lds[lds_pad(elem_index<LOGE, TO>(tid, k))];
}

// Forward full passes at LO = LOGN-LOGE*(P+1), then the partial pass.
template <int LOGN, int LOGE, int P>
__device__ __forceinline__ void fwd_rest(uint64_t (&x)[1 << LOGE], uint64_t* lds, int tid,
                                         const Tw* __restrict__ tw, const LimbConst& c) {
  constexpr int NFULL = LOGN / LOGE, REM = LOGN % LOGE;
  if constexpr (P < NFULL) {
    constexpr int LO = LOGN - LOGE * (P + 1);
    if constexpr (P > 0) exchange<LOGE, LO + LOGE, LO>(lds, x, tid);
    fwd_pass<LOGN, LOGE, LO, 0>(x, tid, tw, c);
    fwd_rest<LOGN, LOGE, P + 1>(x, lds, tid, tw, c);
  } else if constexpr (REM > 0) {
    exchange<LOGE, LOGN - LOGE * NFULL, 0>(lds, x, tid);
    fwd_pass<LOGN, LOGE, 0, LOGE - REM>(x, tid, tw, c);
  }
}

// Inverse full passes at LO = REM + LOGE*P (the partial pass at LO = 0, if
// any, has already run).
template <int LOGN, int LOGE, int P>
__device__ __forceinline__ void inv_rest(uint64_t (&x)[1 << LOGE], uint64_t* lds, int tid,
                                         const Tw* __restrict__ tw, const LimbConst& c) {
  constexpr int NFULL = LOGN / LOGE, REM = LOGN % LOGE;
  if constexpr (P < NFULL) {
    constexpr int LO = REM + LOGE * P;
    constexpr int PREV = (P == 0) ? 0 : REM + LOGE * (P - 1);
    if constexpr (P > 0 || REM > 0) exchange<LOGE, PREV, LO>(lds, x, tid);
    inv_pass<LOGN, LOGE, LO, 0, (P == NFULL - 1)>(x, tid, tw, c);
    inv_rest<LOGN, LOGE, P + 1>(x, lds, tid, tw, c);
  }
}

// Forward transform of one limb polynomial a[N] (in place) by the calling
// workgroup of N/2^LOGE threads.
template <int LOGN, int LOGE>
__device__ __forceinline__ void ntt_fwd_poly(gword* __restrict__ a, const Tw* __restrict__ tw, const LimbConst& c,
                                             uint64_t* lds, int tid) {
  constexpr int N = 1 << LOGN, E = 1 << LOGE, T = N / E, TOP = LOGN - LOGE;
  uint64_t x[E];
#pragma unroll
  for (int k = 0; k < E; k++) x[k] = a[tid + k * T];
  fwd_rest<LOGN, LOGE, 0>(x, lds, tid, tw, c);
#pragma unroll
  for (int k = 0; k < E; k++) x[k] = fwd_canon(x[k], c);
  exchange<LOGE, 0, TOP>(lds, x, tid);  // back to j = tid + k*T for a coalesced store
#pragma unroll
  for (int k = 0; k < E; k++) a[tid + k * T] = x[k];
}

// Inverse transform of NTT values already in registers in the top mapping
// (register k of thread t = entry t + k*N/E); leaves the coefficients, in
// the same mapping, canonical.
template <int LOGN, int LOGE>
__device__ __forceinline__ void ntt_inv_regs(uint64_t (&x)[1 << LOGE], const Tw* __restrict__ tw, const LimbConst& c,
                                             uint64_t* lds, int tid) {
  constexpr int TOP = LOGN - LOGE, REM = LOGN % LOGE;
  exchange<LOGE, TOP, 0>(lds, x, tid);
  if constexpr (REM > 0) inv_pass<LOGN, LOGE, 0, LOGE - REM, false>(x, tid, tw, c);
  inv_rest<LOGN, LOGE, 0>(x, lds, tid, tw, c);
}

// Inverse transform of one limb polynomial a[N] (in place).  With NT the
// input is loaded and the result stored non-temporally: a layer's MAC output
// is read once here, and its result is not read again soon, so streaming
// both past the caches keeps L2 and the Infinity Cache for the weights.
template <int LOGN, int LOGE, bool NT = false>
__device__ __forceinline__ void ntt_inv_poly(gword* __restrict__ a, const Tw* __restrict__ tw, const LimbConst& c,
                                             uint64_t* lds, int tid) {
  constexpr int N = 1 << LOGN, E = 1 << LOGE, T = N / E;
  uint64_t x[E];
#pragma unroll
  for (int k = 0; k < E; k++) {  // coalesced, top mapping
    if constexpr (NT)
      x[k] = __builtin_nontemporal_load(&a[tid + k * T]);
    else
      x[k] = a[tid + k * T];
  }
  ntt_inv_regs<LOGN, LOGE>(x, tw, c, lds, tid);
#pragma unroll
  for (int k = 0; k < E; k++) {
    if constexpr (NT)
      __builtin_nontemporal_store(x[k], &a[tid + k * T]);
    else
      a[tid + k * T] = x[k];
  }
}

}  // namespace heconv
