// Channel-block multiply-accumulate in the NTT domain (device part), used by
// the standalone MAC kernel and by the batch executor.
#pragma once
#include "modarith.h"

namespace heconv {

// ---------------------------------------------------------------------------
// MAC over channel blocks.  Every NTT point (l, k) is an independent small
// product Out[(b,s,c), m] = sum_cb In[(b,s,c), cb] * W[cb, m] mod q_l.  A
// thread owns one k for a tile of MT output channels x RT rows (b, s, c).
// Each operand is split into 30-bit halves and the four partial products
// are accumulated exactly in 64-bit registers (16 channel blocks per
// accumulator), then folded mod q once per 16 blocks; the folded residue
// seeds the next 16 blocks' accumulators (its low 30 bits in a00, the rest
// in a01), so no separate running sum is kept.  Consecutive lanes take
// consecutive k: every load and store is a coalesced 512-byte wave access.
// ---------------------------------------------------------------------------
constexpr uint32_t MAC_CHUNK = 16;

// Workgroups are dispatched round-robin over the 8 XCDs.  Remap so that
// consecutive tile ids land on one XCD: the tiles of one k-chunk (which
// read the same input and weight words) then share that XCD's L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nblocks) {
  const uint32_t full = nblocks / 8 * 8;
  if (bid >= full) return bid;
  const uint32_t per = full / 8;
  return (bid % 8) * per + bid / 8;
}

// Buffer resources (gfx9 layout: base, no stride, size in bytes, raw dword
// access) let a load take a uniform byte offset in a scalar register and
// the lane's offset in one 32-bit register, with no per-lane 64-bit address
// arithmetic.  Every offset used here stays below 2^31 bytes; the launchers
// check that one image's input and one output channel's weights do.
constexpr int MAC_BUF_FLAGS = 0x00020000;
constexpr uint64_t MAC_BUF_MAX_BYTES = 0x7fffffffull;

// A value the caller knows to be the same in every lane, moved to scalar
// registers (integer division of uniform values is expanded with vector
// instructions, after which the compiler no longer sees the result as
// uniform and would wrap every buffer load in a loop over lane values).
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t mac_rsrc(const void* base, uint64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, MAC_BUF_FLAGS);
}

__device__ __forceinline__ uint64_t mac_load(__amdgpu_buffer_rsrc_t r, uint32_t lane_bytes, uint32_t uniform_bytes) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)lane_bytes, (int)uniform_bytes, 0);
  return ((uint64_t)v[1] << 32) | v[0];
}

#ifndef HECONV_MAC_DEPTH
#define HECONV_MAC_DEPTH 4
#endif
constexpr int MAC_DEPTH = HECONV_MAC_DEPTH;

// One channel block: the four 30-bit partial products of every (m, row).
template <int MT, int RT>
__device__ __forceinline__ void mac_step(const uint64_t (&xr)[RT], const uint64_t (&wr)[MT], uint64_t (&a00)[MT][RT],
                                         uint64_t (&a01)[MT][RT], uint64_t (&a10)[MT][RT],
                                         uint64_t (&a11)[MT][RT]) {
  Half30 xs[RT], ws[MT];
#pragma unroll
  for (int i = 0; i < RT; i++) xs[i] = split30(xr[i]);
#pragma unroll
  for (int j = 0; j < MT; j++) ws[j] = split30(wr[j]);
#pragma unroll
  for (int j = 0; j < MT; j++)
#pragma unroll
    for (int i = 0; i < RT; i++) {
      a00[j][i] += (uint64_t)xs[i].lo * ws[j].lo;
      a01[j][i] += (uint64_t)xs[i].lo * ws[j].hi;
      a10[j][i] += (uint64_t)xs[i].hi * ws[j].lo;
      a11[j][i] += (uint64_t)xs[i].hi * ws[j].hi;
    }
}

// Fold every (m, row) accumulator set of a tile into its residue mod q and
// leave it as the seed of the next blocks: a00 = r mod 2^30, a01 = r >> 30,
// a10 = a11 = 0 (the bounds of both folds hold for 16 blocks plus that
// seed).  Primes 2^60 - delta with delta < 2^20 (c.pmd = delta) take the
// shift-and-multiply-by-delta fold, other primes the Shoup fold.
template <int MT, int RT>
__device__ __forceinline__ void mac_fold(uint64_t (&a00)[MT][RT], uint64_t (&a01)[MT][RT], uint64_t (&a10)[MT][RT],
                                         uint64_t (&a11)[MT][RT], const LimbConst& c) {
  if (c.pmd) {
#pragma unroll
    for (int j = 0; j < MT; j++)
#pragma unroll
      for (int i = 0; i < RT; i++) {
        const uint64_t r = fold30_pm(a00[j][i], a01[j][i], a10[j][i], a11[j][i], (uint32_t)c.pmd, (uint32_t)c.c30);
        a00[j][i] = r & 0x3fffffffu, a01[j][i] = r >> 30, a10[j][i] = 0, a11[j][i] = 0;
      }
  } else {
#pragma unroll
    for (int j = 0; j < MT; j++)
#pragma unroll
      for (int i = 0; i < RT; i++) {
        const uint64_t r = fold30(a00[j][i], a01[j][i], a10[j][i], a11[j][i], c);
        a00[j][i] = r & 0x3fffffffu, a01[j][i] = r >> 30, a10[j][i] = 0, a11[j][i] = 0;
      }
  }
}

// The tile's residues, each folded once more and stored non-temporally
// (streamed past the caches, which keep the weights).  Output (row i,
// channel j) starts at a uniform address, obase[i] + j * mstride words, and
// the lane adds its own word: the store takes the scalar-base form.  The
// fold is chosen once for the whole tile (PM: q = 2^60 - delta).
template <int MT, int RT, bool PM>
__device__ __forceinline__ void mac_store(const uint64_t (&a00)[MT][RT], const uint64_t (&a01)[MT][RT],
                                          const uint64_t (&a10)[MT][RT], const uint64_t (&a11)[MT][RT],
                                          const LimbConst& c, gword* __restrict__ out, const uint64_t (&obase)[RT],
                                          uint64_t mstride, const bool (&mv)[MT], const bool (&rv)[RT],
                                          uint32_t lane) {
#pragma unroll
  for (int j = 0; j < MT; j++)
#pragma unroll
    for (int i = 0; i < RT; i++) {
      const uint64_t r = PM ? fold30_pm(a00[j][i], a01[j][i], a10[j][i], a11[j][i], (uint32_t)c.pmd, (uint32_t)c.c30)
                            : fold30(a00[j][i], a01[j][i], a10[j][i], a11[j][i], c);
      if (mv[j] && rv[i]) {
        gword* o = out + uniform64(obase[i] + (uint64_t)j * mstride);
        __builtin_nontemporal_store(r, &o[lane]);
      }
    }
}

// One MAC tile: k-chunk kc (THREADS consecutive NTT points of limb
// kc / (N/THREADS)), output channels mt*MT.., rows rt*RT.., for the calling
// workgroup of THREADS threads.  c = constants of that limb.
template <int MT, int RT, int THREADS>
__device__ __forceinline__ void mac_tile(cgword* __restrict__ in, cgword* __restrict__ w, gword* __restrict__ out, uint32_t CB, uint32_t S, uint32_t M, uint32_t L,
                                         uint32_t N, uint32_t rows, uint32_t kc, uint32_t mt, uint32_t rt,
                                         const LimbConst& c, int tid) {
  const uint32_t chunks_per_limb = N / THREADS;
  const uint32_t l = kc / chunks_per_limb;
  // element (l, k) with k = kbase + tid: every address is a uniform base
  // (scalar registers) plus the lane's tid, so the loads take the
  // scalar-base form and need no per-lane address arithmetic
  const uint64_t kofs = (uint64_t)l * N + (kc % chunks_per_limb) * THREADS;
  const uint64_t LN = (uint64_t)L * N;

  // row r = (b*S + s)*2 + comp; input of (r, cb) at ib[i] + cb*in_cb_stride,
  // weights of (m, cb) at wb[j] + cb*LN, output of (r, m) at out_off[i] + m*out_m_stride
  const uint64_t in_cb_stride = (uint64_t)S * 2 * LN;  // cb -> cb+1 in the input
  const uint64_t out_m_stride = (uint64_t)S * 2 * LN;  // m -> m+1 in the output
  __amdgpu_buffer_rsrc_t ib[RT], wb[MT];
  uint64_t out_off[RT];
  bool rv[RT];
#pragma unroll
  for (int i = 0; i < RT; i++) {
    const uint32_t r = rt * RT + i;
    rv[i] = r < rows;
    const uint32_t rr = rv[i] ? r : 0;
    const uint32_t comp = rr & 1, bs = rr >> 1;
    const uint32_t b = bs / S, s = bs % S;
    ib[i] = mac_rsrc((const uint64_t*)in + uniform64(((((uint64_t)b * CB) * S + s) * 2 + comp) * LN + kofs),
                     (uint64_t)CB * in_cb_stride * 8);
    out_off[i] = ((((uint64_t)b * M) * S + s) * 2 + comp) * LN + kofs;
  }
  bool mv[MT];
#pragma unroll
  for (int j = 0; j < MT; j++) {
    const uint32_t m = mt * MT + j;
    mv[j] = m < M;
    wb[j] = mac_rsrc((const uint64_t*)w + uniform64(((uint64_t)(mv[j] ? m : 0) * CB) * LN + kofs),
                     (uint64_t)CB * LN * 8);
  }
  const uint32_t lane = (uint32_t)tid * 8;

  uint64_t a00[MT][RT], a01[MT][RT], a10[MT][RT], a11[MT][RT];
#pragma unroll
  for (int j = 0; j < MT; j++)
#pragma unroll
    for (int i = 0; i < RT; i++) a00[j][i] = a01[j][i] = a10[j][i] = a11[j][i] = 0;

  // Rows and channels past the end read row 0 / channel 0 (valid memory);
  // their sums are never stored, so every load is unconditional.
  for (uint32_t cb0 = 0; cb0 < CB; cb0 += MAC_CHUNK) {
    const uint32_t cb1 = cb0 + MAC_CHUNK < CB ? cb0 + MAC_CHUNK : CB;
    uint32_t cb = cb0;
    // MAC_DEPTH channel blocks per step: all their loads are issued before
    // the first product, so that many loads per thread are in flight
    for (; cb + MAC_DEPTH <= cb1; cb += MAC_DEPTH) {
      uint64_t xr[MAC_DEPTH][RT], wr[MAC_DEPTH][MT];
#pragma unroll
      for (int d = 0; d < MAC_DEPTH; d++) {
#pragma unroll
        for (int i = 0; i < RT; i++) xr[d][i] = mac_load(ib[i], lane, (uint32_t)((cb + d) * in_cb_stride * 8));
#pragma unroll
        for (int j = 0; j < MT; j++) wr[d][j] = mac_load(wb[j], lane, (uint32_t)((cb + d) * LN * 8));
      }
#pragma unroll
      for (int d = 0; d < MAC_DEPTH; d++) mac_step<MT, RT>(xr[d], wr[d], a00, a01, a10, a11);
    }
    for (; cb < cb1; cb++) {
      uint64_t xr[RT], wr[MT];
#pragma unroll
      for (int i = 0; i < RT; i++) xr[i] = mac_load(ib[i], lane, (uint32_t)(cb * in_cb_stride * 8));
#pragma unroll
      for (int j = 0; j < MT; j++) wr[j] = mac_load(wb[j], lane, (uint32_t)(cb * LN * 8));
      mac_step<MT, RT>(xr, wr, a00, a01, a10, a11);
    }
    if (cb1 < CB) mac_fold<MT, RT>(a00, a01, a10, a11, c);
  }
  uint64_t obase[RT];
#pragma unroll
  for (int i = 0; i < RT; i++) obase[i] = out_off[i] + (uint64_t)(mt * MT) * out_m_stride;
  if (c.pmd)
    mac_store<MT, RT, true>(a00, a01, a10, a11, c, out, obase, out_m_stride, mv, rv, (uint32_t)tid);
  else
    mac_store<MT, RT, false>(a00, a01, a10, a11, c, out, obase, out_m_stride, mv, rv, (uint32_t)tid);
}

// ---------------------------------------------------------------------------
// Helpers of the streamed MAC (mac_stream.h), whose operands are staged in
// LDS by direct buffer-to-LDS loads (gfx950 buffer_load_dwordx4 ... lds):
// every wave streams its own 64 NTT points through a private ring of P
// stages of MT + RT rows (512 bytes a row), one load instruction filling two
// rows (lanes 0-31 the first row's 512 bytes, lanes 32-63 the second's).
// LDS per workgroup: (THREADS / 64) * P * (MT + RT) * 512 bytes.
// ---------------------------------------------------------------------------
template <int MT, int RT, int THREADS, int P>
constexpr uint32_t mac_dma_lds_words() {
  return (uint32_t)(THREADS / 64) * P * (MT + RT) * 64;
}

__device__ __forceinline__ void mac_dma_load(__amdgpu_buffer_rsrc_t r, uint64_t* lds_row_pair, uint32_t lane_bytes,
                                             uint32_t uniform_bytes) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds_row_pair, 16,
                                           (int)lane_bytes, (int)uniform_bytes, 0, 0);
}

// s_waitcnt with only the vector-memory counter limited (gfx9 encoding:
// vmcnt bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at their maxima).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt is six bits");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

}  // namespace heconv
