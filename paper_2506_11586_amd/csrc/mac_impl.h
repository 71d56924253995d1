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
// accumulator), then folded mod q once per 16 blocks.  Consecutive lanes
// take consecutive k: every load and store is a coalesced 512-byte wave
// access.
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

// One MAC tile: k-chunk kc (THREADS consecutive NTT points of limb
// kc / (N/THREADS)), output channels mt*MT.., rows rt*RT.., for the calling
// workgroup of THREADS threads.  c = constants of that limb.
template <int MT, int RT, int THREADS>
__device__ __forceinline__ void mac_tile(cgword* __restrict__ in, cgword* __restrict__ w, gword* __restrict__ out, uint32_t CB, uint32_t S, uint32_t M, uint32_t L,
                                         uint32_t N, uint32_t rows, uint32_t kc, uint32_t mt, uint32_t rt,
                                         const LimbConst& c, int tid) {
  const uint32_t chunks_per_limb = N / THREADS;
  const uint32_t l = kc / chunks_per_limb;
  const uint32_t k = (kc % chunks_per_limb) * THREADS + tid;
  const uint64_t LN = (uint64_t)L * N;

  // row r = (b*S + s)*2 + comp; input address of (r, cb) and output of (r, m)
  cgword* ip[RT];
  uint64_t out_off[RT];
  bool rv[RT];
#pragma unroll
  for (int i = 0; i < RT; i++) {
    const uint32_t r = rt * RT + i;
    rv[i] = r < rows;
    const uint32_t rr = rv[i] ? r : 0;
    const uint32_t comp = rr & 1, bs = rr >> 1;
    const uint32_t b = bs / S, s = bs % S;
    ip[i] = in + ((((uint64_t)b * CB) * S + s) * 2 + comp) * LN + (uint64_t)l * N + k;
    out_off[i] = ((((uint64_t)b * M) * S + s) * 2 + comp) * LN + (uint64_t)l * N + k;
  }
  const uint64_t in_cb_stride = (uint64_t)S * 2 * LN;  // cb -> cb+1 in the input
  const uint64_t out_m_stride = (uint64_t)S * 2 * LN;  // m -> m+1 in the output
  bool mv[MT];
  cgword* wp[MT];
#pragma unroll
  for (int j = 0; j < MT; j++) {
    const uint32_t m = mt * MT + j;
    mv[j] = m < M;
    wp[j] = w + ((uint64_t)(mv[j] ? m : 0) * CB) * LN + (uint64_t)l * N + k;
  }

  uint64_t res[MT][RT];
#pragma unroll
  for (int j = 0; j < MT; j++)
#pragma unroll
    for (int i = 0; i < RT; i++) res[j][i] = 0;

  // Rows and channels past the end read row 0 / channel 0 (valid memory);
  // their sums are never stored, so every load is unconditional.
  for (uint32_t cb0 = 0; cb0 < CB; cb0 += MAC_CHUNK) {
    const uint32_t cb1 = cb0 + MAC_CHUNK < CB ? cb0 + MAC_CHUNK : CB;
    uint64_t a00[MT][RT], a01[MT][RT], a10[MT][RT], a11[MT][RT];
#pragma unroll
    for (int j = 0; j < MT; j++)
#pragma unroll
      for (int i = 0; i < RT; i++) a00[j][i] = a01[j][i] = a10[j][i] = a11[j][i] = 0;
    uint32_t cb = cb0;
    // MAC_DEPTH channel blocks per step: all their loads are issued before
    // the first product, so that many loads per thread are in flight
    for (; cb + MAC_DEPTH <= cb1; cb += MAC_DEPTH) {
      uint64_t xr[MAC_DEPTH][RT], wr[MAC_DEPTH][MT];
#pragma unroll
      for (int d = 0; d < MAC_DEPTH; d++) {
#pragma unroll
        for (int i = 0; i < RT; i++) xr[d][i] = ip[i][(uint64_t)(cb + d) * in_cb_stride];
#pragma unroll
        for (int j = 0; j < MT; j++) {
#ifdef HECONV_MAC_NT
          wr[d][j] = __builtin_nontemporal_load(&wp[j][(uint64_t)(cb + d) * LN]);
#else
          wr[d][j] = wp[j][(uint64_t)(cb + d) * LN];
#endif
        }
      }
#pragma unroll
      for (int d = 0; d < MAC_DEPTH; d++) mac_step<MT, RT>(xr[d], wr[d], a00, a01, a10, a11);
    }
    for (; cb < cb1; cb++) {
      uint64_t xr[RT], wr[MT];
#pragma unroll
      for (int i = 0; i < RT; i++) xr[i] = ip[i][(uint64_t)cb * in_cb_stride];
#pragma unroll
      for (int j = 0; j < MT; j++) wr[j] = wp[j][(uint64_t)cb * LN];
      mac_step<MT, RT>(xr, wr, a00, a01, a10, a11);
    }
#pragma unroll
    for (int j = 0; j < MT; j++)
#pragma unroll
      for (int i = 0; i < RT; i++)
        res[j][i] = csub(res[j][i] + fold30(a00[j][i], a01[j][i], a10[j][i], a11[j][i], c), c.q);
  }
#pragma unroll
  for (int j = 0; j < MT; j++)
#pragma unroll
    for (int i = 0; i < RT; i++)
      if (mv[j] && rv[i]) out[out_off[i] + (uint64_t)(mt * MT + j) * out_m_stride] = res[j][i];
}

}  // namespace heconv
