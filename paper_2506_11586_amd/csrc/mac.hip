// Weight packing and the channel-block multiply-accumulate (NTT domain).
#include "kernels.h"

namespace heconv {

// ---------------------------------------------------------------------------
// Kernel-polynomial packing (offline).  Each thread writes one coefficient
// k of (m, cb, l): with d = O - k, the coefficient holds K[m][cb*Cw+cc][i][j]
// when d = cc*Hw*Ww + i*Ww + j with cc < Cw, i < kh, j < kw and the channel
// exists, and 0 otherwise.  Signed values are lifted into [0, q_l).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pack_weights_kernel(PackGeom g, const int64_t* __restrict__ w,
                                                           uint64_t* __restrict__ out,
                                                           const LimbConst* __restrict__ lcs) {
  const uint64_t total = (uint64_t)g.M * g.CB * g.L * g.N;
  const uint32_t HW = g.Hw * g.Ww;
  for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t k = (uint32_t)(idx % g.N);
    uint64_t r = idx / g.N;
    const uint32_t l = (uint32_t)(r % g.L);
    r /= g.L;
    const uint32_t cb = (uint32_t)(r % g.CB);
    const uint32_t m = (uint32_t)(r / g.CB);
    uint64_t v = 0;
    if (k <= g.O) {
      const uint32_t d = g.O - k;
      const uint32_t cc = d / HW, rem = d % HW;
      const uint32_t i = rem / g.Ww, j = rem % g.Ww;
      const uint32_t c = cb * g.Cw + cc;
      if (cc < g.Cw && c < g.C && i < g.kh && j < g.kw) {
        const int64_t s = w[(((uint64_t)m * g.C + c) * g.kh + i) * g.kw + j];
        const uint64_t q = lcs[l].q;
        if (s >= 0) {
          v = (uint64_t)s % q;
        } else {
          const uint64_t a = (uint64_t)0 - (uint64_t)s;  // |s|, exact also for INT64_MIN
          const uint64_t am = a % q;
          v = am ? q - am : 0;
        }
      }
    }
    out[idx] = v;
  }
}

hipError_t pack_weights_launch(const PackGeom& g, const int64_t* w, uint64_t* out, const LimbConst* lc,
                               hipStream_t st) {
  const uint64_t total = (uint64_t)g.M * g.CB * g.L * g.N;
  uint64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(pack_weights_kernel, dim3((uint32_t)blocks), dim3(256), 0, st, g, w, out, lc);
  return hipGetLastError();
}

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
constexpr int MAC_THREADS = 256;
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

constexpr int MAC_DEPTH = 4;

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

template <int MT, int RT>
__global__ __launch_bounds__(MAC_THREADS) void mac_kernel(const uint64_t* __restrict__ in,
                                                          const uint64_t* __restrict__ w,
                                                          uint64_t* __restrict__ out, uint32_t CB, uint32_t S,
                                                          uint32_t M, uint32_t L, uint32_t N, uint32_t rows,
                                                          uint32_t n_mt, uint32_t n_rt,
                                                          const LimbConst* __restrict__ lcs) {
  const uint32_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t per_chunk = n_mt * n_rt;
  const uint32_t kc = tile / per_chunk;
  const uint32_t mt = (tile % per_chunk) / n_rt;
  const uint32_t rt = tile % n_rt;
  const uint32_t chunks_per_limb = N / MAC_THREADS;
  const uint32_t l = kc / chunks_per_limb;
  const uint32_t k = (kc % chunks_per_limb) * MAC_THREADS + threadIdx.x;
  const LimbConst c = lcs[l];
  const uint64_t LN = (uint64_t)L * N;

  // row r = (b*S + s)*2 + comp; input address of (r, cb) and output of (r, m)
  const uint64_t* ip[RT];
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
  const uint64_t* wp[MT];
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
        for (int j = 0; j < MT; j++) wr[d][j] = wp[j][(uint64_t)(cb + d) * LN];
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

template <int MT, int RT>
static hipError_t mac_go(const uint64_t* in, const uint64_t* w, uint64_t* out, uint32_t CB, uint32_t S, uint32_t M,
                         uint32_t L, uint32_t N, uint32_t rows, const LimbConst* lc, hipStream_t st) {
  const uint32_t n_mt = (M + MT - 1) / MT, n_rt = (rows + RT - 1) / RT;
  const uint64_t blocks = (uint64_t)L * (N / MAC_THREADS) * n_mt * n_rt;
  if (blocks > 0x7fffffffull) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((mac_kernel<MT, RT>), dim3((uint32_t)blocks), dim3(MAC_THREADS), 0, st, in, w, out, CB, S, M,
                     L, N, rows, n_mt, n_rt, lc);
  return hipGetLastError();
}

hipError_t mac_launch(const uint64_t* in, const uint64_t* w, uint64_t* out, uint32_t B, uint32_t CB, uint32_t S,
                      uint32_t M, uint32_t L, uint32_t N, const LimbConst* lc, uint32_t mt, uint32_t rt,
                      hipStream_t st) {
  const uint32_t rows = B * S * 2;
  if (mt == 0 || rt == 0) {  // default tile by shape
    if (rows >= 4 && M >= 4) mt = 4, rt = 4;
    else mt = 2, rt = 2;
  }
#define HECONV_MAC_TILE(A, Bt) \
  if (mt == A && rt == Bt) return mac_go<A, Bt>(in, w, out, CB, S, M, L, N, rows, lc, st);
  HECONV_MAC_TILE(4, 4)
  HECONV_MAC_TILE(4, 2)
  HECONV_MAC_TILE(2, 4)
  HECONV_MAC_TILE(8, 2)
  HECONV_MAC_TILE(2, 8)
  HECONV_MAC_TILE(8, 1)
  HECONV_MAC_TILE(1, 8)
  HECONV_MAC_TILE(2, 2)
#undef HECONV_MAC_TILE
  return hipErrorInvalidValue;
}

}  // namespace heconv
