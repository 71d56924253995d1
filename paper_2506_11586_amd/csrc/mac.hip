// Weight packing and the channel-block multiply-accumulate (NTT domain).
#include "kernels.h"
#include "mac_impl.h"

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
// Standalone MAC kernel: one workgroup of MAC_THREADS threads per tile; the
// tile itself is in mac_impl.h.
// ---------------------------------------------------------------------------
constexpr int MAC_THREADS = 256;

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
  const LimbConst c = lcs[kc / (N / MAC_THREADS)];
  mac_tile<MT, RT, MAC_THREADS>(as_global(in), as_global(w), as_global(out), CB, S, M, L, N, rows, kc, mt, rt, c, threadIdx.x);
}

// (Bounding the 4x4 tile to three workgroups per compute unit, 168 VGPRs,
// spills part of the fold and measured slower: 128.6 against 121.1 ms on the
// 16-image bottleneck CNN's MAC grid, 69.7 against 57.0 us on the 64->64
// layer's MAC with the caches flushed.)
template <int MT, int RT, int P>
__global__ __launch_bounds__(MAC_THREADS) void mac_dma_kernel(const uint64_t* __restrict__ in,
                                                              const uint64_t* __restrict__ w,
                                                              uint64_t* __restrict__ out, uint32_t CB, uint32_t S,
                                                              uint32_t M, uint32_t L, uint32_t N, uint32_t rows,
                                                              uint32_t n_mt, uint32_t n_rt,
                                                              const LimbConst* __restrict__ lcs) {
  __shared__ uint64_t lds[mac_dma_lds_words<MT, RT, MAC_THREADS, P>()];
  const uint32_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t per_chunk = n_mt * n_rt;
  const uint32_t kc = tile / per_chunk;
  const uint32_t mt = (tile % per_chunk) / n_rt;
  const uint32_t rt = tile % n_rt;
  const LimbConst c = lcs[kc / (N / MAC_THREADS)];
  mac_tile_dma<MT, RT, MAC_THREADS, P>(as_global(in), as_global(w), as_global(out), CB, S, M, L, N, rows, kc, mt, rt,
                                       c, threadIdx.x, lds);
}

template <int MT, int RT, int P>
static hipError_t mac_dma_go(const uint64_t* in, const uint64_t* w, uint64_t* out, uint32_t CB, uint32_t S, uint32_t M,
                             uint32_t L, uint32_t N, uint32_t rows, const LimbConst* lc, hipStream_t st) {
  const uint32_t n_mt = (M + MT - 1) / MT, n_rt = (rows + RT - 1) / RT;
  const uint64_t blocks = (uint64_t)L * (N / MAC_THREADS) * n_mt * n_rt;
  if (blocks > grid_max_blocks(MAC_THREADS)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((mac_dma_kernel<MT, RT, P>), dim3((uint32_t)blocks), dim3(MAC_THREADS), 0, st, in, w, out, CB, S,
                     M, L, N, rows, n_mt, n_rt, lc);
  return hipGetLastError();
}

template <int MT, int RT>
static hipError_t mac_dma_p(uint32_t P, const uint64_t* in, const uint64_t* w, uint64_t* out, uint32_t CB, uint32_t S,
                            uint32_t M, uint32_t L, uint32_t N, uint32_t rows, const LimbConst* lc, hipStream_t st) {
  if (P == 2) return mac_dma_go<MT, RT, 2>(in, w, out, CB, S, M, L, N, rows, lc, st);
  if (P == 3) return mac_dma_go<MT, RT, 3>(in, w, out, CB, S, M, L, N, rows, lc, st);
  return mac_dma_go<MT, RT, 4>(in, w, out, CB, S, M, L, N, rows, lc, st);
}

template <int MT, int RT>
static hipError_t mac_go(const uint64_t* in, const uint64_t* w, uint64_t* out, uint32_t CB, uint32_t S, uint32_t M,
                         uint32_t L, uint32_t N, uint32_t rows, const LimbConst* lc, hipStream_t st) {
  const uint32_t n_mt = (M + MT - 1) / MT, n_rt = (rows + RT - 1) / RT;
  const uint64_t blocks = (uint64_t)L * (N / MAC_THREADS) * n_mt * n_rt;
  if (blocks > grid_max_blocks(MAC_THREADS)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((mac_kernel<MT, RT>), dim3((uint32_t)blocks), dim3(MAC_THREADS), 0, st, in, w, out, CB, S, M,
                     L, N, rows, n_mt, n_rt, lc);
  return hipGetLastError();
}

hipError_t mac_launch(const uint64_t* in, const uint64_t* w, uint64_t* out, uint32_t B, uint32_t CB, uint32_t S,
                      uint32_t M, uint32_t L, uint32_t N, const LimbConst* lc, uint32_t mt, uint32_t rt,
                      uint32_t lds_stages, hipStream_t st) {
  const uint32_t rows = B * S * 2;
  if ((mt == 6 || mt == 8 || mt == 4) && rt == (mt == 4 ? 8u : 4u)) mt = rt = 0;  // batch-only tiles
  if (mt == 0 || rt == 0) {  // default tile by shape
    if (rows >= 4 && M >= 4) mt = 4, rt = 4;
    else mt = 2, rt = 2;
  }
  if (lds_stages >= 2 && mac_dma_fits(CB, L, N)) {
#define HECONV_MAC_DMA(A, Bt) \
  if (mt == A && rt == Bt) return mac_dma_p<A, Bt>(lds_stages, in, w, out, CB, S, M, L, N, rows, lc, st);
    HECONV_MAC_DMA(4, 4)
    HECONV_MAC_DMA(4, 2)
    HECONV_MAC_DMA(2, 4)
    HECONV_MAC_DMA(2, 2)
#undef HECONV_MAC_DMA
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
