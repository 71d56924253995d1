// Weight packing and the channel-block multiply-accumulate (NTT domain).
#include "kernels.h"
#include "mac_impl.h"
#include "mac_grid.h"
#include "mac_stream.h"
#include "udiv.h"

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
// the streamed MAC's default tile for layers with at least 4 rows and output
// channels: 4 output channels x 4 rows
constexpr uint32_t MAC_STREAM_DEFAULT_MT = 4;

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

// Streamed MAC for one layer (mac_stream): one tile per workgroup, decoded
// from the block index with scalar divisions by invariant integers (udiv.h).
// Tiles are k-chunk-major; xcd_remap keeps the tiles of one k-chunk on one
// XCD.
struct MacDivs {
  UDiv chunk, rt, s;  // by n_mt * n_rt, by n_rt, by S
};

template <int MT, int RT, int P, bool PM>
__global__ __launch_bounds__(MAC_THREADS) void mac_stream_kernel(const uint64_t* __restrict__ in,
                                                                 const uint64_t* __restrict__ w,
                                                                 uint64_t* __restrict__ out, uint32_t CB, uint32_t S,
                                                                 uint32_t M, uint32_t L, uint32_t logN, uint32_t rows,
                                                                 uint32_t n_mt, uint32_t n_rt, MacDivs dv,
                                                                 const LimbConst* __restrict__ lcs) {
  __shared__ uint64_t lds[mac_dma_lds_words<MT, RT, MAC_THREADS, P>()];
  const uint32_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t kc = udiv(tile, dv.chunk), rem = tile - kc * (n_mt * n_rt);
  const uint32_t mt = udiv(rem, dv.rt), rt = rem - mt * n_rt;
  const uint32_t bs0 = rt * RT / 2, b0 = udiv(bs0, dv.s), s0 = bs0 - b0 * S;
  const MacOneSrc src{MacItem{0, kc, mt, rt, b0, s0},
                      BatchJob{const_cast<uint64_t*>(in), w, out, CB, S, M, rows, n_mt, n_rt}};
  mac_stream<MT, RT, MAC_THREADS, P, PM>(src, lcs, L, logN, lds, threadIdx.x);
}

template <int MT, int RT, int P, bool PM>
static hipError_t mac_stream_go(const uint64_t* in, const uint64_t* w, uint64_t* out, uint32_t CB, uint32_t S,
                                uint32_t M, uint32_t L, uint32_t N, uint32_t rows, const LimbConst* lc, hipStream_t st) {
  const uint32_t n_mt = (M + MT - 1) / MT, n_rt = (rows + RT - 1) / RT;
  const uint64_t blocks = (uint64_t)L * (N / MAC_THREADS) * n_mt * n_rt;
  if (blocks > grid_max_blocks(MAC_THREADS) || blocks >= (1ull << 31)) return hipErrorInvalidConfiguration;
  uint32_t logN = 0;
  while ((1u << logN) < N) logN++;
  const MacDivs dv{udiv_make(n_mt * n_rt), udiv_make(n_rt), udiv_make(S)};
  hipLaunchKernelGGL((mac_stream_kernel<MT, RT, P, PM>), dim3((uint32_t)blocks), dim3(MAC_THREADS), 0, st, in, w, out,
                     CB, S, M, L, logN, rows, n_mt, n_rt, dv, lc);
  return hipGetLastError();
}

template <int MT, int RT>
static hipError_t mac_stream_p(uint32_t P, bool pm, const uint64_t* in, const uint64_t* w, uint64_t* out, uint32_t CB,
                               uint32_t S, uint32_t M, uint32_t L, uint32_t N, uint32_t rows, const LimbConst* lc,
                               hipStream_t st) {
  if (pm) {
    if (P == 2) return mac_stream_go<MT, RT, 2, true>(in, w, out, CB, S, M, L, N, rows, lc, st);
    if (P == 3) return mac_stream_go<MT, RT, 3, true>(in, w, out, CB, S, M, L, N, rows, lc, st);
    return mac_stream_go<MT, RT, 4, true>(in, w, out, CB, S, M, L, N, rows, lc, st);
  }
  if (P == 2) return mac_stream_go<MT, RT, 2, false>(in, w, out, CB, S, M, L, N, rows, lc, st);
  if (P == 3) return mac_stream_go<MT, RT, 3, false>(in, w, out, CB, S, M, L, N, rows, lc, st);
  return mac_stream_go<MT, RT, 4, false>(in, w, out, CB, S, M, L, N, rows, lc, st);
}

// Streamed MAC on the 2x2 wave grid for one layer (mac_grid): one tile of
// 2*MT channels x 2*RT rows over 64 NTT points per workgroup, decoded from
// the block index as above (k-chunk-major, the tiles of one k-chunk on one
// XCD).
template <int MT, int RT, int P, bool PM>
__global__ __launch_bounds__(MAC_THREADS) void mac_grid_kernel(const uint64_t* __restrict__ in,
                                                               const uint64_t* __restrict__ w,
                                                               uint64_t* __restrict__ out, uint32_t CB, uint32_t S,
                                                               uint32_t M, uint32_t L, uint32_t logN, uint32_t rows,
                                                               uint32_t n_mt, uint32_t n_rt, MacDivs dv,
                                                               const LimbConst* __restrict__ lcs) {
  __shared__ uint64_t lds[P * MacGridShape<MT, RT>::ROWS * 64];
  const uint32_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t kc = udiv(tile, dv.chunk), rem = tile - kc * (n_mt * n_rt);
  const uint32_t mt = udiv(rem, dv.rt), rt = rem - mt * n_rt;
  const uint32_t bs0 = rt * RT, b0 = udiv(bs0, dv.s), s0 = bs0 - b0 * S;  // first row pair of the tile's 2*RT rows
  const MacOneSrc src{MacItem{0, kc, mt, rt, b0, s0},
                      BatchJob{const_cast<uint64_t*>(in), w, out, CB, S, M, rows, n_mt, n_rt}};
  mac_grid<MT, RT, MAC_THREADS, P, PM>(src, lcs, L, logN, lds, threadIdx.x);
}

template <int MT, int RT, int P, bool PM>
static hipError_t mac_grid_go(const uint64_t* in, const uint64_t* w, uint64_t* out, uint32_t CB, uint32_t S,
                              uint32_t M, uint32_t L, uint32_t N, uint32_t rows, const LimbConst* lc, hipStream_t st) {
  const uint32_t n_mt = (M + 2 * MT - 1) / (2 * MT), n_rt = (rows + 2 * RT - 1) / (2 * RT);
  const uint64_t blocks = (uint64_t)L * (N / 64) * n_mt * n_rt;
  if (blocks > grid_max_blocks(MAC_THREADS) || blocks >= (1ull << 31)) return hipErrorInvalidConfiguration;
  uint32_t logN = 0;
  while ((1u << logN) < N) logN++;
  const MacDivs dv{udiv_make(n_mt * n_rt), udiv_make(n_rt), udiv_make(S)};
  hipLaunchKernelGGL((mac_grid_kernel<MT, RT, P, PM>), dim3((uint32_t)blocks), dim3(MAC_THREADS), 0, st, in, w, out,
                     CB, S, M, L, logN, rows, n_mt, n_rt, dv, lc);
  return hipGetLastError();
}

template <int MT, int RT>
static hipError_t mac_grid_p(uint32_t P, bool pm, const uint64_t* in, const uint64_t* w, uint64_t* out, uint32_t CB,
                             uint32_t S, uint32_t M, uint32_t L, uint32_t N, uint32_t rows, const LimbConst* lc,
                             hipStream_t st) {
  if (pm) {
    if (P == 2) return mac_grid_go<MT, RT, 2, true>(in, w, out, CB, S, M, L, N, rows, lc, st);
    if (P == 3) return mac_grid_go<MT, RT, 3, true>(in, w, out, CB, S, M, L, N, rows, lc, st);
    return mac_grid_go<MT, RT, 4, true>(in, w, out, CB, S, M, L, N, rows, lc, st);
  }
  if (P == 2) return mac_grid_go<MT, RT, 2, false>(in, w, out, CB, S, M, L, N, rows, lc, st);
  if (P == 3) return mac_grid_go<MT, RT, 3, false>(in, w, out, CB, S, M, L, N, rows, lc, st);
  return mac_grid_go<MT, RT, 4, false>(in, w, out, CB, S, M, L, N, rows, lc, st);
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
                      uint32_t lds_stages, bool all_pm, bool grid, hipStream_t st) {
  const uint32_t rows = B * S * 2;
  const bool small = rows < 4 || M < 4;
  if (lds_stages >= 2 && mac_dma_fits(CB, L, N)) {
    // streamed: (4,4) (6,4) (4,2) (2,4) (2,2); others take the shape's default
    const bool ok = (mt == 4 && (rt == 4 || rt == 2)) || (mt == 6 && rt == 4) || (mt == 2 && (rt == 4 || rt == 2));
    if (!ok) mt = small ? 2 : MAC_STREAM_DEFAULT_MT, rt = small ? 2 : 4;
    if (grid && rows >= 2 * rt && M >= 2 * mt) {
#define HECONV_MAC_GRID(A, Bt) \
  if (mt == A && rt == Bt) return mac_grid_p<A, Bt>(lds_stages, all_pm, in, w, out, CB, S, M, L, N, rows, lc, st);
      HECONV_MAC_GRID(4, 4)
      HECONV_MAC_GRID(6, 4)
      HECONV_MAC_GRID(4, 2)
      HECONV_MAC_GRID(2, 4)
      HECONV_MAC_GRID(2, 2)
#undef HECONV_MAC_GRID
    }
#define HECONV_MAC_STREAM(A, Bt) \
  if (mt == A && rt == Bt) return mac_stream_p<A, Bt>(lds_stages, all_pm, in, w, out, CB, S, M, L, N, rows, lc, st);
    HECONV_MAC_STREAM(4, 4)
    HECONV_MAC_STREAM(6, 4)
    HECONV_MAC_STREAM(4, 2)
    HECONV_MAC_STREAM(2, 4)
    HECONV_MAC_STREAM(2, 2)
#undef HECONV_MAC_STREAM
    return hipErrorInvalidValue;
  }
  // register loads: (4,4) (4,2) (2,4) (8,2) (2,8) (8,1) (1,8) (2,2)
  const bool reg_ok = (mt == 4 && (rt == 4 || rt == 2)) || (mt == 2 && (rt == 4 || rt == 8 || rt == 2)) ||
                      (mt == 8 && (rt == 2 || rt == 1)) || (mt == 1 && rt == 8);
  if (!reg_ok) mt = rt = small ? 2 : 4;
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
