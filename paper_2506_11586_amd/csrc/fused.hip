// Fused multiply-accumulate + inverse NTT: one workgroup per output limb
// polynomial (b, m, s, c, l).  Its threads accumulate the channel-block sum
// of every NTT point in registers (30-bit split products, as in the MAC
// kernel), then inverse-transform the result in registers and LDS and store
// the coefficients.  The NTT-form output never goes to HBM, and the
// weight-streaming MAC of one workgroup overlaps the transform arithmetic of
// others on the same CU.
//
// Workgroups of the rows (b, s, c) that share one (m, l) -- and so read the
// same weight words -- are consecutive and, through the XCD remap, on the
// same XCD, so the weights are fetched from HBM about once.
#include "kernels.h"
#include "mac_impl.h"
#include "ntt_impl.h"

namespace heconv {

constexpr int FUSED_E = 16;     // NTT points per thread (the inverse NTT's 16-word passes)
constexpr int FUSED_G = 4;      // points accumulated per MAC pass
constexpr int FUSED_DEPTH = 2;  // channel blocks whose loads are issued together

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / FUSED_E, 4) void mac_intt_kernel(const uint64_t* __restrict__ in_,
                                                                          const uint64_t* __restrict__ w_,
                                                                          uint64_t* __restrict__ out_, uint32_t B,
                                                                          uint32_t CB, uint32_t S, uint32_t M,
                                                                          uint32_t L, const Tw* __restrict__ twi,
                                                                          const LimbConst* __restrict__ lcs) {
  constexpr int N = 1 << LOGN, E = FUSED_E, T = N / E, G = FUSED_G;
  __shared__ uint64_t lds[N + N / 16];
  cgword* in = as_global(in_);
  cgword* w = as_global(w_);
  gword* out = as_global(out_);
  const int tid = threadIdx.x;
  const uint32_t rows = B * S * 2;
  const uint32_t id = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t r = id % rows, ml = id / rows;
  const uint32_t l = ml % L, m = ml / L;
  const uint32_t comp = r & 1, bs = r >> 1, b = bs / S, s = bs % S;
  const uint64_t LN = (uint64_t)L * N;
  cgword* ip = in + ((((uint64_t)b * CB) * S + s) * 2 + comp) * LN + (uint64_t)l * N + tid;
  cgword* wp = w + ((uint64_t)m * CB) * LN + (uint64_t)l * N + tid;
  const uint64_t in_cb = (uint64_t)S * 2 * LN;  // cb -> cb+1 in the input
  const LimbConst c = lcs[l];

  uint64_t x[E];
#pragma unroll
  for (int g0 = 0; g0 < E; g0 += G) {
    uint64_t res[G];
#pragma unroll
    for (int e = 0; e < G; e++) res[e] = 0;
    for (uint32_t cb0 = 0; cb0 < CB; cb0 += MAC_CHUNK) {
      const uint32_t cb1 = cb0 + MAC_CHUNK < CB ? cb0 + MAC_CHUNK : CB;
      uint64_t a00[G], a01[G], a10[G], a11[G];
#pragma unroll
      for (int e = 0; e < G; e++) a00[e] = a01[e] = a10[e] = a11[e] = 0;
      uint32_t cb = cb0;
      for (; cb + FUSED_DEPTH <= cb1; cb += FUSED_DEPTH) {
        uint64_t xv[FUSED_DEPTH][G], wv[FUSED_DEPTH][G];
#pragma unroll
        for (int d = 0; d < FUSED_DEPTH; d++)
#pragma unroll
          for (int e = 0; e < G; e++) {
            xv[d][e] = ip[(uint64_t)(cb + d) * in_cb + (g0 + e) * T];
            wv[d][e] = wp[(uint64_t)(cb + d) * LN + (g0 + e) * T];
          }
#pragma unroll
        for (int d = 0; d < FUSED_DEPTH; d++)
#pragma unroll
          for (int e = 0; e < G; e++) {
            const Half30 xs = split30(xv[d][e]), ws = split30(wv[d][e]);
            a00[e] += (uint64_t)xs.lo * ws.lo;
            a01[e] += (uint64_t)xs.lo * ws.hi;
            a10[e] += (uint64_t)xs.hi * ws.lo;
            a11[e] += (uint64_t)xs.hi * ws.hi;
          }
      }
      for (; cb < cb1; cb++) {
#pragma unroll
        for (int e = 0; e < G; e++) {
          const Half30 xs = split30(ip[(uint64_t)cb * in_cb + (g0 + e) * T]);
          const Half30 ws = split30(wp[(uint64_t)cb * LN + (g0 + e) * T]);
          a00[e] += (uint64_t)xs.lo * ws.lo;
          a01[e] += (uint64_t)xs.lo * ws.hi;
          a10[e] += (uint64_t)xs.hi * ws.lo;
          a11[e] += (uint64_t)xs.hi * ws.hi;
        }
      }
#pragma unroll
      for (int e = 0; e < G; e++) res[e] = csub(res[e] + fold30(a00[e], a01[e], a10[e], a11[e], c), c.q);
    }
#pragma unroll
    for (int e = 0; e < G; e++) x[g0 + e] = res[e];
  }
  // x holds the NTT-form output in the top mapping (point tid + k*T)
  ntt_inv_regs<LOGN, 4>(x, twi + (size_t)l * N, c, lds, tid);
  gword* op = out + ((((uint64_t)b * M + m) * S + s) * 2 + comp) * LN + (uint64_t)l * N + tid;
#pragma unroll
  for (int k = 0; k < E; k++) op[k * T] = x[k];
}

template <int LOGN>
static hipError_t go(const uint64_t* in, const uint64_t* w, uint64_t* out, uint32_t B, uint32_t CB, uint32_t S,
                     uint32_t M, uint32_t L, const Tw* twi, const LimbConst* lc, hipStream_t st) {
  const uint64_t blocks = (uint64_t)B * S * 2 * M * L;
  if (blocks > grid_max_blocks((1u << LOGN) / FUSED_E)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((mac_intt_kernel<LOGN>), dim3((uint32_t)blocks), dim3((1 << LOGN) / FUSED_E), 0, st,
                     in, w, out, B, CB, S, M, L, twi, lc);
  return hipGetLastError();
}

hipError_t mac_intt_launch(uint32_t logN, const uint64_t* in, const uint64_t* w, uint64_t* out, uint32_t B,
                           uint32_t CB, uint32_t S, uint32_t M, uint32_t L, const Tw* twi, const LimbConst* lc,
                           hipStream_t st) {
  switch (logN) {
    case 10: return go<10>(in, w, out, B, CB, S, M, L, twi, lc, st);
    case 11: return go<11>(in, w, out, B, CB, S, M, L, twi, lc, st);
    case 12: return go<12>(in, w, out, B, CB, S, M, L, twi, lc, st);
    case 13: return go<13>(in, w, out, B, CB, S, M, L, twi, lc, st);
    case 14: return go<14>(in, w, out, B, CB, S, M, L, twi, lc, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace heconv
