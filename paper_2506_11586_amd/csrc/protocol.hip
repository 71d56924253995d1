// The server's steps either side of the layer in the online protocol for a
// linear layer (Sec. 7; extraction of the sparse results, Sec. 6.2):
//   add_share:    b_l += delta_l * pack(share) mod q_l on the client's input
//                 ciphertexts (coefficient form), before the forward NTT;
//   mask_extract: after the inverse NTT, gather only the b coefficients that
//                 hold outputs, minus delta_l * mask, plus a signed smudging
//                 term, into a dense [B][M][L][Ho][Wo] array.
// Both are elementwise and HBM/latency bound: one thread per coefficient
// (add_share) or per output value (mask_extract), consecutive threads on
// consecutive words.
#include "kernels.h"

namespace heconv {

constexpr uint32_t PROTO_THREADS = 256;

// v mod t in [0, t) for a signed value (t <= 2^62).
__device__ __forceinline__ uint64_t mod_t(int64_t v, uint64_t t) {
  int64_t r = v % (int64_t)t;
  return (uint64_t)(r < 0 ? r + (int64_t)t : r);
}

// v mod q in [0, q) for a signed value, via the Shoup reduction by 1.
__device__ __forceinline__ uint64_t mod_q_signed(int64_t v, const LimbConst& c) {
  const uint64_t mag = v < 0 ? 0ull - (uint64_t)v : (uint64_t)v;
  const uint64_t r = csub(reduce64_lazy(mag, c.mu64, c.q), c.q);
  return v < 0 && r ? c.q - r : r;
}

__global__ __launch_bounds__(PROTO_THREADS) void add_share_kernel(uint64_t* __restrict__ in_,
                                                                  const int64_t* __restrict__ share, ProtoGeom g,
                                                                  const LimbConst* __restrict__ lcs) {
  gword* in = as_global(in_);
  const uint32_t per_ct = g.N / PROTO_THREADS;
  const uint32_t ct = blockIdx.x / per_ct;  // (b, cb, s)
  const uint32_t k = (blockIdx.x % per_ct) * PROTO_THREADS + threadIdx.x;
  const uint32_t s = ct % g.S, cb = (ct / g.S) % g.CB, b = ct / (g.S * g.CB);
  // packed position -> padded (and, for a strided 1x1 conv, subsampled) input
  const uint32_t HW = g.Hw * g.Ww;
  const uint32_t cc = k / HW, rem = k - cc * HW, i = rem / g.Ww, j = rem - i * g.Ww;
  const uint32_t c = cb * g.Cw + cc;
  const uint32_t si = s / g.nsj, sj = s - si * g.nsj;
  const uint32_t pr = si * g.bh + i, pc = sj * g.bw + j;
  uint64_t m = 0;
  if (cc < g.Cw && c < g.C && pr < g.He && pc < g.We) {
    const int64_t y = (int64_t)pr * g.step - g.pad, x = (int64_t)pc * g.step - g.pad;
    if (y >= 0 && y < g.H && x >= 0 && x < g.W)
      m = mod_t(share[(((uint64_t)b * g.C + c) * g.H + y) * g.W + x], g.t);
  }
  gword* bp = in + ((uint64_t)ct * 2 + 1) * g.L * g.N + k;
  for (uint32_t l = 0; l < g.L; l++) {
    const LimbConst lc = lcs[l];
    const uint64_t d = csub(mul_shoup_lazy(m, lc.delta, lc.delta_sh, lc.q), lc.q);
    bp[(uint64_t)l * g.N] = csub(bp[(uint64_t)l * g.N] + d, lc.q);
  }
}

__global__ __launch_bounds__(PROTO_THREADS) void mask_extract_kernel(const uint64_t* __restrict__ out_,
                                                                     const int64_t* __restrict__ mask,
                                                                     const int64_t* __restrict__ noise,
                                                                     uint64_t* __restrict__ y_, ProtoGeom g,
                                                                     const LimbConst* __restrict__ lcs) {
  cgword* out = as_global(out_);
  gword* y = as_global(y_);
  const uint32_t HoWo = g.Ho * g.Wo;
  const uint32_t per_row = (HoWo + PROTO_THREADS - 1) / PROTO_THREADS;
  const uint32_t row = blockIdx.x / per_row;  // (b, m, l)
  const uint32_t pos = (blockIdx.x % per_row) * PROTO_THREADS + threadIdx.x;
  if (pos >= HoWo) return;
  const uint32_t l = row % g.L, bm = row / g.L;
  const uint32_t oy = pos / g.Wo, ox = pos - oy * g.Wo;
  const uint32_t r = oy * g.ostep, cl = ox * g.ostep;  // stride-1 output position
  const uint32_t si = r / g.bh, i = r - si * g.bh, sj = cl / g.bw, j = cl - sj * g.bw;
  const uint32_t s = si * g.nsj + sj, k = g.O + i * g.Ww + j;
  const LimbConst lc = lcs[l];
  const uint64_t word = out[(((uint64_t)bm * g.S + s) * 2 + 1) * g.L * g.N + (uint64_t)l * g.N + k];
  const uint64_t slot = (uint64_t)bm * HoWo + pos;
  const uint64_t dm = csub(mul_shoup_lazy(mod_t(mask[slot], g.t), lc.delta, lc.delta_sh, lc.q), lc.q);
  uint64_t v = csub(word + (lc.q - dm), lc.q);
  if (noise) v = csub(v + mod_q_signed(noise[slot], lc), lc.q);
  y[(uint64_t)row * HoWo + pos] = v;
}

hipError_t add_share_launch(uint64_t* in, const int64_t* share, const ProtoGeom& g, const LimbConst* lc,
                            hipStream_t st) {
  const uint64_t blocks = (uint64_t)g.B * g.CB * g.S * (g.N / PROTO_THREADS);
  if (blocks == 0) return hipSuccess;
  if (blocks > grid_max_blocks(PROTO_THREADS)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(add_share_kernel, dim3((uint32_t)blocks), dim3(PROTO_THREADS), 0, st, in, share, g, lc);
  return hipGetLastError();
}

hipError_t mask_extract_launch(const uint64_t* out, const int64_t* mask, const int64_t* noise, uint64_t* y,
                               const ProtoGeom& g, const LimbConst* lc, hipStream_t st) {
  const uint64_t per_row = ((uint64_t)g.Ho * g.Wo + PROTO_THREADS - 1) / PROTO_THREADS;
  const uint64_t blocks = (uint64_t)g.B * g.M * g.L * per_row;
  if (blocks == 0) return hipSuccess;
  if (blocks > grid_max_blocks(PROTO_THREADS)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(mask_extract_kernel, dim3((uint32_t)blocks), dim3(PROTO_THREADS), 0, st, out, mask, noise, y,
                     g, lc);
  return hipGetLastError();
}

}  // namespace heconv
