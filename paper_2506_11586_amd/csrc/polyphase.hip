// Polyphase form of a strided convolution: a stride-s conv equals a
// stride-1, pad-0 conv on s*s*C phase channels of the padded input with a
// ceil(k/s) kernel (the same outputs, first Ho x Wo of them).  With
// u = s*i + a and v = s*j + b, xpad[c][s*y + u][s*x + v] = X_(c,a,b)[y + i][x + j].
// These kernels rearrange the integer weights (offline) and int64 inputs
// (the server's input share); the layer itself is the library's ordinary
// stride-1 layer on the polyphase descriptor.
#include "kernels.h"

namespace heconv {

constexpr uint32_t PP_THREADS = 256;

// Kp[m][c*s*s + a*s + b][i][j] = K[m][c][s*i + a][s*j + b], zero where the
// source lies outside the kh x kw kernel.
__global__ __launch_bounds__(PP_THREADS) void polyphase_weights_kernel(const int64_t* __restrict__ K,
                                                                        int64_t* __restrict__ Kp, PolyGeom g) {
  const uint64_t idx = (uint64_t)blockIdx.x * PP_THREADS + threadIdx.x;
  const uint64_t total = (uint64_t)g.M * g.Cp * g.khp * g.kwp;
  if (idx >= total) return;
  const uint32_t j = (uint32_t)(idx % g.kwp);
  const uint32_t i = (uint32_t)((idx / g.kwp) % g.khp);
  const uint32_t cp = (uint32_t)((idx / ((uint64_t)g.kwp * g.khp)) % g.Cp);
  const uint64_t m = idx / ((uint64_t)g.kwp * g.khp * g.Cp);
  const uint32_t s2 = g.s * g.s, c = cp / s2, a = (cp % s2) / g.s, b = cp % g.s;
  const uint32_t u = g.s * i + a, v = g.s * j + b;
  Kp[idx] = u < g.kh && v < g.kw ? K[((m * g.C + c) * g.kh + u) * g.kw + v] : 0;
}

// X[n][c*s*s + a*s + b][y][x] = x[n][c][s*y + a - pad][s*x + b - pad], zero
// outside the input.
__global__ __launch_bounds__(PP_THREADS) void polyphase_input_kernel(const int64_t* __restrict__ x,
                                                                      int64_t* __restrict__ X, PolyGeom g,
                                                                      uint64_t total) {
  const uint64_t idx = (uint64_t)blockIdx.x * PP_THREADS + threadIdx.x;
  if (idx >= total) return;
  const uint32_t xx = (uint32_t)(idx % g.Wp);
  const uint32_t yy = (uint32_t)((idx / g.Wp) % g.Hp);
  const uint32_t cp = (uint32_t)((idx / ((uint64_t)g.Wp * g.Hp)) % g.Cp);
  const uint64_t n = idx / ((uint64_t)g.Wp * g.Hp * g.Cp);
  const uint32_t s2 = g.s * g.s, c = cp / s2, a = (cp % s2) / g.s, b = cp % g.s;
  const int64_t r = (int64_t)g.s * yy + a - g.pad, col = (int64_t)g.s * xx + b - g.pad;
  X[idx] = r >= 0 && r < g.H && col >= 0 && col < g.W ? x[((n * g.C + c) * g.H + r) * g.W + col] : 0;
}

hipError_t polyphase_weights_launch(const int64_t* K, int64_t* Kp, const PolyGeom& g, hipStream_t st) {
  const uint64_t total = (uint64_t)g.M * g.Cp * g.khp * g.kwp;
  const uint64_t blocks = (total + PP_THREADS - 1) / PP_THREADS;
  if (blocks > grid_max_blocks(PP_THREADS)) return hipErrorInvalidConfiguration;
  if (!blocks) return hipSuccess;
  hipLaunchKernelGGL(polyphase_weights_kernel, dim3((uint32_t)blocks), dim3(PP_THREADS), 0, st, K, Kp, g);
  return hipGetLastError();
}

hipError_t polyphase_input_launch(const int64_t* x, int64_t* X, const PolyGeom& g, uint64_t B, hipStream_t st) {
  const uint64_t total = B * g.Cp * g.Hp * g.Wp;
  const uint64_t blocks = (total + PP_THREADS - 1) / PP_THREADS;
  if (blocks > grid_max_blocks(PP_THREADS)) return hipErrorInvalidConfiguration;
  if (!blocks) return hipSuccess;
  hipLaunchKernelGGL(polyphase_input_kernel, dim3((uint32_t)blocks), dim3(PP_THREADS), 0, st, x, X, g, total);
  return hipGetLastError();
}

}  // namespace heconv
