// The Z_P variant's plaintext side and linear kernel (Sec. 6.1: its kernels
// multiply the input by NTT-preprocessed weights, accumulate, and rotate the
// accumulated result once per iteration).
//
// Slots: with t prime, t = 1 mod 2N, a plaintext m in Z_t[X]/(X^N+1) holds
// in slot s the value m(zeta^e_s), e_s = 5^j mod 2N in row 0 and -5^j mod 2N
// in row 1 (s = r*N/2 + j).  The forward NTT over t evaluates at
// psi^(2 brv(i) + 1) at index i, so slot s is NTT index brv((e_s - 1)/2):
// encoding scatters the slots to those indexes and runs the inverse NTT of
// a one-prime context over t; decoding runs the forward NTT and gathers.
// X -> X^5 then moves every row left by one slot.
//
// Diagonals: for an n x n matrix (n a power of two dividing N/2), diagonal i
// holds W[(k - i) mod n][k mod n] in slot k of each row; with the input x
// repeated with period n, sum_i rot^i(d_i * x) = W x, computed as
// acc = x*d_{n-1}, then acc = rot(acc) + x*d_i for i = n-2 .. 0.
#include "kernels.h"

namespace heconv {

constexpr uint32_t ZP_THREADS = 256;

// NTT index of slot s (N = 2^logN).
__device__ __forceinline__ uint32_t slot_index(uint32_t s, uint32_t logN) {
  const uint32_t N = 1u << logN, h = N >> 1, m2 = 2 * N - 1;
  uint32_t j = s & (h - 1), p = 1, b = 5;
  for (; j; j >>= 1, b = (b * b) & m2)
    if (j & 1) p = (p * b) & m2;
  const uint32_t e = s < h ? p : (2 * N - p) & m2;
  return __brev((e - 1) >> 1) >> (32 - logN);
}

// encode: out[i][slot_index(s)] = in[i][s]; decode: out[i][s] = in[i][slot_index(s)]
__global__ __launch_bounds__(ZP_THREADS) void slot_permute_kernel(const uint64_t* __restrict__ in,
                                                                   uint64_t* __restrict__ out, uint32_t logN,
                                                                   int encode) {
  const uint32_t N = 1u << logN;
  const uint64_t i = blockIdx.y;
  const uint32_t s = blockIdx.x * ZP_THREADS + threadIdx.x;
  if (s >= N) return;
  const uint32_t k = slot_index(s, logN);
  if (encode)
    out[i * N + k] = in[i * N + s];
  else
    out[i * N + s] = in[i * N + k];
}

// v in [0, t) -> v - t when 2v >= t (the centred representative)
__global__ __launch_bounds__(ZP_THREADS) void centre_kernel(uint64_t* __restrict__ v, uint64_t words, uint64_t t) {
  const uint64_t idx = (uint64_t)blockIdx.x * ZP_THREADS + threadIdx.x;
  if (idx >= words) return;
  const uint64_t x = v[idx];
  v[idx] = 2 * x >= t ? x - t : x;  // as int64: x - t wraps to the negative value
}

// int64 -> [0, t)
__global__ __launch_bounds__(ZP_THREADS) void reduce_t_kernel(const int64_t* __restrict__ in,
                                                               uint64_t* __restrict__ out, uint64_t words,
                                                               LimbConst tc) {
  const uint64_t idx = (uint64_t)blockIdx.x * ZP_THREADS + threadIdx.x;
  if (idx >= words) return;
  const int64_t v = in[idx];
  const uint64_t mag = v < 0 ? 0ull - (uint64_t)v : (uint64_t)v;
  const uint64_t r = csub(csub(reduce64_lazy(mag, tc.mu64, tc.q), tc.two_q), tc.q);
  out[idx] = v < 0 && r ? tc.q - r : r;
}

// slots[i][r*N/2 + j] = W[(k - i) mod n_out][k] mod t with k = j mod n_in
// (zero outside rows x cols), for i < n_out, both rows r.  n_out = n_in is
// the square layout; n_out < n_in the generalized diagonals of a matrix
// with fewer rows than columns.
__global__ __launch_bounds__(ZP_THREADS) void diagonals_kernel(const int64_t* __restrict__ W, uint32_t rows,
                                                                uint32_t cols, uint32_t n_out, uint32_t n_in,
                                                                uint32_t N, uint64_t* __restrict__ slots,
                                                                LimbConst tc) {
  const uint64_t i = blockIdx.y;
  const uint32_t s = blockIdx.x * ZP_THREADS + threadIdx.x;
  if (s >= N) return;
  const uint32_t k = s & (n_in - 1);
  const uint32_t r = (uint32_t)((k + n_out - (uint32_t)i) & (n_out - 1));
  uint64_t v = 0;
  if (r < rows && k < cols) {
    const int64_t w = W[(uint64_t)r * cols + k];
    const uint64_t mag = w < 0 ? 0ull - (uint64_t)w : (uint64_t)w;
    const uint64_t red = csub(csub(reduce64_lazy(mag, tc.mu64, tc.q), tc.two_q), tc.q);
    v = w < 0 && red ? tc.q - red : red;
  }
  slots[i * N + s] = v;
}

// out[i][l][k] = (c[i][k] mod q_l) * scale_l mod q_l: a plaintext with
// integer coefficients lifted to every ciphertext modulus and multiplied by
// scale_l (-P mod q_l) before its transform.
__global__ __launch_bounds__(ZP_THREADS) void lift_scaled_kernel(const int64_t* __restrict__ c,
                                                                  uint64_t* __restrict__ out, uint32_t N, uint32_t L,
                                                                  ScaleConst sc,
                                                                  const LimbConst* __restrict__ lcs) {
  const uint64_t i = blockIdx.y;
  const uint32_t j = blockIdx.x * ZP_THREADS + threadIdx.x;
  if (j >= L * N) return;
  const uint32_t l = j / N, k = j % N;
  const LimbConst q = lcs[l];
  const int64_t v = c[i * N + k];
  const uint64_t mag = v < 0 ? 0ull - (uint64_t)v : (uint64_t)v;
  const uint64_t r = csub(reduce64_lazy(mag, q.mu64, q.q), q.q);
  const uint64_t lifted = v < 0 && r ? q.q - r : r;
  out[i * L * N + j] = csub(mul_shoup_lazy(lifted, sc.v[l], sc.sh[l], q.q), q.q);
}

static dim3 zp_grid(uint64_t words, uint64_t n) {
  return dim3((uint32_t)((words + ZP_THREADS - 1) / ZP_THREADS), (uint32_t)n);
}

hipError_t slot_permute_launch(const uint64_t* in, uint64_t* out, uint64_t n, uint32_t logN, bool encode,
                               hipStream_t st) {
  if (!n) return hipSuccess;
  if (n > 65535) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(slot_permute_kernel, zp_grid(1u << logN, n), dim3(ZP_THREADS), 0, st, in, out, logN,
                     encode ? 1 : 0);
  return hipGetLastError();
}

hipError_t centre_launch(uint64_t* v, uint64_t words, uint64_t t, hipStream_t st) {
  if (!words) return hipSuccess;
  hipLaunchKernelGGL(centre_kernel, dim3((uint32_t)((words + ZP_THREADS - 1) / ZP_THREADS)), dim3(ZP_THREADS), 0,
                     st, v, words, t);
  return hipGetLastError();
}

hipError_t reduce_t_launch(const int64_t* in, uint64_t* out, uint64_t words, const LimbConst& tc, hipStream_t st) {
  if (!words) return hipSuccess;
  hipLaunchKernelGGL(reduce_t_kernel, dim3((uint32_t)((words + ZP_THREADS - 1) / ZP_THREADS)), dim3(ZP_THREADS), 0,
                     st, in, out, words, tc);
  return hipGetLastError();
}

hipError_t diagonals_launch(const int64_t* W, uint32_t rows, uint32_t cols, uint32_t n_out, uint32_t n_in, uint32_t N,
                            uint64_t* slots, const LimbConst& tc, hipStream_t st) {
  if (n_out > 65535) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(diagonals_kernel, zp_grid(N, n_out), dim3(ZP_THREADS), 0, st, W, rows, cols, n_out, n_in, N,
                     slots, tc);
  return hipGetLastError();
}

hipError_t lift_scaled_launch(const int64_t* c, uint64_t* out, uint64_t n, uint32_t N, uint32_t L,
                              const ScaleConst& sc, const LimbConst* lc, hipStream_t st) {
  if (!n) return hipSuccess;
  if (n > 65535) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(lift_scaled_kernel, zp_grid((uint64_t)L * N, n), dim3(ZP_THREADS), 0, st, c, out, N, L, sc,
                     lc);
  return hipGetLastError();
}

}  // namespace heconv
