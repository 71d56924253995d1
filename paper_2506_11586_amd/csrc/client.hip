// Client-side BFV steps on the GPU, for load generation and for checking
// results (App. C: encryption b = a*sk + delta*m + e, decryption by
// b - a*sk and rounding t*V/Q).  The server path never calls these; they
// hold the secret key.  The products a*sk go through the transforms of
// ntt.hip: a copy of a is transformed, multiplied point by point by the
// transformed key, and transformed back, in a caller-provided work buffer.
//
// Decoding without a big-integer CRT: with Qh_l = Q/q_l and
// y_l = Qh_l^-1 mod q_l, t*V/Q = sum_l v_l * t*y_l/q_l - t*k for an
// integer k, so m = round(sum_l v_l * (I_l + F_l)) mod t with
// I_l = floor(t*y_l/q_l) and F_l its fraction.  F_l is held as a 128-bit
// fixed-point fraction (truncation error below L * 2^60 * 2^-128 in total);
// the integer part is summed in 128 bits and reduced mod t at the end, so t
// may be any modulus below 2^62 (a power of two or a prime).
#include "kernels.h"

namespace heconv {

constexpr uint32_t CLIENT_THREADS = 256;

__device__ __forceinline__ uint64_t mod_q_signed_c(int64_t v, const LimbConst& c) {
  const uint64_t mag = v < 0 ? 0ull - (uint64_t)v : (uint64_t)v;
  const uint64_t r = csub(reduce64_lazy(mag, c.mu64, c.q), c.q);
  return v < 0 && r ? c.q - r : r;
}

// sk_ntt[l][k] = sk[k] mod q_l (the forward transform follows).
__global__ __launch_bounds__(CLIENT_THREADS) void lift_key_kernel(const int64_t* __restrict__ sk,
                                                                   uint64_t* __restrict__ out, uint32_t N,
                                                                   uint32_t L, const LimbConst* __restrict__ lcs) {
  const uint64_t idx = (uint64_t)blockIdx.x * CLIENT_THREADS + threadIdx.x;
  if (idx >= (uint64_t)L * N) return;
  const uint32_t l = (uint32_t)(idx / N), k = (uint32_t)(idx % N);
  out[idx] = mod_q_signed_c(sk[k], lcs[l]);
}

// work[i] = ct[i][0]; with ct_a_out, also ct_a_out[i][0] = src[i] (encryption
// writes a into the ciphertext).  src: [n][L][N] at stride src_stride words.
__global__ __launch_bounds__(CLIENT_THREADS) void copy_a_kernel(const uint64_t* __restrict__ src, uint64_t src_stride,
                                                                 uint64_t* __restrict__ work,
                                                                 uint64_t* __restrict__ ct_out, uint32_t LN) {
  const uint64_t i = blockIdx.y;
  const uint32_t j = blockIdx.x * CLIENT_THREADS + threadIdx.x;
  if (j >= LN) return;
  const uint64_t v = src[i * src_stride + j];
  work[i * LN + j] = v;
  if (ct_out) ct_out[i * 2 * LN + j] = v;
}

// work[i][l][k] *= sk_ntt[l][k] mod q_l
__global__ __launch_bounds__(CLIENT_THREADS) void pointwise_key_kernel(uint64_t* __restrict__ work,
                                                                        const uint64_t* __restrict__ sk_ntt,
                                                                        uint32_t N, uint32_t L,
                                                                        const LimbConst* __restrict__ lcs) {
  const uint64_t i = blockIdx.y;
  const uint32_t j = blockIdx.x * CLIENT_THREADS + threadIdx.x;
  if (j >= L * N) return;
  const LimbConst c = lcs[j / N];
  uint64_t hi, lo;
  mul_wide(work[i * L * N + j], sk_ntt[j], hi, lo);
  work[i * L * N + j] = reduce128(hi, lo, c);
}

// ct[i][1][l][k] = as[i][l][k] + delta_l * (m mod t) + e mod q_l
__global__ __launch_bounds__(CLIENT_THREADS) void encrypt_finish_kernel(const uint64_t* __restrict__ as,
                                                                         const int64_t* __restrict__ msg,
                                                                         const int64_t* __restrict__ err,
                                                                         uint64_t* __restrict__ ct, uint32_t N,
                                                                         uint32_t L, uint64_t t,
                                                                         const LimbConst* __restrict__ lcs) {
  const uint64_t i = blockIdx.y;
  const uint32_t j = blockIdx.x * CLIENT_THREADS + threadIdx.x;
  if (j >= L * N) return;
  const uint32_t k = j % N;
  const LimbConst c = lcs[j / N];
  const int64_t mv = msg[i * N + k];
  int64_t r = mv % (int64_t)t;
  const uint64_t m = (uint64_t)(r < 0 ? r + (int64_t)t : r);
  const uint64_t dm = csub(mul_shoup_lazy(m, c.delta, c.delta_sh, c.q), c.q);
  uint64_t v = csub(as[i * L * N + j] + dm, c.q);
  v = csub(v + mod_q_signed_c(err[i * N + k], c), c.q);
  ct[(i * 2 + 1) * L * N + j] = v;
}

// out[i][k] = round(t * V / Q) mod t, centred, with v_l = ct[i][1][l][k] - as[i][l][k].
__global__ __launch_bounds__(CLIENT_THREADS) void decrypt_finish_kernel(const uint64_t* __restrict__ ct,
                                                                         const uint64_t* __restrict__ as,
                                                                         int64_t* __restrict__ out, uint32_t N,
                                                                         uint32_t L, LimbConst tc,
                                                                         const DecodeConst* __restrict__ dcs,
                                                                         const LimbConst* __restrict__ lcs) {
  const uint64_t i = blockIdx.y;
  const uint32_t k = blockIdx.x * CLIENT_THREADS + threadIdx.x;
  if (k >= N) return;
  uint64_t ih = 0, il = 0;           // sum v_l * I_l as a 128-bit number (each term below 2^122, L <= 8)
  uint64_t w2 = 0, w1 = 0, w0 = 0;  // sum v_l * F_l * 2^128 as a 192-bit number
  for (uint32_t l = 0; l < L; l++) {
    const LimbConst c = lcs[l];
    const DecodeConst d = dcs[l];
    const uint64_t b = ct[((i * 2 + 1) * L + l) * N + k], a = as[(i * L + l) * N + k];
    const uint64_t v = csub(b + (c.q - a), c.q);
    uint64_t ph, pl;
    mul_wide(v, d.ipart, ph, pl);
    il += pl;
    ih += ph + (il < pl);
    uint64_t h1, l1, h2, l2;
    mul_wide(v, d.frac_hi, h1, l1);  // v * F_hi: weight 2^64 in the 2^128 scale
    mul_wide(v, d.frac_lo, h2, l2);  // v * F_lo: weight 1
    // add (h1, l1) at words (w2, w1) and (h2, l2) at words (w1, w0)
    uint64_t s0 = w0 + l2;
    uint64_t c0 = s0 < w0;
    uint64_t s1 = w1 + l1;
    uint64_t c1 = s1 < w1;
    uint64_t s1b = s1 + h2;
    c1 += s1b < s1;
    s1b += c0;
    c1 += s1b < c0;
    w0 = s0, w1 = s1b, w2 += h1 + c1;
  }
  // integer part plus the rounded fraction sum, reduced mod t
  const uint64_t r = w2 + (w1 >> 63);
  il += r;
  ih += il < r;
  const uint64_t m = reduce128(ih, il, tc);
  out[i * N + k] = m >= tc.q / 2 + (tc.q & 1) ? (int64_t)m - (int64_t)tc.q : (int64_t)m;
}

static dim3 grid_of(uint64_t words, uint64_t n) { return dim3((uint32_t)((words + CLIENT_THREADS - 1) / CLIENT_THREADS), (uint32_t)n); }

hipError_t key_lift_launch(const int64_t* sk, uint64_t* out, uint32_t N, uint32_t L, const LimbConst* lc,
                           hipStream_t st) {
  hipLaunchKernelGGL(lift_key_kernel, dim3((uint32_t)(((uint64_t)L * N + CLIENT_THREADS - 1) / CLIENT_THREADS)),
                     dim3(CLIENT_THREADS), 0, st, sk, out, N, L, lc);
  return hipGetLastError();
}

hipError_t copy_a_launch(const uint64_t* src, uint64_t src_stride, uint64_t* work, uint64_t* ct_out, uint64_t n,
                         uint32_t N, uint32_t L, hipStream_t st) {
  hipLaunchKernelGGL(copy_a_kernel, grid_of((uint64_t)L * N, n), dim3(CLIENT_THREADS), 0, st, src, src_stride, work,
                     ct_out, L * N);
  return hipGetLastError();
}

hipError_t pointwise_key_launch(uint64_t* work, const uint64_t* sk_ntt, uint64_t n, uint32_t N, uint32_t L,
                                const LimbConst* lc, hipStream_t st) {
  hipLaunchKernelGGL(pointwise_key_kernel, grid_of((uint64_t)L * N, n), dim3(CLIENT_THREADS), 0, st, work, sk_ntt, N,
                     L, lc);
  return hipGetLastError();
}

hipError_t encrypt_finish_launch(const uint64_t* as, const int64_t* msg, const int64_t* err, uint64_t* ct, uint64_t n,
                                 uint32_t N, uint32_t L, uint64_t t, const LimbConst* lc, hipStream_t st) {
  hipLaunchKernelGGL(encrypt_finish_kernel, grid_of((uint64_t)L * N, n), dim3(CLIENT_THREADS), 0, st, as, msg, err,
                     ct, N, L, t, lc);
  return hipGetLastError();
}

hipError_t decrypt_finish_launch(const uint64_t* ct, const uint64_t* as, int64_t* out, uint64_t n, uint32_t N,
                                 uint32_t L, const LimbConst& tc, const DecodeConst* dc, const LimbConst* lc,
                                 hipStream_t st) {
  hipLaunchKernelGGL(decrypt_finish_kernel, grid_of(N, n), dim3(CLIENT_THREADS), 0, st, ct, as, out, N, L, tc, dc,
                     lc);
  return hipGetLastError();
}

}  // namespace heconv
