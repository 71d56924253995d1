// Ciphertext rotation for the Z_P variant (rotations need key switching
// with evaluation keys, Sec. 2; the Z_P kernels rotate once per
// multiply-accumulate iteration, Sec. 6.1): the Galois automorphism
// a(X) -> a(X^g) and hybrid key switching with one special prime P, the
// last modulus of an extended context q_0..q_{L-1}, P.  For a ciphertext
// (a, b) whose phase is b - a*s':
//   digits d_l = limb l of a, integers below q_l, reduced into every
//   modulus of the extended basis and transformed (modup_kernel + NTT);
//   A = sum_l d_l * k_a[l], B = sum_l d_l * k_b[l], point-wise in the NTT
//   domain (ks_inner_kernel), transformed back;
//   y = (x - [x]_P) / P with [x]_P the residue mod P centred into
//   (-P/2, P/2]: per modulus q_j, (x_j - ([x]_P mod q_j)) * P^-1 mod q_j
//   (moddown_kernel), giving (-A', b - B') under s.
// A rotation applies the automorphism to a while the digits are read and to
// b in the last step, so the rotated ciphertext is never stored.  Every
// kernel is elementwise over the N coefficients of a row; the transforms
// are the library's NTT kernels on the extended context.
#include "kernels.h"

namespace heconv {

constexpr uint32_t ROT_THREADS = 256;

__device__ __forceinline__ uint64_t red_word(uint64_t x, const LimbConst& c) {
  return csub(reduce64_lazy(x, c.mu64, c.q), c.q);
}

// Coefficient j of a(X^g) for the row a of N canonical residues mod q:
// with k = j * g^-1 mod 2N, a_k when k < N, else -a_{k-N}.  ginv = 1 reads
// the row as it is.
__device__ __forceinline__ uint64_t perm_load(const uint64_t* __restrict__ row, uint32_t j, uint32_t ginv, uint32_t N,
                                              uint64_t q) {
  const uint32_t k = (uint32_t)(((uint64_t)j * ginv) & (2 * N - 1));
  if (k < N) return row[k];
  const uint64_t v = row[k - N];
  return v ? q - v : 0;
}

// out[r] = in[r](X^g) for every row r of N coefficients; row r is limb
// r % L and uses modulus lcs[r % L].
__global__ __launch_bounds__(ROT_THREADS) void automorph_kernel(const uint64_t* __restrict__ in,
                                                                 uint64_t* __restrict__ out, uint32_t N,
                                                                 uint32_t L, uint32_t ginv,
                                                                 const LimbConst* __restrict__ lcs) {
  const uint32_t per_row = N / ROT_THREADS;
  const uint64_t row = blockIdx.x / per_row;
  const uint32_t j = (blockIdx.x % per_row) * ROT_THREADS + threadIdx.x;
  out[row * N + j] = perm_load(in + row * N, j, ginv, N, lcs[row % L].q);
}

// work[i][l][m][k] = (a_i(X^g))[l][k] mod p_m: digit l of ciphertext i in
// extended modulus m < L+1 (ct [n][2][L][N], a is component 0).
__global__ __launch_bounds__(ROT_THREADS) void modup_kernel(const uint64_t* __restrict__ ct,
                                                             uint64_t* __restrict__ work, uint32_t N, uint32_t L,
                                                             uint32_t ginv, const LimbConst* __restrict__ ext) {
  const uint32_t per_row = N / ROT_THREADS;
  const uint64_t row = blockIdx.x / per_row;  // (i, l, m)
  const uint32_t k = (blockIdx.x % per_row) * ROT_THREADS + threadIdx.x;
  const uint32_t m = (uint32_t)(row % (L + 1));
  const uint64_t il = row / (L + 1);
  const uint32_t l = (uint32_t)(il % L);
  const uint64_t i = il / L;
  const uint64_t d = perm_load(ct + (i * 2 * L + l) * N, k, ginv, N, ext[l].q);
  work[row * N + k] = m == l ? d : red_word(d, ext[m]);
}

// acc[i][c][m][k] = sum_l work[i][l][m][k] * ksk[l][c][m][k] mod p_m: the L
// products summed in 128 bits (each below 2^120, L <= 7), reduced once.
__global__ __launch_bounds__(ROT_THREADS) void ks_inner_kernel(const uint64_t* __restrict__ work,
                                                                const uint64_t* __restrict__ ksk,
                                                                uint64_t* __restrict__ acc, uint32_t N, uint32_t L,
                                                                const LimbConst* __restrict__ ext) {
  const uint32_t per_row = N / ROT_THREADS;
  const uint64_t row = blockIdx.x / per_row;  // (i, m)
  const uint32_t k = (blockIdx.x % per_row) * ROT_THREADS + threadIdx.x;
  const uint32_t L1 = L + 1;
  const uint32_t m = (uint32_t)(row % L1);
  const uint64_t i = row / L1;
  uint64_t ah = 0, al = 0, bh = 0, bl = 0;
  for (uint32_t l = 0; l < L; l++) {
    const uint64_t d = work[((i * L + l) * L1 + m) * N + k];
    uint64_t hi, lo;
    mul_wide(d, ksk[((uint64_t)(l * 2 + 0) * L1 + m) * N + k], hi, lo);
    al += lo;
    ah += hi + (al < lo);
    mul_wide(d, ksk[((uint64_t)(l * 2 + 1) * L1 + m) * N + k], hi, lo);
    bl += lo;
    bh += hi + (bl < lo);
  }
  const LimbConst c = ext[m];
  acc[((i * 2 + 0) * L1 + m) * N + k] = reduce128(ah, al, c);
  acc[((i * 2 + 1) * L1 + m) * N + k] = reduce128(bh, bl, c);
}

// out[i] = (-A', b(X^g) - B') with y = (x_j - ([x]_P mod q_j)) * P^-1 mod q_j
__global__ __launch_bounds__(ROT_THREADS) void moddown_kernel(const uint64_t* __restrict__ acc,
                                                               const uint64_t* __restrict__ ct,
                                                               uint64_t* __restrict__ out, uint32_t N, uint32_t L,
                                                               uint32_t ginv, PinvConst pinv,
                                                               const LimbConst* __restrict__ ext) {
  const uint32_t per_row = N / ROT_THREADS;
  const uint64_t row = blockIdx.x / per_row;  // (i, j), j < L
  const uint32_t k = (blockIdx.x % per_row) * ROT_THREADS + threadIdx.x;
  const uint32_t L1 = L + 1;
  const uint32_t j = (uint32_t)(row % L);
  const uint64_t i = row / L;
  const LimbConst c = ext[j];
  const uint64_t P = ext[L].q;
  uint64_t y[2];
#pragma unroll
  for (int comp = 0; comp < 2; comp++) {
    const uint64_t xj = acc[((i * 2 + comp) * L1 + j) * N + k];
    const uint64_t xp = acc[((i * 2 + comp) * L1 + L) * N + k];
    uint64_t cm;  // [x]_P mod q_j
    if (xp <= P / 2) {
      cm = red_word(xp, c);
    } else {
      const uint64_t mag = red_word(P - xp, c);
      cm = mag ? c.q - mag : 0;
    }
    const uint64_t d = csub(xj + (c.q - cm), c.q);
    y[comp] = csub(mul_shoup_lazy(d, pinv.v[j], pinv.sh[j], c.q), c.q);
  }
  out[((i * 2 + 0) * L + j) * N + k] = y[0] ? c.q - y[0] : 0;
  const uint64_t b = perm_load(ct + ((i * 2 + 1) * L + j) * N, k, ginv, N, c.q);
  out[((i * 2 + 1) * L + j) * N + k] = csub(b + (c.q - y[1]), c.q);
}

namespace {

hipError_t rows_grid(uint64_t rows, uint32_t N, uint32_t& blocks) {
  const uint64_t b = rows * (N / ROT_THREADS);
  if (b > 0x7fffffffull) return hipErrorInvalidConfiguration;
  blocks = (uint32_t)b;
  return hipSuccess;
}

}  // namespace

hipError_t automorph_launch(const uint64_t* in, uint64_t* out, uint64_t rows, uint32_t N, uint32_t L, uint32_t ginv,
                            const LimbConst* lc, hipStream_t st) {
  uint32_t blocks = 0;
  if (hipError_t e = rows_grid(rows, N, blocks)) return e;
  if (!blocks) return hipSuccess;
  hipLaunchKernelGGL(automorph_kernel, dim3(blocks), dim3(ROT_THREADS), 0, st, in, out, N, L, ginv, lc);
  return hipGetLastError();
}

hipError_t modup_launch(const uint64_t* ct, uint64_t* work, uint64_t n, uint32_t N, uint32_t L, uint32_t ginv,
                        const LimbConst* ext, hipStream_t st) {
  uint32_t blocks = 0;
  if (hipError_t e = rows_grid(n * L * (L + 1), N, blocks)) return e;
  if (!blocks) return hipSuccess;
  hipLaunchKernelGGL(modup_kernel, dim3(blocks), dim3(ROT_THREADS), 0, st, ct, work, N, L, ginv, ext);
  return hipGetLastError();
}

hipError_t ks_inner_launch(const uint64_t* work, const uint64_t* ksk, uint64_t* acc, uint64_t n, uint32_t N,
                           uint32_t L, const LimbConst* ext, hipStream_t st) {
  uint32_t blocks = 0;
  if (hipError_t e = rows_grid(n * (L + 1), N, blocks)) return e;
  if (!blocks) return hipSuccess;
  hipLaunchKernelGGL(ks_inner_kernel, dim3(blocks), dim3(ROT_THREADS), 0, st, work, ksk, acc, N, L, ext);
  return hipGetLastError();
}

hipError_t moddown_launch(const uint64_t* acc, const uint64_t* ct, uint64_t* out, uint64_t n, uint32_t N, uint32_t L,
                          uint32_t ginv, const PinvConst& pinv, const LimbConst* ext, hipStream_t st) {
  uint32_t blocks = 0;
  if (hipError_t e = rows_grid(n * L, N, blocks)) return e;
  if (!blocks) return hipSuccess;
  hipLaunchKernelGGL(moddown_kernel, dim3(blocks), dim3(ROT_THREADS), 0, st, acc, ct, out, N, L, ginv, pinv, ext);
  return hipGetLastError();
}

}  // namespace heconv
