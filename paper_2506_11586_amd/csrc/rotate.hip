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
// b in the last step, so the rotated ciphertext is never stored.
// By default the steps run as three kernels: modup_ntt_kernel (digit
// extension in the forward transform's load), inner_intt_kernel (the inner
// product in the inverse transform's load) and moddown_kernel.  The
// elementwise modup_kernel and ks_inner_kernel with the library's NTT
// kernels between them are the separate-steps form, and ks_fwd_kernel the
// form with both sums kept in registers (tuning ks_fused 0 and 2).
#include "kernels.h"
#include "mac_impl.h"
#include "ntt_impl.h"

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
// With addp non-null, the ciphertext addp[i] is added to the result.
__global__ __launch_bounds__(ROT_THREADS) void moddown_kernel(const uint64_t* __restrict__ acc,
                                                               const uint64_t* __restrict__ ct,
                                                               uint64_t* __restrict__ out, uint32_t N, uint32_t L,
                                                               uint32_t ginv, PinvConst pinv,
                                                               const uint64_t* __restrict__ addp,
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
  const uint64_t b = ct ? perm_load(ct + ((i * 2 + 1) * L + j) * N, k, ginv, N, c.q) : 0;  // null: a zero ciphertext
  uint64_t oa = y[0] ? c.q - y[0] : 0, ob = csub(b + (c.q - y[1]), c.q);
  if (addp) {
    oa = csub(oa + addp[((i * 2 + 0) * L + j) * N + k], c.q);
    ob = csub(ob + addp[((i * 2 + 1) * L + j) * N + k], c.q);
  }
  out[((i * 2 + 0) * L + j) * N + k] = oa;
  out[((i * 2 + 1) * L + j) * N + k] = ob;
}

// Digit extension, forward transform and inner product fused: one workgroup
// per (ciphertext i, extended modulus m) runs the L digits one after the
// other.  Digit l is read from the ciphertext's a row (the automorphism
// applied through LDS: the row is staged with coalesced loads, then each
// thread gathers its permuted entries), reduced mod p_m, transformed in
// registers, and multiplied by the key's transformed rows; the two sums stay
// in registers and only they are stored.  The L+1 workgroups of one
// ciphertext run on the same XCD (block b runs on XCD b % 8), so they share
// its a rows in that XCD's L2.  Grid: ceil(n/8)*8*(L+1) workgroups.
template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) >> 3) void ks_fwd_kernel(const uint64_t* __restrict__ ct,
                                                                   const uint64_t* __restrict__ ksk,
                                                                   uint64_t* __restrict__ acc, uint64_t n, uint32_t L,
                                                                   uint32_t ginv, const Tw* __restrict__ tw_all,
                                                                   const LimbConst* __restrict__ ext) {
  constexpr int LOGE = 3, E = 1 << LOGE, N = 1 << LOGN, T = N / E, TOP = LOGN - LOGE;
  __shared__ uint64_t lds[N + N / 16];
  const uint32_t L1 = L + 1;
  const uint32_t xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
  const uint64_t i = (uint64_t)(slot / L1) * 8 + xcd;
  const uint32_t m = slot % L1;
  if (i >= n) return;  // the whole workgroup leaves before any barrier
  const LimbConst c = ext[m];
  uint64_t sa[E], sb[E];
#pragma unroll
  for (int k = 0; k < E; k++) sa[k] = sb[k] = 0;
  for (uint32_t l = 0; l < L; l++) {
    // The thread index and twiddle offset pass through an empty asm
    // statement each digit, so that the address arithmetic and twiddle loads
    // (the same for every digit) are redone instead of hoisted out of the
    // loop, where they would stay live across it and spill.
    int tid = threadIdx.x;
    uint32_t off = m * N;
    asm volatile("" : "+v"(tid), "+v"(off));
    const Tw* tw = tw_all + __builtin_amdgcn_readfirstlane(off);
    const uint64_t* row = ct + (i * 2 * L + l) * N;
    uint64_t x[E];
    if (ginv == 1) {
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = row[tid + k * T];
    } else {
      const uint64_t ql = ext[l].q;
      __syncthreads();  // the previous digit's last LDS reads are done
#pragma unroll
      for (int k = 0; k < E; k++) lds[lds_pad(tid + k * T)] = row[tid + k * T];
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; k++) {
        const uint32_t src = (uint32_t)(((uint64_t)(tid + k * T) * ginv) & (2 * N - 1));
        const uint64_t v = lds[lds_pad(src & (N - 1))];
        x[k] = src >= (uint32_t)N && v ? ql - v : v;
      }
    }
    if (m != l) {
#pragma unroll
      for (int k = 0; k < E; k++) x[k] = red_word(x[k], c);
    }
    fwd_rest<LOGN, LOGE, 0>(x, lds, tid, tw, c);
#pragma unroll
    for (int k = 0; k < E; k++) x[k] = fwd_canon(x[k], c);
    exchange<LOGE, 0, TOP>(lds, x, tid);  // entry tid + k*T, as the key rows are read
    // the key loads are addressed from a value defined here, so they are
    // issued after the transform rather than held in registers through it
    int tk = tid;
    asm volatile("" : "+v"(tk));
    const uint64_t* ka = ksk + ((uint64_t)(l * 2) * L1 + m) * N;
    const uint64_t* kb = ka + (uint64_t)L1 * N;
#pragma unroll
    for (int k = 0; k < E; k++) {
      uint64_t hi, lo;
      mul_wide(x[k], ka[tk + k * T], hi, lo);
      sa[k] = csub(sa[k] + reduce128(hi, lo, c), c.q);
      mul_wide(x[k], kb[tk + k * T], hi, lo);
      sb[k] = csub(sb[k] + reduce128(hi, lo, c), c.q);
    }
  }
  const int tid = threadIdx.x;
  uint64_t* oa = acc + ((i * 2) * L1 + m) * N;
  uint64_t* ob = oa + (uint64_t)L1 * N;
#pragma unroll
  for (int k = 0; k < E; k++) {
    oa[tid + k * T] = sa[k];
    ob[tid + k * T] = sb[k];
  }
}

// Digit extension fused into the forward transform: one workgroup per
// (ciphertext i, digit l, extended modulus m) reads limb l of a (through the
// automorphism, staged in LDS as in ks_fwd_kernel), reduces it mod p_m and
// stores its transform to digits[i][l][m].  The L+1 workgroups that read one
// a row run on the same XCD.  Grid: ceil(n*L/8)*8*(L+1) workgroups.
template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) >> 3) void modup_ntt_kernel(const uint64_t* __restrict__ ct,
                                                                      uint64_t* __restrict__ digits, uint64_t n,
                                                                      uint32_t L, uint32_t ginv,
                                                                      const Tw* __restrict__ tw_all,
                                                                      const LimbConst* __restrict__ ext) {
  constexpr int LOGE = 3, E = 1 << LOGE, N = 1 << LOGN, T = N / E, TOP = LOGN - LOGE;
  __shared__ uint64_t lds[N + N / 16];
  const uint32_t L1 = L + 1;
  const uint32_t xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
  const uint64_t il = (uint64_t)(slot / L1) * 8 + xcd;  // (i, l)
  const uint32_t m = slot % L1;
  if (il >= n * L) return;  // the whole workgroup leaves before any barrier
  const uint32_t l = (uint32_t)(il % L);
  const uint64_t i = il / L;
  const int tid = threadIdx.x;
  const LimbConst c = ext[m];
  const uint64_t* row = ct + (i * 2 * L + l) * N;
  uint64_t x[E];
  if (ginv == 1) {
#pragma unroll
    for (int k = 0; k < E; k++) x[k] = row[tid + k * T];
  } else {
    const uint64_t ql = ext[l].q;
#pragma unroll
    for (int k = 0; k < E; k++) lds[lds_pad(tid + k * T)] = row[tid + k * T];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; k++) {
      const uint32_t src = (uint32_t)(((uint64_t)(tid + k * T) * ginv) & (2 * N - 1));
      const uint64_t v = lds[lds_pad(src & (N - 1))];
      x[k] = src >= (uint32_t)N && v ? ql - v : v;
    }
  }
  if (m != l) {
#pragma unroll
    for (int k = 0; k < E; k++) x[k] = red_word(x[k], c);
  }
  fwd_rest<LOGN, LOGE, 0>(x, lds, tid, tw_all + (size_t)m * N, c);
#pragma unroll
  for (int k = 0; k < E; k++) x[k] = fwd_canon(x[k], c);
  exchange<LOGE, 0, TOP>(lds, x, tid);
  uint64_t* out = digits + (il * L1 + m) * N;
#pragma unroll
  for (int k = 0; k < E; k++) out[tid + k * T] = x[k];
}

// Inner product fused into the inverse transform: one workgroup per
// (ciphertext i, component c, extended modulus m) sums the L products of the
// transformed digits with the key row (c, m) in 128 bits as it loads them,
// reduces once, transforms back in registers and stores acc[i][c][m].  The
// two workgroups that read the same digit rows run on the same XCD.  Grid:
// ceil(n*(L+1)/8)*8*2 workgroups.
//
// With a plaintext term (xp, wp non-null; the Z_P multiply-accumulate-rotate
// step), the sum for a ciphertext modulus m < L also takes
// xp[i][c][m] * wp[m]: the input ciphertext times a plaintext already
// multiplied by -P mod q_m.  The term is 0 mod P, so the division by P in
// moddown_kernel leaves the rotated ciphertext plus (x * plaintext) exactly.
// nd digits are summed (L, or 0 when the rotated ciphertext is zero).  The
// batch may hold several chains of chain_cts ciphertexts that share the
// input x but take different weights: ciphertext i uses x[i % chain_cts]
// and the plaintext at wp + (i / chain_cts) * w_stride.
template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) >> 3) void inner_intt_kernel(const uint64_t* __restrict__ digits,
                                                                       const uint64_t* __restrict__ ksk,
                                                                       uint64_t* __restrict__ acc, uint64_t n,
                                                                       uint32_t L, uint32_t nd,
                                                                       const uint64_t* __restrict__ xp,
                                                                       const uint64_t* __restrict__ wp,
                                                                       uint64_t chain_cts, uint64_t w_stride,
                                                                       const Tw* __restrict__ tw_all,
                                                                       const LimbConst* __restrict__ ext) {
  constexpr int LOGE = 3, E = 1 << LOGE, N = 1 << LOGN, T = N / E;
  __shared__ uint64_t lds[N + N / 16];
  const uint32_t L1 = L + 1;
  const uint32_t xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
  const uint64_t im = (uint64_t)(slot / 2) * 8 + xcd;  // (i, m)
  const uint32_t comp = slot % 2;
  if (im >= n * L1) return;  // the whole workgroup leaves before any barrier
  const uint32_t m = (uint32_t)(im % L1);
  const uint64_t i = im / L1;
  const int tid = threadIdx.x;
  const LimbConst c = ext[m];
  uint64_t hi[E], lo[E];
#pragma unroll
  for (int k = 0; k < E; k++) hi[k] = lo[k] = 0;
  // L <= 7 digit products and one plaintext product, each below 2^120: the
  // 128-bit sums do not overflow.  Rows are read through buffer resources
  // (the row base in scalar registers, the lane's byte offset fixed, the
  // register's offset k*T*8 a scalar), so a load costs no per-lane address
  // arithmetic.
  const bool plain = xp && m < L;
  const uint32_t lane = (uint32_t)tid * 8;
  for (uint32_t l = 0; l < nd + (plain ? 1 : 0); l++) {
    const uint64_t* d =
        l < nd ? digits + ((i * L + l) * L1 + m) * N : xp + (((i % chain_cts) * 2 + comp) * L + m) * N;
    const uint64_t* kr =
        l < nd ? ksk + ((uint64_t)(l * 2 + comp) * L1 + m) * N : wp + (i / chain_cts) * w_stride + (uint64_t)m * N;
    const __amdgpu_buffer_rsrc_t rd = mac_rsrc((const uint64_t*)uniform64((uint64_t)d), (uint64_t)N * 8);
    const __amdgpu_buffer_rsrc_t rk = mac_rsrc((const uint64_t*)uniform64((uint64_t)kr), (uint64_t)N * 8);
#pragma unroll
    for (int k = 0; k < E; k++) {
      uint64_t ph, pl;
      mul_wide(mac_load(rd, lane, (uint32_t)(k * T * 8)), mac_load(rk, lane, (uint32_t)(k * T * 8)), ph, pl);
      lo[k] += pl;
      hi[k] += ph + (lo[k] < pl);
    }
  }
  uint64_t x[E];
#pragma unroll
  for (int k = 0; k < E; k++) x[k] = reduce128(hi[k], lo[k], c);
  ntt_inv_regs<LOGN, LOGE>(x, tw_all + (size_t)m * N, c, lds, tid);
  uint64_t* out = acc + ((i * 2 + comp) * L1 + m) * N;
#pragma unroll
  for (int k = 0; k < E; k++) out[tid + k * T] = x[k];
}

// Galois key for digit l and extended modulus m, in NTT form:
//   ksk[l][0][m] = a[l][m],
//   ksk[l][1][m] = a[l][m]*s + e[l] + (m == l ? P mod q_l : 0) * s(X^g)  (mod p_m),
// since G_l = P * Qhat_l * (Qhat_l^-1 mod q_l) is P mod q_l in limb l and 0
// in every other limb (Qhat_l holds every other q, P is a factor).  Inputs
// are the transforms: work = [a: L][e: L][s][s(X^g)] RNS polynomials of L+1
// limbs.
__global__ __launch_bounds__(ROT_THREADS) void galois_key_kernel(const uint64_t* __restrict__ work,
                                                                  uint64_t* __restrict__ ksk, uint32_t N,
                                                                  uint32_t L, const LimbConst* __restrict__ ext) {
  const uint32_t per_row = N / ROT_THREADS;
  const uint64_t row = blockIdx.x / per_row;  // (l, m)
  const uint32_t k = (blockIdx.x % per_row) * ROT_THREADS + threadIdx.x;
  const uint32_t L1 = L + 1;
  const uint32_t m = (uint32_t)(row % L1), l = (uint32_t)(row / L1);
  const LimbConst c = ext[m];
  const uint64_t LN1 = (uint64_t)L1 * N;
  const uint64_t a = work[row * N + k];
  const uint64_t e = work[L * LN1 + row * N + k];
  const uint64_t sv = work[2 * L * LN1 + (uint64_t)m * N + k];
  uint64_t hi, lo;
  mul_wide(a, sv, hi, lo);
  uint64_t v = csub(reduce128(hi, lo, c) + e, c.q);
  if (m == l) {
    const uint64_t sg = work[(2 * L + 1) * LN1 + (uint64_t)m * N + k];
    mul_wide(red_word(ext[L].q, c), sg, hi, lo);
    v = csub(v + reduce128(hi, lo, c), c.q);
  }
  ksk[((uint64_t)(l * 2 + 0) * L1 + m) * N + k] = a;
  ksk[((uint64_t)(l * 2 + 1) * L1 + m) * N + k] = v;
}

namespace {

hipError_t rows_grid(uint64_t rows, uint32_t N, uint32_t& blocks) {
  const uint64_t b = rows * (N / ROT_THREADS);
  if (b > grid_max_blocks(ROT_THREADS)) return hipErrorInvalidConfiguration;
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
                          uint32_t ginv, const PinvConst& pinv, const LimbConst* ext, hipStream_t st,
                          const uint64_t* addp) {
  uint32_t blocks = 0;
  if (hipError_t e = rows_grid(n * L, N, blocks)) return e;
  if (!blocks) return hipSuccess;
  hipLaunchKernelGGL(moddown_kernel, dim3(blocks), dim3(ROT_THREADS), 0, st, acc, ct, out, N, L, ginv, pinv, addp, ext);
  return hipGetLastError();
}

bool ks_fwd_supported(uint32_t logN) { return logN >= 10 && logN <= 13; }

hipError_t ks_fwd_launch(uint32_t logN, const uint64_t* ct, const uint64_t* ksk, uint64_t* acc, uint64_t n, uint32_t L,
                         uint32_t ginv, const Tw* tw, const LimbConst* ext, hipStream_t st) {
  const uint64_t blocks = (n + 7) / 8 * 8 * (L + 1);
  if (blocks > grid_max_blocks(1024)) return hipErrorInvalidConfiguration;  // up to N/8 = 1024 threads
  if (!blocks) return hipSuccess;
  const dim3 grid((uint32_t)blocks);
  switch (logN) {
    case 10: hipLaunchKernelGGL(ks_fwd_kernel<10>, grid, dim3(128), 0, st, ct, ksk, acc, n, L, ginv, tw, ext); break;
    case 11: hipLaunchKernelGGL(ks_fwd_kernel<11>, grid, dim3(256), 0, st, ct, ksk, acc, n, L, ginv, tw, ext); break;
    case 12: hipLaunchKernelGGL(ks_fwd_kernel<12>, grid, dim3(512), 0, st, ct, ksk, acc, n, L, ginv, tw, ext); break;
    case 13: hipLaunchKernelGGL(ks_fwd_kernel<13>, grid, dim3(1024), 0, st, ct, ksk, acc, n, L, ginv, tw, ext); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t modup_ntt_launch(uint32_t logN, const uint64_t* ct, uint64_t* digits, uint64_t n, uint32_t L, uint32_t ginv,
                            const Tw* tw, const LimbConst* ext, hipStream_t st) {
  const uint64_t blocks = (n * L + 7) / 8 * 8 * (L + 1);
  if (blocks > grid_max_blocks(1024)) return hipErrorInvalidConfiguration;  // up to N/8 = 1024 threads
  if (!blocks) return hipSuccess;
  const dim3 grid((uint32_t)blocks);
  switch (logN) {
    case 10: hipLaunchKernelGGL(modup_ntt_kernel<10>, grid, dim3(128), 0, st, ct, digits, n, L, ginv, tw, ext); break;
    case 11: hipLaunchKernelGGL(modup_ntt_kernel<11>, grid, dim3(256), 0, st, ct, digits, n, L, ginv, tw, ext); break;
    case 12: hipLaunchKernelGGL(modup_ntt_kernel<12>, grid, dim3(512), 0, st, ct, digits, n, L, ginv, tw, ext); break;
    case 13: hipLaunchKernelGGL(modup_ntt_kernel<13>, grid, dim3(1024), 0, st, ct, digits, n, L, ginv, tw, ext); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t inner_intt_launch(uint32_t logN, const uint64_t* digits, const uint64_t* ksk, uint64_t* acc, uint64_t n,
                             uint32_t L, uint32_t nd, const uint64_t* xp, const uint64_t* wp, uint64_t chain_cts,
                             uint64_t w_stride, const Tw* tw_inv, const LimbConst* ext, hipStream_t st) {
  if (chain_cts == 0) chain_cts = n ? n : 1;
  const uint64_t blocks = (n * (L + 1) + 7) / 8 * 8 * 2;
  if (blocks > grid_max_blocks(1024)) return hipErrorInvalidConfiguration;  // up to N/8 = 1024 threads
  if (!blocks) return hipSuccess;
  const dim3 grid((uint32_t)blocks);
  switch (logN) {
    case 10:
      hipLaunchKernelGGL(inner_intt_kernel<10>, grid, dim3(128), 0, st, digits, ksk, acc, n, L, nd, xp, wp, chain_cts,
                         w_stride, tw_inv, ext);
      break;
    case 11:
      hipLaunchKernelGGL(inner_intt_kernel<11>, grid, dim3(256), 0, st, digits, ksk, acc, n, L, nd, xp, wp, chain_cts,
                         w_stride, tw_inv, ext);
      break;
    case 12:
      hipLaunchKernelGGL(inner_intt_kernel<12>, grid, dim3(512), 0, st, digits, ksk, acc, n, L, nd, xp, wp, chain_cts,
                         w_stride, tw_inv, ext);
      break;
    case 13:
      hipLaunchKernelGGL(inner_intt_kernel<13>, grid, dim3(1024), 0, st, digits, ksk, acc, n, L, nd, xp, wp, chain_cts,
                         w_stride, tw_inv, ext);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t galois_key_launch(const uint64_t* work, uint64_t* ksk, uint32_t N, uint32_t L, const LimbConst* ext,
                             hipStream_t st) {
  uint32_t blocks = 0;
  if (hipError_t e = rows_grid((uint64_t)L * (L + 1), N, blocks)) return e;
  hipLaunchKernelGGL(galois_key_kernel, dim3(blocks), dim3(ROT_THREADS), 0, st, work, ksk, N, L, ext);
  return hipGetLastError();
}

}  // namespace heconv
