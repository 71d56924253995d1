// NTT / inverse NTT in double precision for primes below 2^50: every
// residue is an exact double, and a modular product takes two products, two
// fused multiply-adds, a rounding and one conditional add -- all full-rate
// fp64 operations on gfx950, where the integer path's 32-bit multiplies run
// at half rate.  Same transform, order, mapping and passes as ntt_impl.h.
// Between stages values are balanced residues, |x| <= q/2 + 1, so no
// compare-and-select is needed anywhere but in the final canonical step.
//
// mulmod(a, b), |a| <= 2^50, 0 <= b < q < 2^50:
//   hi = RN(a*b), lo = a*b - hi (exact, by the fused multiply-add),
//   k = rint(RN(hi * RN(1/q))) is within 0.875 of a*b/q (three roundings of
//   relative size 2^-53 on a quotient below 2^50, plus the rounding to an
//   integer), and r = RN(hi - k*q) + lo = a*b - k*q exactly (integers below
//   2^52), so |r| < 0.875 q.
// red(s), |s| < 2^51: s - rint(RN(s * RN(1/q))) * q, exact, |result| <= q/2 + 1.
// A forward butterfly is red(x0 + T), red(x0 - T) with T = mulmod(x1, w);
// an inverse one red(X + Y), red(mulmod(X - Y, w)); with canonical inputs
// (|x| < q) or balanced ones, every mulmod input stays below q + 2.
#include "kernels.h"
#include "ntt_impl.h"

namespace heconv {

struct F64Const {
  double q, qinv, ninv, ninv_w;  // q, RN(1/q), N^-1, N^-1 times the last inverse twiddle
};

__device__ __forceinline__ double mulmod_f64(double a, double b, double q, double qinv) {
  const double hi = a * b;
  const double lo = __fma_rn(a, b, -hi);
  const double k = rint(hi * qinv);
  return __fma_rn(-k, q, hi) + lo;
}

__device__ __forceinline__ double red_f64(double s, double q, double qinv) { return __fma_rn(-rint(s * qinv), q, s); }

__device__ __forceinline__ double canon_f64(double r, double q) { return r < 0.0 ? r + q : r; }

template <int LOGN, int LOGE, int LO, int U0>
__device__ __forceinline__ void fwd_pass_f64(double (&x)[1 << LOGE], int tid, const double* __restrict__ tw,
                                             const F64Const& c) {
  const int high = tid >> LO;
#pragma unroll
  for (int u = U0; u < LOGE; u++) {
    const int s = LOGN - LOGE - LO + u;
    const int half = 1 << (LOGE - 1 - u);
#pragma unroll
    for (int g = 0; g < (1 << u); g++) {
      const double w = tw[(1 << s) + (high << u) + g];
#pragma unroll
      for (int e = 0; e < half; e++) {
        const int k0 = g * 2 * half + e, k1 = k0 + half;
        const double T = mulmod_f64(x[k1], w, c.q, c.qinv);
        const double X = x[k0];
        x[k0] = red_f64(X + T, c.q, c.qinv);
        x[k1] = red_f64(X - T, c.q, c.qinv);
      }
    }
  }
}

template <int LOGN, int LOGE, int LO, int U0, bool LAST>
__device__ __forceinline__ void inv_pass_f64(double (&x)[1 << LOGE], int tid, const double* __restrict__ tw,
                                             const F64Const& c) {
  const int high = tid >> LO;
#pragma unroll
  for (int u = LOGE - 1; u >= U0; u--) {
    const int s = LOGN - LOGE - LO + u;
    const int half = 1 << (LOGE - 1 - u);
    if (LAST && u == 0) {
#pragma unroll
      for (int e = 0; e < half; e++) {
        const double X = x[e], Y = x[e + half];
        x[e] = canon_f64(mulmod_f64(red_f64(X + Y, c.q, c.qinv), c.ninv, c.q, c.qinv), c.q);
        x[e + half] = canon_f64(mulmod_f64(X - Y, c.ninv_w, c.q, c.qinv), c.q);
      }
      continue;
    }
#pragma unroll
    for (int g = 0; g < (1 << u); g++) {
      const double w = tw[(1 << s) + (high << u) + g];
#pragma unroll
      for (int e = 0; e < half; e++) {
        const int k0 = g * 2 * half + e, k1 = k0 + half;
        const double X = x[k0], Y = x[k1];
        x[k0] = red_f64(X + Y, c.q, c.qinv);
        x[k1] = red_f64(mulmod_f64(X - Y, w, c.q, c.qinv), c.q, c.qinv);
      }
    }
  }
}

template <int LOGE, int FROM, int TO>
__device__ __forceinline__ void exchange_f64(double* lds, double (&x)[1 << LOGE], int tid) {
  __syncthreads();
#pragma unroll
  for (int k = 0; k < (1 << LOGE); k++) lds[lds_pad(elem_index<LOGE, FROM>(tid, k))] = x[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < (1 << LOGE); k++) x[k] = lds[lds_pad(elem_index<LOGE, TO>(tid, k))];
}

template <int LOGN, int LOGE, int P>
__device__ __forceinline__ void fwd_rest_f64(double (&x)[1 << LOGE], double* lds, int tid,
                                             const double* __restrict__ tw, const F64Const& c) {
  constexpr int NFULL = LOGN / LOGE, REM = LOGN % LOGE;
  if constexpr (P < NFULL) {
    constexpr int LO = LOGN - LOGE * (P + 1);
    if constexpr (P > 0) exchange_f64<LOGE, LO + LOGE, LO>(lds, x, tid);
    fwd_pass_f64<LOGN, LOGE, LO, 0>(x, tid, tw, c);
    fwd_rest_f64<LOGN, LOGE, P + 1>(x, lds, tid, tw, c);
  } else if constexpr (REM > 0) {
    exchange_f64<LOGE, LOGN - LOGE * NFULL, 0>(lds, x, tid);
    fwd_pass_f64<LOGN, LOGE, 0, LOGE - REM>(x, tid, tw, c);
  }
}

template <int LOGN, int LOGE, int P>
__device__ __forceinline__ void inv_rest_f64(double (&x)[1 << LOGE], double* lds, int tid,
                                             const double* __restrict__ tw, const F64Const& c) {
  constexpr int NFULL = LOGN / LOGE, REM = LOGN % LOGE;
  if constexpr (P < NFULL) {
    constexpr int LO = REM + LOGE * P;
    constexpr int PREV = (P == 0) ? 0 : REM + LOGE * (P - 1);
    if constexpr (P > 0 || REM > 0) exchange_f64<LOGE, PREV, LO>(lds, x, tid);
    inv_pass_f64<LOGN, LOGE, LO, 0, (P == NFULL - 1)>(x, tid, tw, c);
    inv_rest_f64<LOGN, LOGE, P + 1>(x, lds, tid, tw, c);
  }
}

template <int LOGN, int LOGE>
__global__ __launch_bounds__((1 << LOGN) >> LOGE) void ntt_fwd_f64_kernel(uint64_t* __restrict__ polys_, uint32_t L,
                                                                           const double* __restrict__ tw_all,
                                                                           const F64Const* __restrict__ fcs) {
  constexpr int N = 1 << LOGN, E = 1 << LOGE, T = N / E, TOP = LOGN - LOGE;
  __shared__ double lds[N + N / 16];
  const uint32_t p = blockIdx.x, l = p % L;
  const F64Const c = fcs[l];
  const double* tw = tw_all + (size_t)l * N;
  gword* a = as_global(polys_) + (size_t)p * N;
  const int tid = threadIdx.x;
  double x[E];
#pragma unroll
  for (int k = 0; k < E; k++) x[k] = (double)a[tid + k * T];
  fwd_rest_f64<LOGN, LOGE, 0>(x, lds, tid, tw, c);
#pragma unroll
  for (int k = 0; k < E; k++) x[k] = canon_f64(x[k], c.q);
  exchange_f64<LOGE, 0, TOP>(lds, x, tid);
#pragma unroll
  for (int k = 0; k < E; k++) a[tid + k * T] = (uint64_t)x[k];
}

template <int LOGN, int LOGE>
__global__ __launch_bounds__((1 << LOGN) >> LOGE) void ntt_inv_f64_kernel(uint64_t* __restrict__ polys_, uint32_t L,
                                                                           const double* __restrict__ tw_all,
                                                                           const F64Const* __restrict__ fcs) {
  constexpr int N = 1 << LOGN, E = 1 << LOGE, T = N / E, TOP = LOGN - LOGE, REM = LOGN % LOGE;
  __shared__ double lds[N + N / 16];
  const uint32_t p = blockIdx.x, l = p % L;
  const F64Const c = fcs[l];
  const double* tw = tw_all + (size_t)l * N;
  gword* a = as_global(polys_) + (size_t)p * N;
  const int tid = threadIdx.x;
  double x[E];
#pragma unroll
  for (int k = 0; k < E; k++) x[k] = (double)a[tid + k * T];
  exchange_f64<LOGE, TOP, 0>(lds, x, tid);
  if constexpr (REM > 0) inv_pass_f64<LOGN, LOGE, 0, LOGE - REM, false>(x, tid, tw, c);
  inv_rest_f64<LOGN, LOGE, 0>(x, lds, tid, tw, c);
#pragma unroll
  for (int k = 0; k < E; k++) a[tid + k * T] = (uint64_t)x[k];
}

template <int LOGN, int LOGE>
static hipError_t go_f64(bool inverse, uint64_t* polys, uint64_t nlp, uint32_t L, const double* tw,
                         const F64Const* fc, hipStream_t st) {
  constexpr int T = (1 << LOGN) >> LOGE;
  const uint64_t max_blocks = grid_max_blocks(T) / L * L;  // whole RNS polynomials per launch
  for (uint64_t off = 0; off < nlp; off += max_blocks) {
    const uint64_t cnt = nlp - off < max_blocks ? nlp - off : max_blocks;
    uint64_t* base = polys + off * (1ull << LOGN);
    if (inverse)
      hipLaunchKernelGGL((ntt_inv_f64_kernel<LOGN, LOGE>), dim3((uint32_t)cnt), dim3(T), 0, st, base, L, tw, fc);
    else
      hipLaunchKernelGGL((ntt_fwd_f64_kernel<LOGN, LOGE>), dim3((uint32_t)cnt), dim3(T), 0, st, base, L, tw, fc);
  }
  return hipGetLastError();
}

template <int LOGN>
static hipError_t go_f64_e(bool inverse, uint32_t loge, uint64_t* polys, uint64_t nlp, uint32_t L, const double* tw,
                           const F64Const* fc, hipStream_t st) {
  if constexpr (LOGN <= 13) {
    if (loge == 3) return go_f64<LOGN, 3>(inverse, polys, nlp, L, tw, fc, st);
  }
  return go_f64<LOGN, 4>(inverse, polys, nlp, L, tw, fc, st);
}

size_t f64_const_size() { return sizeof(F64Const); }

void f64_const_fill(void* out, double q, double qinv, double ninv, double ninv_w) {
  *static_cast<F64Const*>(out) = F64Const{q, qinv, ninv, ninv_w};
}

hipError_t ntt_f64_launch(bool inverse, uint32_t logN, uint32_t loge, uint64_t* polys, uint64_t n_rns_polys,
                          uint32_t L, const double* tw, const void* fc, hipStream_t st) {
  const uint64_t nlp = n_rns_polys * L;
  if (nlp == 0) return hipSuccess;
  const F64Const* f = static_cast<const F64Const*>(fc);
  switch (logN) {
    case 10: return go_f64_e<10>(inverse, loge, polys, nlp, L, tw, f, st);
    case 11: return go_f64_e<11>(inverse, loge, polys, nlp, L, tw, f, st);
    case 12: return go_f64_e<12>(inverse, loge, polys, nlp, L, tw, f, st);
    case 13: return go_f64_e<13>(inverse, loge, polys, nlp, L, tw, f, st);
    case 14: return go_f64_e<14>(inverse, loge, polys, nlp, L, tw, f, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace heconv
