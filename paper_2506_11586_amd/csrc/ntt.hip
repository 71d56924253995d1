// Fused negacyclic NTT / inverse NTT for gfx950: one workgroup per limb
// polynomial, 16 coefficients per thread in registers, radix-16 passes
// (four butterfly stages each) with an LDS transpose between passes.
//
// Forward (Cooley-Tukey, natural order in, bit-reversed order out): the
// butterfly on bit b pairs j and j + 2^b with twiddle psi^brv(2^(n-1-b) +
// (j >> (b+1))), n = log2 N; stages run from bit n-1 down to bit 0.  The
// inverse (Gentleman-Sande) uses the same index with psi^-1 and runs from
// bit 0 up; its last stage also applies N^-1.  Lazy reduction after Harvey:
// forward values stay in [0, 4q), inverse values in [0, 2q), and every
// stored word is canonical.
//
// Thread/element mapping of a pass over bits [lo, lo+4): register k of thread
// t holds element j = (t mod 2^lo) | k << lo | (t >> lo) << (lo+4).  The first
// forward pass (lo = n-4) is therefore j = t + k*N/16, a coalesced load; the
// inverse ends on the same mapping and stores coalesced.  When n is not a
// multiple of 4 the leftover bits are done by a partial pass at lo = 0.
#include "kernels.h"

namespace heconv {

constexpr int E = 16;

__device__ __forceinline__ int lds_pad(int j) { return j + (j >> 4); }

template <int LO>
__device__ __forceinline__ int elem_index(int tid, int k) {
  const int low = tid & ((1 << LO) - 1);
  const int high = tid >> LO;
  return low | (k << LO) | (high << (LO + 4));
}

// Forward stages u in [U0, 4) of the pass at bit offset LO.
template <int LOGN, int LO, int U0>
__device__ __forceinline__ void fwd_pass(uint64_t (&x)[E], int tid, const Tw* __restrict__ tw, uint64_t q,
                                         uint64_t q2) {
  const int high = tid >> LO;
#pragma unroll
  for (int u = U0; u < 4; u++) {
    const int s = LOGN - 4 - LO + u;  // stage index: butterflies on bit LO+3-u
    const int half = 1 << (3 - u);
#pragma unroll
    for (int g = 0; g < (1 << u); g++) {
      const Tw t = tw[(1 << s) + (high << u) + g];
#pragma unroll
      for (int e = 0; e < half; e++) {
        const int k0 = g * 2 * half + e, k1 = k0 + half;
        uint64_t X = csub(x[k0], q2);
        uint64_t T = mul_shoup_lazy(x[k1], t.w, t.wsh, q);
        x[k0] = X + T;
        x[k1] = X - T + q2;
      }
    }
  }
}

// Inverse stages u from 3 down to U0 of the pass at LO.  With LAST, the
// stage on the top bit (u = 0 of the pass at LOGN-4) also applies N^-1.
template <int LOGN, int LO, int U0, bool LAST>
__device__ __forceinline__ void inv_pass(uint64_t (&x)[E], int tid, const Tw* __restrict__ tw,
                                         const LimbConst& c) {
  const int high = tid >> LO;
  const uint64_t q = c.q, q2 = c.two_q;
#pragma unroll
  for (int u = 3; u >= U0; u--) {
    const int s = LOGN - 4 - LO + u;
    const int half = 1 << (3 - u);
    if (LAST && u == 0) {
#pragma unroll
      for (int e = 0; e < half; e++) {
        const int k0 = e, k1 = e + half;
        uint64_t X = x[k0], Y = x[k1];
        x[k0] = csub(mul_shoup_lazy(X + Y, c.ninv, c.ninv_sh, q), q);
        x[k1] = csub(mul_shoup_lazy(X - Y + q2, c.ninv_w, c.ninv_w_sh, q), q);
      }
      continue;
    }
#pragma unroll
    for (int g = 0; g < (1 << u); g++) {
      const Tw t = tw[(1 << s) + (high << u) + g];
#pragma unroll
      for (int e = 0; e < half; e++) {
        const int k0 = g * 2 * half + e, k1 = k0 + half;
        uint64_t X = x[k0], Y = x[k1];
        x[k0] = csub(X + Y, q2);
        x[k1] = mul_shoup_lazy(X - Y + q2, t.w, t.wsh, q);
      }
    }
  }
}

template <int LO>
__device__ __forceinline__ void to_lds(uint64_t* lds, const uint64_t (&x)[E], int tid) {
#pragma unroll
  for (int k = 0; k < E; k++) lds[lds_pad(elem_index<LO>(tid, k))] = x[k];
}

template <int LO>
__device__ __forceinline__ void from_lds(const uint64_t* lds, uint64_t (&x)[E], int tid) {
#pragma unroll
  for (int k = 0; k < E; k++) x[k] = lds[lds_pad(elem_index<LO>(tid, k))];
}

// Forward passes at LO = LOGN-4, LOGN-8, ... (P counts full passes done).
template <int LOGN, int P>
__device__ __forceinline__ void fwd_rest(uint64_t (&x)[E], uint64_t* lds, int tid, const Tw* __restrict__ tw,
                                         uint64_t q, uint64_t q2) {
  constexpr int NFULL = LOGN / 4, REM = LOGN % 4;
  if constexpr (P < NFULL) {
    constexpr int LO = LOGN - 4 * (P + 1);
    constexpr int PREV = LOGN - 4 * P;  // previous pass offset (only used when P > 0)
    if constexpr (P > 0) {
      __syncthreads();
      to_lds<PREV>(lds, x, tid);
      __syncthreads();
      from_lds<LO>(lds, x, tid);
    }
    fwd_pass<LOGN, LO, 0>(x, tid, tw, q, q2);
    fwd_rest<LOGN, P + 1>(x, lds, tid, tw, q, q2);
  } else if constexpr (REM > 0) {
    constexpr int PREV = LOGN - 4 * NFULL;
    __syncthreads();
    to_lds<PREV>(lds, x, tid);
    __syncthreads();
    from_lds<0>(lds, x, tid);
    fwd_pass<LOGN, 0, 4 - REM>(x, tid, tw, q, q2);
  }
}

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / E) void ntt_fwd_kernel(uint64_t* __restrict__ polys, uint32_t L,
                                                                   const Tw* __restrict__ tw_all,
                                                                   const LimbConst* __restrict__ lcs) {
  constexpr int N = 1 << LOGN, T = N / E;
  __shared__ uint64_t lds[N + N / 16];
  const int tid = threadIdx.x;
  const uint32_t p = blockIdx.x;
  const uint32_t l = p % L;
  uint64_t* a = polys + (size_t)p * N;
  const Tw* tw = tw_all + (size_t)l * N;
  const uint64_t q = lcs[l].q, q2 = lcs[l].two_q;
  uint64_t x[E];
#pragma unroll
  for (int k = 0; k < E; k++) x[k] = a[tid + k * T];
  fwd_rest<LOGN, 0>(x, lds, tid, tw, q, q2);
  // the last pass used LO = 0: thread holds the 16 consecutive words tid*16 + k
#pragma unroll
  for (int k = 0; k < E; k++) x[k] = csub(csub(x[k], q2), q);
  ulonglong2* dst = reinterpret_cast<ulonglong2*>(a) + tid * (E / 2);
#pragma unroll
  for (int k = 0; k < E / 2; k++) dst[k] = make_ulonglong2(x[2 * k], x[2 * k + 1]);
}

// Inverse: optional partial pass at LO = 0 (bits 0..REM-1), then full passes
// at LO = REM, REM+4, ..., LOGN-4.
template <int LOGN, int P>
__device__ __forceinline__ void inv_rest(uint64_t (&x)[E], uint64_t* lds, int tid, const Tw* __restrict__ tw,
                                         const LimbConst& c) {
  constexpr int NFULL = LOGN / 4, REM = LOGN % 4;
  if constexpr (P < NFULL) {
    constexpr int LO = REM + 4 * P;
    constexpr int PREV = (P == 0) ? 0 : REM + 4 * (P - 1);
    if constexpr (P > 0 || REM > 0) {
      __syncthreads();
      to_lds<PREV>(lds, x, tid);
      __syncthreads();
      from_lds<LO>(lds, x, tid);
    }
    inv_pass<LOGN, LO, 0, (P == NFULL - 1)>(x, tid, tw, c);
    inv_rest<LOGN, P + 1>(x, lds, tid, tw, c);
  }
}

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / E) void ntt_inv_kernel(uint64_t* __restrict__ polys, uint32_t L,
                                                                   const Tw* __restrict__ tw_all,
                                                                   const LimbConst* __restrict__ lcs) {
  constexpr int N = 1 << LOGN, T = N / E, REM = LOGN % 4;
  __shared__ uint64_t lds[N + N / 16];
  const int tid = threadIdx.x;
  const uint32_t p = blockIdx.x;
  const uint32_t l = p % L;
  uint64_t* a = polys + (size_t)p * N;
  const Tw* tw = tw_all + (size_t)l * N;
  const LimbConst c = lcs[l];
  uint64_t x[E];
  // first mapping: LO = 0, the 16 consecutive words tid*16 + k
  const ulonglong2* src = reinterpret_cast<const ulonglong2*>(a) + tid * (E / 2);
#pragma unroll
  for (int k = 0; k < E / 2; k++) {
    ulonglong2 v = src[k];
    x[2 * k] = v.x;
    x[2 * k + 1] = v.y;
  }
  if constexpr (REM > 0) inv_pass<LOGN, 0, 4 - REM, false>(x, tid, tw, c);
  inv_rest<LOGN, 0>(x, lds, tid, tw, c);
  // last pass used LO = LOGN-4: element j = tid + k*T, values canonical
#pragma unroll
  for (int k = 0; k < E; k++) a[tid + k * T] = x[k];
}

template <int LOGN>
static hipError_t launch_ntt(bool inverse, uint64_t* polys, uint64_t nlimbpolys, uint32_t L, const Tw* tw,
                             const LimbConst* lc, hipStream_t st) {
  constexpr int T = (1 << LOGN) / E;
  // grid.x is limited to 2^31-1 workgroups: split larger batches into chunks
  // of whole RNS polynomials so that blockIdx.x % L stays the limb index
  const uint64_t max_blocks = (1ull << 30) / L * L;
  for (uint64_t off = 0; off < nlimbpolys; off += max_blocks) {
    uint64_t cnt = nlimbpolys - off < max_blocks ? nlimbpolys - off : max_blocks;
    uint64_t* base = polys + off * (1ull << LOGN);
    if (inverse)
      hipLaunchKernelGGL(ntt_inv_kernel<LOGN>, dim3((uint32_t)cnt), dim3(T), 0, st, base, L, tw, lc);
    else
      hipLaunchKernelGGL(ntt_fwd_kernel<LOGN>, dim3((uint32_t)cnt), dim3(T), 0, st, base, L, tw, lc);
  }
  return hipGetLastError();
}

hipError_t ntt_launch(bool inverse, uint32_t logN, uint64_t* polys, uint64_t n_rns_polys, uint32_t L,
                      const Tw* tw, const LimbConst* lc, hipStream_t st) {
  const uint64_t nlp = n_rns_polys * L;
  switch (logN) {
    case 10: return launch_ntt<10>(inverse, polys, nlp, L, tw, lc, st);
    case 11: return launch_ntt<11>(inverse, polys, nlp, L, tw, lc, st);
    case 12: return launch_ntt<12>(inverse, polys, nlp, L, tw, lc, st);
    case 13: return launch_ntt<13>(inverse, polys, nlp, L, tw, lc, st);
    case 14: return launch_ntt<14>(inverse, polys, nlp, L, tw, lc, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace heconv
