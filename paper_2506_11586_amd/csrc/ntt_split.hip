// Forward NTT of a few limb polynomials in two grids, so that more compute
// units share the work: with fewer limb polynomials than compute units the
// one-workgroup-per-polynomial kernel leaves units idle, and each busy unit
// is bound by its own integer issue rate.
//
// For N = 2^n, write j = g + G*i with G = 2^(n-6), i < 64.  The stages on
// bits n-1 .. n-6 (the first six) combine only elements of one residue g,
// and those on bits n-7 .. 0 only elements of one block of G consecutive
// indexes.  Grid A: a workgroup of 128 threads takes 16 consecutive
// residues (1024 elements) and runs the first six stages; seen through the
// index v = i*16 + (g - g0), this is the first six stages of a 1024-point
// transform whose twiddle indexes coincide with the N-point ones.  Grid B:
// a workgroup takes 1024 consecutive elements and runs the remaining
// stages, its twiddle indexes offset by its first element.  Each limb
// polynomial's workgroups of both grids run on one XCD when the count
// allows, so the intermediate stays in that XCD's L2.
#include "kernels.h"
#include "ntt_impl.h"

namespace heconv {

constexpr int SPLIT_T = 128;  // threads per workgroup (8 words each)

// Workgroup b -> (limb polynomial, part).  With W = 8 parts and the count a
// multiple of 8, the parts of polynomial p all have b = p (mod 8).
__device__ __forceinline__ void split_index(uint32_t b, uint32_t nlp, uint32_t W, uint32_t& p, uint32_t& w) {
  if (W == 8 && nlp % 8 == 0) {
    p = (b / 64) * 8 + b % 8;
    w = (b / 8) % 8;
  } else {
    p = b / W;
    w = b % W;
  }
}

template <int LOGN>
__global__ __launch_bounds__(SPLIT_T) void ntt_fwd_split_a(uint64_t* __restrict__ polys_, uint32_t nlp, uint32_t L,
                                                            const Tw* __restrict__ tw_all,
                                                            const LimbConst* __restrict__ lcs) {
  constexpr int G = 1 << (LOGN - 6), W = G / 16;
  __shared__ uint64_t lds[1024 + 1024 / 16];
  uint32_t p, w;
  split_index(blockIdx.x, nlp, W, p, w);
  const uint32_t l = p % L;
  const LimbConst c = lcs[l];
  const Tw* tw = tw_all + (size_t)l * (1 << LOGN);
  gword* a = as_global(polys_) + (size_t)p * (1 << LOGN) + (size_t)w * 16;
  const int tid = threadIdx.x;
  uint64_t x[8];
  // virtual index v = tid + 128k  ->  residue g0 + (v & 15), i = v >> 4
#pragma unroll
  for (int k = 0; k < 8; k++) {
    const int v = tid + 128 * k;
    x[k] = a[(v & 15) + (size_t)G * (v >> 4)];
  }
  fwd_pass<10, 3, 7, 0>(x, tid, tw, c);
  exchange<3, 7, 4>(lds, x, tid);
  fwd_pass<10, 3, 4, 0>(x, tid, tw, c);
#pragma unroll
  for (int k = 0; k < 8; k++) {
    const int v = elem_index<3, 4>(tid, k);
    a[(v & 15) + (size_t)G * (v >> 4)] = x[k];
  }
}

// Remaining stages (bits n-7 .. 0) of one 1024-element block.
template <int LOGN, int P>
__device__ __forceinline__ void split_b_rest(uint64_t (&x)[8], uint64_t* lds, int tid, const Tw* __restrict__ tw,
                                             const LimbConst& c, uint32_t jb) {
  constexpr int NB = LOGN - 6;  // stages in this grid
  constexpr int NFULL = NB / 3, REM = NB % 3;
  if constexpr (P < NFULL) {
    constexpr int LO = NB - 3 * (P + 1);
    if constexpr (P > 0) exchange<3, LO + 3, LO>(lds, x, tid);
    fwd_pass<LOGN, 3, LO, 0>(x, tid, tw, c, jb);
    split_b_rest<LOGN, P + 1>(x, lds, tid, tw, c, jb);
  } else if constexpr (REM > 0) {
    exchange<3, NB - 3 * NFULL, 0>(lds, x, tid);
    fwd_pass<LOGN, 3, 0, 3 - REM>(x, tid, tw, c, jb);
  }
}

template <int LOGN>
__global__ __launch_bounds__(SPLIT_T) void ntt_fwd_split_b(uint64_t* __restrict__ polys_, uint32_t nlp, uint32_t L,
                                                            const Tw* __restrict__ tw_all,
                                                            const LimbConst* __restrict__ lcs) {
  constexpr int W = (1 << LOGN) / 1024, NB = LOGN - 6, LO0 = NB - 3;
  __shared__ uint64_t lds[1024 + 1024 / 16];
  uint32_t p, w;
  split_index(blockIdx.x, nlp, W, p, w);
  const uint32_t l = p % L;
  const LimbConst c = lcs[l];
  const Tw* tw = tw_all + (size_t)l * (1 << LOGN);
  const uint32_t jb = w * 1024;
  gword* a = as_global(polys_) + (size_t)p * (1 << LOGN) + jb;
  const int tid = threadIdx.x;
  uint64_t x[8];
#pragma unroll
  for (int k = 0; k < 8; k++) x[k] = a[elem_index<3, LO0>(tid, k)];
  split_b_rest<LOGN, 0>(x, lds, tid, tw, c, jb);
#pragma unroll
  for (int k = 0; k < 8; k++) x[k] = fwd_canon(x[k], c);
  exchange<3, 0, 7>(lds, x, tid);  // to local index tid + 128k for a coalesced store
#pragma unroll
  for (int k = 0; k < 8; k++) a[tid + 128 * k] = x[k];
}

// Inverse in two grids, the mirror image: grid C takes 1024 consecutive
// elements and runs the stages on bits 0 .. n-7 (within blocks of G), its
// twiddle indexes offset by its first element; grid D takes 16 residues and
// runs the stages on bits n-6 .. n-1 as the last six stages of a 1024-point
// inverse in the index v = i*16 + (g - g0), the top one applying N^-1.
// Values stay in [0, 2q) between the grids; the result is canonical.
template <int LOGN, int P>
__device__ __forceinline__ void inv_split_c_rest(uint64_t (&x)[8], uint64_t* lds, int tid,
                                                 const Tw* __restrict__ tw, const LimbConst& c, uint32_t jb) {
  constexpr int NB = LOGN - 6, NFULL = NB / 3, REM = NB % 3;
  if constexpr (P < NFULL) {
    constexpr int LO = REM + 3 * P;
    constexpr int PREV = (P == 0) ? 0 : REM + 3 * (P - 1);
    if constexpr (P > 0 || REM > 0) exchange<3, PREV, LO>(lds, x, tid);
    inv_pass<LOGN, 3, LO, 0, false>(x, tid, tw, c, jb);
    inv_split_c_rest<LOGN, P + 1>(x, lds, tid, tw, c, jb);
  }
}

template <int LOGN>
__global__ __launch_bounds__(SPLIT_T) void ntt_inv_split_c(uint64_t* __restrict__ polys_, uint32_t nlp, uint32_t L,
                                                            const Tw* __restrict__ tw_all,
                                                            const LimbConst* __restrict__ lcs) {
  constexpr int W = (1 << LOGN) / 1024, NB = LOGN - 6, REM = NB % 3, NFULL = NB / 3;
  constexpr int LAST_LO = REM + 3 * (NFULL - 1);
  __shared__ uint64_t lds[1024 + 1024 / 16];
  uint32_t p, w;
  split_index(blockIdx.x, nlp, W, p, w);
  const uint32_t l = p % L;
  const LimbConst c = lcs[l];
  const Tw* tw = tw_all + (size_t)l * (1 << LOGN);
  const uint32_t jb = w * 1024;
  gword* a = as_global(polys_) + (size_t)p * (1 << LOGN) + jb;
  const int tid = threadIdx.x;
  uint64_t x[8];
#pragma unroll
  for (int k = 0; k < 8; k++) x[k] = a[tid + 128 * k];  // local index tid + 128k: the mapping at 7
  exchange<3, 7, 0>(lds, x, tid);
  if constexpr (REM > 0) inv_pass<LOGN, 3, 0, 3 - REM, false>(x, tid, tw, c, jb);
  inv_split_c_rest<LOGN, 0>(x, lds, tid, tw, c, jb);
#pragma unroll
  for (int k = 0; k < 8; k++) a[elem_index<3, LAST_LO>(tid, k)] = x[k];
}

template <int LOGN>
__global__ __launch_bounds__(SPLIT_T) void ntt_inv_split_d(uint64_t* __restrict__ polys_, uint32_t nlp, uint32_t L,
                                                            const Tw* __restrict__ tw_all,
                                                            const LimbConst* __restrict__ lcs) {
  constexpr int G = 1 << (LOGN - 6), W = G / 16;
  __shared__ uint64_t lds[1024 + 1024 / 16];
  uint32_t p, w;
  split_index(blockIdx.x, nlp, W, p, w);
  const uint32_t l = p % L;
  const LimbConst c = lcs[l];
  const Tw* tw = tw_all + (size_t)l * (1 << LOGN);
  gword* a = as_global(polys_) + (size_t)p * (1 << LOGN) + (size_t)w * 16;
  const int tid = threadIdx.x;
  uint64_t x[8];
  // virtual index v -> residue g0 + (v & 15), i = v >> 4
#pragma unroll
  for (int k = 0; k < 8; k++) {
    const int v = elem_index<3, 4>(tid, k);
    x[k] = a[(v & 15) + (size_t)G * (v >> 4)];
  }
  inv_pass<10, 3, 4, 0, false>(x, tid, tw, c);
  exchange<3, 4, 7>(lds, x, tid);
  inv_pass<10, 3, 7, 0, true>(x, tid, tw, c);
#pragma unroll
  for (int k = 0; k < 8; k++) {
    const int v = tid + 128 * k;
    a[(v & 15) + (size_t)G * (v >> 4)] = x[k];
  }
}

template <int LOGN>
static hipError_t inv_split_go(uint64_t* polys, uint64_t nlp, uint32_t L, const Tw* tw, const LimbConst* lc,
                               hipStream_t st) {
  constexpr uint32_t W = (1 << LOGN) / 1024;
  const uint64_t blocks = nlp * W;
  if (blocks > grid_max_blocks(SPLIT_T)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((ntt_inv_split_c<LOGN>), dim3((uint32_t)blocks), dim3(SPLIT_T), 0, st, polys, (uint32_t)nlp, L,
                     tw, lc);
  hipLaunchKernelGGL((ntt_inv_split_d<LOGN>), dim3((uint32_t)blocks), dim3(SPLIT_T), 0, st, polys, (uint32_t)nlp, L,
                     tw, lc);
  return hipGetLastError();
}

// At N = 2^12 one workgroup per polynomial is faster at every count.
bool ntt_inv_split_supported(uint32_t logN) { return logN == 13 || logN == 14; }

hipError_t ntt_inv_split_launch(uint32_t logN, uint64_t* polys, uint64_t n_rns_polys, uint32_t L, const Tw* tw,
                                const LimbConst* lc, hipStream_t st) {
  const uint64_t nlp = n_rns_polys * L;
  if (nlp == 0) return hipSuccess;
  switch (logN) {
    case 13: return inv_split_go<13>(polys, nlp, L, tw, lc, st);
    case 14: return inv_split_go<14>(polys, nlp, L, tw, lc, st);
    default: return hipErrorInvalidValue;
  }
}

template <int LOGN>
static hipError_t split_go(uint64_t* polys, uint64_t nlp, uint32_t L, const Tw* tw, const LimbConst* lc,
                           hipStream_t st) {
  constexpr uint32_t W = (1 << LOGN) / 1024;
  const uint64_t blocks = nlp * W;
  if (blocks > grid_max_blocks(SPLIT_T)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((ntt_fwd_split_a<LOGN>), dim3((uint32_t)blocks), dim3(SPLIT_T), 0, st, polys, (uint32_t)nlp, L,
                     tw, lc);
  hipLaunchKernelGGL((ntt_fwd_split_b<LOGN>), dim3((uint32_t)blocks), dim3(SPLIT_T), 0, st, polys, (uint32_t)nlp, L,
                     tw, lc);
  return hipGetLastError();
}

bool ntt_fwd_split_supported(uint32_t logN) { return logN >= 12 && logN <= 14; }

hipError_t ntt_fwd_split_launch(uint32_t logN, uint64_t* polys, uint64_t n_rns_polys, uint32_t L, const Tw* tw,
                                const LimbConst* lc, hipStream_t st) {
  const uint64_t nlp = n_rns_polys * L;
  if (nlp == 0) return hipSuccess;
  switch (logN) {
    case 12: return split_go<12>(polys, nlp, L, tw, lc, st);
    case 13: return split_go<13>(polys, nlp, L, tw, lc, st);
    case 14: return split_go<14>(polys, nlp, L, tw, lc, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace heconv
