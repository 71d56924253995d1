// Standalone NTT / inverse NTT kernels: one workgroup per limb polynomial.
// The transform itself is in ntt_impl.h.
#include "kernels.h"
#include "ntt_impl.h"

namespace heconv {

template <int LOGN, int LOGE>
__global__ __launch_bounds__((1 << LOGN) >> LOGE) void ntt_fwd_kernel(uint64_t* __restrict__ polys, uint32_t L,
                                                                       const Tw* __restrict__ tw_all,
                                                                       const LimbConst* __restrict__ lcs) {
  constexpr int N = 1 << LOGN;
  __shared__ uint64_t lds[N + N / 16];
  const uint32_t p = blockIdx.x;
  const uint32_t l = p % L;
  const LimbConst c = lcs[l];
  ntt_fwd_poly<LOGN, LOGE>(as_global(polys) + (size_t)p * N, tw_all + (size_t)l * N, c, lds, threadIdx.x);
}

template <int LOGN, int LOGE, bool NT>
__global__ __launch_bounds__((1 << LOGN) >> LOGE) void ntt_inv_kernel(uint64_t* __restrict__ polys, uint32_t L,
                                                                       const Tw* __restrict__ tw_all,
                                                                       const LimbConst* __restrict__ lcs) {
  constexpr int N = 1 << LOGN;
  __shared__ uint64_t lds[N + N / 16];
  const uint32_t p = blockIdx.x;
  const uint32_t l = p % L;
  const LimbConst c = lcs[l];
  ntt_inv_poly<LOGN, LOGE, NT>(as_global(polys) + (size_t)p * N, tw_all + (size_t)l * N, c, lds, threadIdx.x);
}

template <int LOGN, int LOGE>
static hipError_t launch_ntt(bool inverse, uint64_t* polys, uint64_t nlimbpolys, uint32_t L, const Tw* tw,
                             const LimbConst* lc, hipStream_t st, bool nt) {
  constexpr int T = (1 << LOGN) >> LOGE;
  // one launch covers at most 2^32 - 1 work-items: split larger batches into
  // chunks of whole RNS polynomials so that blockIdx.x % L stays the limb index
  const uint64_t max_blocks = grid_max_blocks(T) / L * L;
  for (uint64_t off = 0; off < nlimbpolys; off += max_blocks) {
    uint64_t cnt = nlimbpolys - off < max_blocks ? nlimbpolys - off : max_blocks;
    uint64_t* base = polys + off * (1ull << LOGN);
    if (inverse && nt)
      hipLaunchKernelGGL((ntt_inv_kernel<LOGN, LOGE, true>), dim3((uint32_t)cnt), dim3(T), 0, st, base, L, tw, lc);
    else if (inverse)
      hipLaunchKernelGGL((ntt_inv_kernel<LOGN, LOGE, false>), dim3((uint32_t)cnt), dim3(T), 0, st, base, L, tw, lc);
    else
      hipLaunchKernelGGL((ntt_fwd_kernel<LOGN, LOGE>), dim3((uint32_t)cnt), dim3(T), 0, st, base, L, tw, lc);
  }
  return hipGetLastError();
}

template <int LOGN>
static hipError_t launch_ntt_e(bool inverse, uint32_t loge, uint64_t* polys, uint64_t nlp, uint32_t L,
                               const Tw* tw, const LimbConst* lc, hipStream_t st, bool nt) {
  if constexpr (LOGN <= 13) {  // 8 words per thread needs N/8 <= 1024 threads
    if (loge == 3) return launch_ntt<LOGN, 3>(inverse, polys, nlp, L, tw, lc, st, nt);
  }
  return launch_ntt<LOGN, 4>(inverse, polys, nlp, L, tw, lc, st, nt);
}

hipError_t ntt_launch(bool inverse, uint32_t logN, uint32_t loge, uint64_t* polys, uint64_t n_rns_polys,
                      uint32_t L, const Tw* tw, const LimbConst* lc, hipStream_t st, bool nt) {
  const uint64_t nlp = n_rns_polys * L;
  switch (logN) {
    case 10: return launch_ntt_e<10>(inverse, loge, polys, nlp, L, tw, lc, st, nt);
    case 11: return launch_ntt_e<11>(inverse, loge, polys, nlp, L, tw, lc, st, nt);
    case 12: return launch_ntt_e<12>(inverse, loge, polys, nlp, L, tw, lc, st, nt);
    case 13: return launch_ntt_e<13>(inverse, loge, polys, nlp, L, tw, lc, st, nt);
    case 14: return launch_ntt_e<14>(inverse, loge, polys, nlp, L, tw, lc, st, nt);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace heconv
