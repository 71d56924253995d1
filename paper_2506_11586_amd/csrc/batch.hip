// Batch executor kernels: the three steps of many layer solves of uneven
// shape, each as one grid over a work list (one workgroup per item):
// forward NTT of every input limb polynomial of every job, every MAC tile of
// every job, inverse NTT of every output limb polynomial.  Kernel
// boundaries order the steps; no workgroup waits on another.
#include "batch.h"
#include "mac_impl.h"
#include "mac_grid.h"
#include "mac_stream.h"
#include "ntt_impl.h"

namespace heconv {

template <int LOGN, int LOGE>
__global__ __launch_bounds__((1 << LOGN) >> LOGE) void batch_fwd_kernel(const BatchItem* __restrict__ items,
                                                                         const BatchJob* __restrict__ jobs,
                                                                         const Tw* __restrict__ tw,
                                                                         const LimbConst* __restrict__ lcs,
                                                                         uint32_t L) {
  constexpr int N = 1 << LOGN;
  __shared__ uint64_t lds[N + N / 16];
  const BatchItem it = items[blockIdx.x];
  gword* in = as_global(jobs[it.job].in);
  const uint32_t l = it.idx % L;
  const LimbConst c = lcs[l];
  ntt_fwd_poly<LOGN, LOGE>(in + (size_t)it.idx * N, tw + (size_t)l * N, c, lds, threadIdx.x);
}

template <int LOGN, int LOGE>
__global__ __launch_bounds__((1 << LOGN) >> LOGE) void batch_inv_kernel(const BatchItem* __restrict__ items,
                                                                         const BatchJob* __restrict__ jobs,
                                                                         const Tw* __restrict__ tw,
                                                                         const LimbConst* __restrict__ lcs,
                                                                         uint32_t L) {
  constexpr int N = 1 << LOGN;
  __shared__ uint64_t lds[N + N / 16];
  const BatchItem it = items[blockIdx.x];
  gword* out = as_global(jobs[it.job].out);
  const uint32_t l = it.idx % L;
  const LimbConst c = lcs[l];
  ntt_inv_poly<LOGN, LOGE, true>(out + (size_t)it.idx * N, tw + (size_t)l * N, c, lds, threadIdx.x);
}

// MAC work list: the host interleaves eight per-XCD lists (workgroup b runs
// on XCD b mod 8), each holding that XCD's share of every job's tiles --
// a contiguous range of k-chunks, whose tiles share input and weight words
// in the XCD's L2 -- so every XCD gets an equal slice of every job.  Padding
// entries (job = BATCH_NO_JOB) end at once.
template <int MT, int RT>
__global__ __launch_bounds__(BATCH_MAC_THREADS) void batch_mac_kernel(const BatchItem* __restrict__ items,
                                                                       const BatchJob* __restrict__ jobs,
                                                                       const LimbConst* __restrict__ lcs,
                                                                       uint32_t L, uint32_t N) {
  const BatchItem it = items[blockIdx.x];
  if (it.job == BATCH_NO_JOB) return;
  const BatchJob jd = jobs[it.job];
  const uint32_t per_chunk = jd.n_mt * jd.n_rt;
  const uint32_t kc = it.idx / per_chunk;
  const uint32_t mt = (it.idx % per_chunk) / jd.n_rt;
  const uint32_t rt = it.idx % jd.n_rt;
  const LimbConst c = lcs[kc / (N / BATCH_MAC_THREADS)];
  mac_tile<MT, RT, BATCH_MAC_THREADS>(as_global(jd.in), as_global(jd.w), as_global(jd.out), jd.CB, jd.S, jd.M, L, N,
                                      jd.rows, kc, mt, rt, c, threadIdx.x);
}

// Streamed MAC: workgroup b runs tiles mitems[b*per_wg ..] (see mac_stream).
template <int MT, int RT, int P, bool PM>
__global__ __launch_bounds__(BATCH_MAC_THREADS) void batch_mac_stream_kernel(const MacItem* __restrict__ items,
                                                                              uint32_t per_wg,
                                                                              const BatchJob* __restrict__ jobs,
                                                                              const LimbConst* __restrict__ lcs,
                                                                              uint32_t L, uint32_t logN) {
  __shared__ uint64_t lds[mac_dma_lds_words<MT, RT, BATCH_MAC_THREADS, P>()];
  const MacListSrc src{items + (uint64_t)blockIdx.x * per_wg, per_wg, jobs};
  mac_stream<MT, RT, BATCH_MAC_THREADS, P, PM>(src, lcs, L, logN, lds, threadIdx.x);
}

template <int LOGN, int LOGE>
static void launch_ntt_phase(bool inverse, const BatchPhase& p, const BatchArgs& a, hipStream_t st) {
  constexpr uint32_t T = (1u << LOGN) >> LOGE;
  if (inverse)
    hipLaunchKernelGGL((batch_inv_kernel<LOGN, LOGE>), dim3(p.n), dim3(T), 0, st, p.items, a.jobs, a.twi, a.lcs, a.L);
  else
    hipLaunchKernelGGL((batch_fwd_kernel<LOGN, LOGE>), dim3(p.n), dim3(T), 0, st, p.items, a.jobs, a.twf, a.lcs, a.L);
}

template <int LOGN>
static hipError_t ntt_phase(bool inverse, uint32_t loge, const BatchPhase& p, const BatchArgs& a, hipStream_t st) {
  if constexpr (LOGN <= 13) {
    if (loge == 3) {
      launch_ntt_phase<LOGN, 3>(inverse, p, a, st);
      return hipGetLastError();
    }
  }
  launch_ntt_phase<LOGN, 4>(inverse, p, a, st);
  return hipGetLastError();
}

static hipError_t ntt_phase_n(bool inverse, uint32_t logN, uint32_t loge, const BatchPhase& p, const BatchArgs& a,
                              hipStream_t st) {
  if (p.n == 0) return hipSuccess;
  switch (logN) {
    case 10: return ntt_phase<10>(inverse, loge, p, a, st);
    case 11: return ntt_phase<11>(inverse, loge, p, a, st);
    case 12: return ntt_phase<12>(inverse, loge, p, a, st);
    case 13: return ntt_phase<13>(inverse, loge, p, a, st);
    case 14: return ntt_phase<14>(inverse, loge, p, a, st);
    default: return hipErrorInvalidValue;
  }
}

template <int MT, int RT>
static hipError_t mac_regs(const BatchPhase& p, const BatchArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((batch_mac_kernel<MT, RT>), dim3(p.n), dim3(BATCH_MAC_THREADS), 0, st, p.items, a.jobs, a.lcs,
                     a.L, a.N);
  return hipGetLastError();
}

// Streamed MAC on a 2x2 wave grid: workgroup b runs tiles mitems[b*per_wg ..]
// (see mac_grid).
template <int MT, int RT, int P, bool PM>
__global__ __launch_bounds__(BATCH_MAC_THREADS) void batch_mac_grid_kernel(const MacItem* __restrict__ items,
                                                                            uint32_t per_wg,
                                                                            const BatchJob* __restrict__ jobs,
                                                                            const LimbConst* __restrict__ lcs,
                                                                            uint32_t L, uint32_t logN) {
  __shared__ uint64_t lds[P * MacGridShape<MT, RT>::ROWS * 64];
  const MacListSrc src{items + (uint64_t)blockIdx.x * per_wg, per_wg, jobs};
  mac_grid<MT, RT, BATCH_MAC_THREADS, P, PM>(src, lcs, L, logN, lds, threadIdx.x);
}

template <int MT, int RT, int P>
static void mac_streamed_p(const BatchPhase& p, const BatchArgs& a, hipStream_t st) {
  if (a.mac_grid && a.all_pm)
    hipLaunchKernelGGL((batch_mac_grid_kernel<MT, RT, P, true>), dim3(p.n), dim3(BATCH_MAC_THREADS), 0, st, p.mitems,
                       p.per_wg, a.jobs, a.lcs, a.L, a.logN);
  else if (a.mac_grid)
    hipLaunchKernelGGL((batch_mac_grid_kernel<MT, RT, P, false>), dim3(p.n), dim3(BATCH_MAC_THREADS), 0, st,
                       p.mitems, p.per_wg, a.jobs, a.lcs, a.L, a.logN);
  else if (a.all_pm)
    hipLaunchKernelGGL((batch_mac_stream_kernel<MT, RT, P, true>), dim3(p.n), dim3(BATCH_MAC_THREADS), 0, st, p.mitems,
                       p.per_wg, a.jobs, a.lcs, a.L, a.logN);
  else
    hipLaunchKernelGGL((batch_mac_stream_kernel<MT, RT, P, false>), dim3(p.n), dim3(BATCH_MAC_THREADS), 0, st,
                       p.mitems, p.per_wg, a.jobs, a.lcs, a.L, a.logN);
}

template <int MT, int RT>
static hipError_t mac_streamed(const BatchPhase& p, const BatchArgs& a, hipStream_t st) {
  if (a.mac_lds == 2)
    mac_streamed_p<MT, RT, 2>(p, a, st);
  else if (a.mac_lds == 3)
    mac_streamed_p<MT, RT, 3>(p, a, st);
  else if (a.mac_lds == 4)
    mac_streamed_p<MT, RT, 4>(p, a, st);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

static hipError_t mac_phase(const BatchPhase& p, const BatchArgs& a, hipStream_t st) {
  if (p.n == 0) return hipSuccess;
  const uint32_t mt = a.mac_mt, rt = a.mac_rt;
  if (a.mac_lds == 0) {
    if (mt == 4 && rt == 4) return mac_regs<4, 4>(p, a, st);
    if (mt == 4 && rt == 2) return mac_regs<4, 2>(p, a, st);
    if (mt == 2 && rt == 4) return mac_regs<2, 4>(p, a, st);
    if (mt == 2 && rt == 2) return mac_regs<2, 2>(p, a, st);
    return hipErrorInvalidValue;
  }
  if (mt == 4 && rt == 4) return mac_streamed<4, 4>(p, a, st);
  if (a.mac_grid && (mt == 8 || rt == 8)) return hipErrorInvalidValue;
  if (mt == 8 && rt == 4) return mac_streamed<8, 4>(p, a, st);
  if (mt == 6 && rt == 4) return mac_streamed<6, 4>(p, a, st);
  if (mt == 4 && rt == 8) return mac_streamed<4, 8>(p, a, st);
  if (mt == 4 && rt == 2) return mac_streamed<4, 2>(p, a, st);
  if (mt == 2 && rt == 4) return mac_streamed<2, 4>(p, a, st);
  if (mt == 2 && rt == 2) return mac_streamed<2, 2>(p, a, st);
  return hipErrorInvalidValue;
}

bool batch_tile_supported(uint32_t mt, uint32_t rt, uint32_t lds) {
  const bool base = (mt == 4 && rt == 4) || (mt == 4 && rt == 2) || (mt == 2 && rt == 4) || (mt == 2 && rt == 2);
  return base || (lds >= 2 && ((mt == 6 && rt == 4) || (mt == 8 && rt == 4) || (mt == 4 && rt == 8)));
}

hipError_t batch_phase(const BatchChain& ch, const BatchArgs& a, int phase, hipStream_t st) {
  if (phase == 0) return ntt_phase_n(false, a.logN, ch.fwd.n < 512 ? a.loge_small : a.loge_large, ch.fwd, a, st);
  if (phase == 1) return mac_phase(ch.mac, a, st);
  return ntt_phase_n(true, a.logN, ch.inv.n < 512 ? a.loge_small : a.loge_large, ch.inv, a, st);
}

hipError_t batch_chain(const BatchChain& ch, const BatchArgs& a, hipStream_t st) {
  for (int p = 0; p < 3; p++)
    if (hipError_t e = batch_phase(ch, a, p, st); e != hipSuccess) return e;
  return hipSuccess;
}

}  // namespace heconv
