// Batch executor: one persistent kernel drains a work list that mixes the
// three steps of many layer solves of uneven shape.
//
// Work items, in list order: FWD (forward NTT of one input limb
// polynomial of a job), MAC (one MAC tile of a job), INV (inverse NTT of one
// output limb polynomial).  Workgroups take items in list order from an
// atomic head counter.  A job's MAC items wait until all its FWD items are
// done, its INV items until all its MAC items are done; the host builds the
// list so that every item's prerequisites come earlier in it, and every
// earlier item has been taken by a running workgroup that never waits on a
// later one, so the waits always end.  Each wait is nevertheless bounded: on
// timeout the workgroup raises an error flag and carries on.
//
// Completion signals use agent-scope release fences (and the waiter an
// agent-scope acquire fence), which on gfx950 write back / invalidate the
// per-XCD L2 so that data written on one XCD is seen on another.
#include "batch.h"
#include "mac_impl.h"
#include "ntt_impl.h"

namespace heconv {

// Wall-clock bound of one dependency wait, in ticks of the 100 MHz
// s_memrealtime counter (1 s).
constexpr uint64_t WAIT_TICKS = 100000000ull;

// A wait ends when the count is reached; when spin_limit polls or
// WAIT_TICKS have passed (it then raises the error flag and records the
// count it saw and the target); or as soon as any other wait has raised the
// flag -- so a failed launch drains in about a second instead of hanging.
// Counters live on separate 256-byte lines (CTR_STRIDE words apart).
__device__ __forceinline__ void wait_count(uint32_t* cnt, uint32_t target, uint32_t* err, uint32_t spin_limit,
                                           int tid) {
  if (tid == 0) {
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (uint32_t spins = 0;; spins++) {
      const uint32_t v = __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (v >= target) break;
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
      if (spins + 1 >= spin_limit || __builtin_amdgcn_s_memrealtime() - t0 > WAIT_TICKS) {
        if (__hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
          __hip_atomic_store(err + 1, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(err + 2, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        break;
      }
      __builtin_amdgcn_s_sleep(8);
    }
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ __forceinline__ void signal_count(uint32_t* cnt, int tid) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (tid == 0) __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Counter words (CTR_STRIDE apart): [0] head, [1] error flag (+1 count seen,
// +2 target of the first timed-out wait), [2 + 2j] FWD items of job j done,
// [3 + 2j] MAC items of job j done.
template <int LOGN, int MT, int RT>
__global__ __launch_bounds__((1 << LOGN) / 16, 4) void batch_kernel(const BatchItem* __restrict__ items,
                                                                     uint32_t n_items,
                                                                     const BatchJob* __restrict__ jobs,
                                                                     uint32_t* ctr, const Tw* __restrict__ twf,
                                                                     const Tw* __restrict__ twi,
                                                                     const LimbConst* __restrict__ lcs, uint32_t L,
                                                                     uint32_t spin_limit) {
  constexpr int N = 1 << LOGN, T = N / 16;
  __shared__ uint64_t lds[N + N / 16];
  __shared__ uint32_t s_it;
  const int tid = threadIdx.x;
  uint32_t* head = ctr;
  uint32_t* err = ctr + CTR_STRIDE;
  for (;;) {
    if (tid == 0) s_it = __hip_atomic_fetch_add(head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint32_t it = s_it;
    __syncthreads();
    if (it >= n_items) break;
    const BatchItem item = items[it];
    const uint32_t j = item.jt >> 2, type = item.jt & 3u;
    const BatchJob jd = jobs[j];
    if (type == ITEM_FWD) {
      const uint32_t l = item.idx % L;
      ntt_fwd_poly<LOGN, 4>(jd.in + (size_t)item.idx * N, twf + (size_t)l * N, lcs[l].q, lcs[l].two_q, lds, tid);
      signal_count(ctr + (2 + 2 * j) * CTR_STRIDE, tid);
    } else if (type == ITEM_MAC) {
      wait_count(ctr + (2 + 2 * j) * CTR_STRIDE, jd.n_fwd, err, spin_limit, tid);
      const uint32_t per_chunk = jd.n_mt * jd.n_rt;
      const uint32_t kc = item.idx / per_chunk;
      const uint32_t mt = (item.idx % per_chunk) / jd.n_rt;
      const uint32_t rt = item.idx % jd.n_rt;
      const LimbConst c = lcs[kc / (N / T)];
      mac_tile<MT, RT, T>(jd.in, jd.w, jd.out, jd.CB, jd.S, jd.M, L, N, jd.rows, kc, mt, rt, c, tid);
      signal_count(ctr + (3 + 2 * j) * CTR_STRIDE, tid);
    } else {
      wait_count(ctr + (3 + 2 * j) * CTR_STRIDE, jd.n_mac, err, spin_limit, tid);
      const uint32_t l = item.idx % L;
      const LimbConst c = lcs[l];
      ntt_inv_poly<LOGN, 4>(jd.out + (size_t)item.idx * N, twi + (size_t)l * N, c, lds, tid);
    }
  }
}

__global__ void batch_reset_kernel(uint32_t* ctr, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) ctr[i] = 0;
}

template <int LOGN>
static const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&batch_kernel<LOGN, BATCH_MT, BATCH_RT>);
}

hipError_t batch_occupancy(uint32_t logN, int* blocks_per_cu) {
  const void* f = nullptr;
  switch (logN) {
    case 10: f = kernel_ptr<10>(); break;
    case 11: f = kernel_ptr<11>(); break;
    case 12: f = kernel_ptr<12>(); break;
    case 13: f = kernel_ptr<13>(); break;
    case 14: f = kernel_ptr<14>(); break;
    default: return hipErrorInvalidValue;
  }
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, (1 << logN) / 16, 0);
}

template <int LOGN>
static void launch_batch(const BatchLaunch& a, hipStream_t st) {
  hipLaunchKernelGGL((batch_kernel<LOGN, BATCH_MT, BATCH_RT>), dim3(a.grid), dim3((1 << LOGN) / 16), 0, st, a.items,
                     a.n_items, a.jobs, a.ctr, a.twf, a.twi, a.lcs, a.L, a.spin_limit);
}

hipError_t batch_launch(uint32_t logN, const BatchLaunch& a, hipStream_t st) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(256), 0, st, a.ctr, a.n_ctr);
  switch (logN) {
    case 10: launch_batch<10>(a, st); break;
    case 11: launch_batch<11>(a, st); break;
    case 12: launch_batch<12>(a, st); break;
    case 13: launch_batch<13>(a, st); break;
    case 14: launch_batch<14>(a, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace heconv
