// Integer-VALU rate probes: the measured ceilings that the transform and MAC
// kernels are compared against.  Each probe runs one instruction (or one
// kernel's arithmetic, on operands held in registers, with no memory traffic
// in its loop) over a grid that fills every compute unit, and reports
// operations per second from HIP events.
//
//  HE_PROBE_MAD_U64_U32  v_mad_u64_u32 (32x32+64 -> 64), lane operations/s
//  HE_PROBE_MUL_HI_U32   v_mul_hi_u32, lane operations/s
//  HE_PROBE_MUL_LO_U32   v_mul_lo_u32, lane operations/s
//  HE_PROBE_ADD_U32      v_add_u32 (a full-rate reference), lane operations/s
//  HE_PROBE_MAC_MIX      the batch MAC's channel-block step for its 6x4 tile
//                        (30-bit splits, four multiply-adds per product into
//                        three accumulators, one carry per 8 blocks),
//                        products/s
//  HE_PROBE_INTT_MIX     the inverse transform's butterfly (lazy sum below 3q,
//                        mul_shoup_2q of the difference), butterflies/s
//  HE_PROBE_NTT_MIX      the forward transform's butterfly, butterflies/s
#include <hip/hip_runtime.h>

#include "ctx.h"
#include "heconv_probe.h"
#include "mac_impl.h"
#include "modarith.h"

namespace heconv {
namespace {

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_UNROLL = 16;

// Eight independent chains per thread keep the pipeline full.  Every
// operation's operand is the previous result of its chain, so the compiler
// cannot combine the unrolled steps.
__global__ __launch_bounds__(PROBE_THREADS) void probe_mad_kernel(const uint32_t* __restrict__ seed, uint64_t* out,
                                                                  uint32_t iters) {
  const uint32_t t = blockIdx.x * PROBE_THREADS + threadIdx.x;
  const uint32_t b = seed[(threadIdx.x + 7) & 63] | 1u;
  uint64_t acc[8];
#pragma unroll
  for (int i = 0; i < 8; i++) acc[i] = (uint64_t)(seed[(threadIdx.x + i) & 63] + t) << 7;
  for (uint32_t it = 0; it < iters; it++) {
#pragma unroll
    for (int u = 0; u < PROBE_UNROLL; u++)
#pragma unroll
      for (int i = 0; i < 8; i++) acc[i] = (uint64_t)(uint32_t)acc[i] * b + acc[i];  // v_mad_u64_u32
  }
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) s ^= acc[i];
  out[t] = s;
}

__global__ __launch_bounds__(PROBE_THREADS) void probe_mulhi_kernel(const uint32_t* __restrict__ seed, uint64_t* out,
                                                                    uint32_t iters) {
  const uint32_t t = blockIdx.x * PROBE_THREADS + threadIdx.x;
  const uint32_t b = seed[(threadIdx.x + 7) & 63] | 1u;
  uint32_t x[8];
#pragma unroll
  for (int i = 0; i < 8; i++) x[i] = seed[(threadIdx.x + i) & 63] + t;
  for (uint32_t it = 0; it < iters; it++) {
#pragma unroll
    for (int u = 0; u < PROBE_UNROLL; u++)
#pragma unroll
      for (int i = 0; i < 8; i++) x[i] = __umulhi(x[i], b);
  }
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) s ^= x[i];
  out[t] = s;
}

// Pairs of chains multiply each other: x = x*y, then y = y*x.
__global__ __launch_bounds__(PROBE_THREADS) void probe_mullo_kernel(const uint32_t* __restrict__ seed, uint64_t* out,
                                                                    uint32_t iters) {
  const uint32_t t = blockIdx.x * PROBE_THREADS + threadIdx.x;
  uint32_t x[8];
#pragma unroll
  for (int i = 0; i < 8; i++) x[i] = (seed[(threadIdx.x + i) & 63] + t) | 1u;
  for (uint32_t it = 0; it < iters; it++) {
#pragma unroll
    for (int u = 0; u < PROBE_UNROLL; u++)
#pragma unroll
      for (int i = 0; i < 8; i++) x[i] = x[i] * x[i ^ 1];  // v_mul_lo_u32
  }
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) s ^= x[i];
  out[t] = s;
}

// Each chain adds its neighbour: no two steps combine.
__global__ __launch_bounds__(PROBE_THREADS) void probe_add_kernel(const uint32_t* __restrict__ seed, uint64_t* out,
                                                                  uint32_t iters) {
  const uint32_t t = blockIdx.x * PROBE_THREADS + threadIdx.x;
  uint32_t x[8];
#pragma unroll
  for (int i = 0; i < 8; i++) x[i] = seed[(threadIdx.x + i) & 63] + t;
  for (uint32_t it = 0; it < iters; it++) {
#pragma unroll
    for (int u = 0; u < PROBE_UNROLL; u++)
#pragma unroll
      for (int i = 0; i < 8; i++) x[i] = x[i] + x[(i + 1) & 7];  // v_add_u32
  }
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) s ^= x[i];
  out[t] = s;
}

// The batch MAC's compute for its default 6x4 tile (mac_stream): per
// iteration 8 channel blocks of 30-bit splits and four multiply-adds per
// product into three accumulators, then the carry of every (m, row) pair
// (fold3_pm of the context's first prime, the unreduced value seeding a00)
// -- the arithmetic of one 8-block chunk without its loads.
__global__ __launch_bounds__(PROBE_THREADS) void probe_mac_kernel(const uint64_t* __restrict__ seed, uint64_t* out,
                                                                  uint32_t iters, const LimbConst* __restrict__ lcs) {
  constexpr int MT = 6, RT = 4;
  const uint32_t t = blockIdx.x * PROBE_THREADS + threadIdx.x;
  const LimbConst c = lcs[0];
  const uint32_t delta = (uint32_t)c.pmd, two30 = (uint32_t)c.c30;
  uint64_t xr[RT], wr[MT];
#pragma unroll
  for (int i = 0; i < RT; i++) xr[i] = (seed[(threadIdx.x + i) & 63] + t) % c.q;
#pragma unroll
  for (int j = 0; j < MT; j++) wr[j] = (seed[(threadIdx.x + 5 * j + 11) & 63] + t) % c.q;
  uint64_t a00[MT][RT], am[MT][RT], a11[MT][RT];
#pragma unroll
  for (int j = 0; j < MT; j++)
#pragma unroll
    for (int i = 0; i < RT; i++) a00[j][i] = am[j][i] = a11[j][i] = 0;
  for (uint32_t it = 0; it < iters; it++) {
    for (int cb = 0; cb < 8; cb++) {
      Half30 xs[RT];
#pragma unroll
      for (int i = 0; i < RT; i++) xs[i] = split30(xr[i]);
#pragma unroll
      for (int j = 0; j < MT; j++) {
        const Half30 ws = split30(wr[j]);
#pragma unroll
        for (int i = 0; i < RT; i++) {
          a00[j][i] += (uint64_t)xs[i].lo * ws.lo;
          am[j][i] += (uint64_t)xs[i].lo * ws.hi;
          am[j][i] += (uint64_t)xs[i].hi * ws.lo;
          a11[j][i] += (uint64_t)xs[i].hi * ws.hi;
        }
      }
      // the next block's operands count as new values (no arithmetic), so
      // every block splits its operands again as the kernel does
      __asm__ volatile("" : "+v"(xr[0]), "+v"(xr[1]), "+v"(xr[2]), "+v"(xr[3]));
      __asm__ volatile("" : "+v"(wr[0]), "+v"(wr[1]), "+v"(wr[2]), "+v"(wr[3]), "+v"(wr[4]), "+v"(wr[5]));
    }
#pragma unroll
    for (int j = 0; j < MT; j++)
#pragma unroll
      for (int i = 0; i < RT; i++) {
        a00[j][i] = fold3_pm<false>(a00[j][i], am[j][i], a11[j][i], delta, two30);
        am[j][i] = a11[j][i] = 0;
      }
  }
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < MT; j++)
#pragma unroll
    for (int i = 0; i < RT; i++) s ^= a00[j][i];
  out[t] = s;
}

// Eight independent butterflies per thread, operands and twiddles in
// registers; the values stay in the transforms' lazy ranges.
template <bool INVERSE>
__global__ __launch_bounds__(PROBE_THREADS) void probe_bfly_kernel(const uint64_t* __restrict__ seed, uint64_t* out,
                                                                   uint32_t iters, const LimbConst* __restrict__ lcs) {
  const uint32_t t = blockIdx.x * PROBE_THREADS + threadIdx.x;
  const LimbConst c = lcs[0];
  uint64_t x[16];
#pragma unroll
  for (int i = 0; i < 16; i++) x[i] = (seed[(threadIdx.x + i) & 63] + t) % c.q;
  // a twiddle with its scale-2^63 Shoup quotient: 2^64 mod q from the constants
  const uint64_t w = c.r64, wsh = c.r64_sh63;
  for (uint32_t it = 0; it < iters; it++) {
#pragma unroll
    for (int u = 0; u < PROBE_UNROLL / 4; u++)
#pragma unroll
      for (int e = 0; e < 8; e++) {
        const int k0 = e, k1 = e + 8;
        if (INVERSE) {
          const uint64_t X = x[k0], Y = x[k1];
          x[k0] = csub_neg(X + Y, c.neg3q);
          x[k1] = mul_shoup_2q(X - Y + c.three_q, w, wsh, c.neg2q);
        } else {
          const uint64_t X = csub_neg(x[k0], c.neg3q);
          const uint64_t T = mul_shoup_2q(x[k1], w, wsh, c.neg2q);
          x[k0] = X + T;  // [0, 6q), brought back by the next csub_neg
          x[k1] = X - T + c.three_q;
        }
      }
  }
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < 16; i++) s ^= x[i];
  out[t] = s;
}

}  // namespace
}  // namespace heconv

using namespace heconv;

extern "C" he_status he_probe_valu(const he_ctx* ctx, uint32_t which, uint32_t iters, uint32_t blocks,
                                   uint64_t* d_work, double* ops_per_s, void* stream) {
  if (!ctx || !d_work || !ops_per_s || iters == 0 || blocks == 0) return HE_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const LimbConst* lc = ctx->d_lc;  // the first prime's constants
  const uint64_t* d_seed = d_work;
  const uint32_t* seed32 = (const uint32_t*)d_work;
  uint64_t* d_out = d_work + 64;
  double per_thread_iter = 0;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return HE_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return HE_EDEVICE;
  }
  he_status s = HE_OK;
  auto launch = [&]() -> hipError_t {
    switch (which) {
      case HE_PROBE_MAD_U64_U32:
        hipLaunchKernelGGL(probe_mad_kernel, dim3(blocks), dim3(PROBE_THREADS), 0, st, seed32, d_out, iters);
        per_thread_iter = PROBE_UNROLL * 8;
        break;
      case HE_PROBE_MUL_HI_U32:
        hipLaunchKernelGGL(probe_mulhi_kernel, dim3(blocks), dim3(PROBE_THREADS), 0, st, seed32, d_out, iters);
        per_thread_iter = PROBE_UNROLL * 8;
        break;
      case HE_PROBE_MUL_LO_U32:
        hipLaunchKernelGGL(probe_mullo_kernel, dim3(blocks), dim3(PROBE_THREADS), 0, st, seed32, d_out, iters);
        per_thread_iter = PROBE_UNROLL * 8;
        break;
      case HE_PROBE_ADD_U32:
        hipLaunchKernelGGL(probe_add_kernel, dim3(blocks), dim3(PROBE_THREADS), 0, st, seed32, d_out, iters);
        per_thread_iter = PROBE_UNROLL * 8;
        break;
      case HE_PROBE_MAC_MIX:
        if (!lc) return hipErrorInvalidValue;
        hipLaunchKernelGGL(probe_mac_kernel, dim3(blocks), dim3(PROBE_THREADS), 0, st, d_seed, d_out, iters, lc);
        per_thread_iter = 24.0 * 8;  // 6x4 products per block, 8 blocks
        break;
      case HE_PROBE_INTT_MIX:
        if (!lc) return hipErrorInvalidValue;
        hipLaunchKernelGGL(probe_bfly_kernel<true>, dim3(blocks), dim3(PROBE_THREADS), 0, st, d_seed, d_out, iters,
                           lc);
        per_thread_iter = (PROBE_UNROLL / 4) * 8;
        break;
      case HE_PROBE_NTT_MIX:
        if (!lc) return hipErrorInvalidValue;
        hipLaunchKernelGGL(probe_bfly_kernel<false>, dim3(blocks), dim3(PROBE_THREADS), 0, st, d_seed, d_out, iters,
                           lc);
        per_thread_iter = (PROBE_UNROLL / 4) * 8;
        break;
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  };
  // one untimed launch (clocks, code load), then the timed one
  hipError_t e = launch();
  if (e == hipErrorInvalidValue) s = HE_EINVAL;
  else if (e != hipSuccess) s = HE_EDEVICE;
  if (!s && hipEventRecord(e0, st) != hipSuccess) s = HE_EDEVICE;
  if (!s && launch() != hipSuccess) s = HE_EDEVICE;
  if (!s && hipEventRecord(e1, st) != hipSuccess) s = HE_EDEVICE;
  if (!s && hipEventSynchronize(e1) != hipSuccess) s = HE_EDEVICE;
  float ms = 0;
  if (!s && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) s = HE_EDEVICE;
  if (!s) *ops_per_s = per_thread_iter * iters * (double)blocks * PROBE_THREADS / (ms * 1e-3);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return s;
}
