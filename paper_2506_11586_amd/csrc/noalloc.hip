// Rotation without a caller-provided work buffer and without any device
// allocation: the key-switching scratch lives in a fixed device array of
// this library (one copy per GPU, held until the process ends).
#include <hip/hip_runtime.h>

#include <mutex>

#include "ctx.h"
#include "heconv.h"

namespace {

// 64 MiB of uint64 words: n * (L+2) * (L+1) * N words for n ciphertexts,
// e.g. 51 ciphertexts at N = 8192 with 3 ciphertext primes.
constexpr uint64_t SCRATCH_WORDS = HE_ROTATE_NOALLOC_MAX_WORDS;
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) uint64_t scratch[SCRATCH_WORDS];

std::mutex g_mu;
uint64_t* g_ptr[MAX_DEVICES] = {};

// The device address of `scratch` on `dev` (the host-side name is not a
// device address), looked up once per device with that device current.
he_status scratch_ptr(int dev, uint64_t** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return HE_EDEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return HE_EDEVICE;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return HE_EDEVICE;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) return HE_EDEVICE;
    g_ptr[dev] = static_cast<uint64_t*>(p);
  }
  *out = g_ptr[dev];
  return HE_OK;
}

}  // namespace

extern "C" he_status he_rotate_noalloc(const he_ctx* ext, uint64_t g, uint64_t n, const uint64_t* d_ct,
                                       const uint64_t* d_ksk_ntt, uint64_t* d_out, void* stream) {
  if (!ext) return HE_EINVAL;
  uint64_t words = 0;
  if (he_status s = he_keyswitch_work_words(ext, n, &words)) return s;
  if (n == 0) return HE_OK;
  if (words > SCRATCH_WORDS) return HE_ESHAPE;
  uint64_t* work = nullptr;
  if (he_status s = scratch_ptr(ext->device, &work)) return s;
  return he_rotate(ext, g, n, d_ct, d_ksk_ntt, d_out, work, stream);
}
