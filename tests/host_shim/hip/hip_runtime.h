// Host-only stand-in for <hip/hip_runtime.h>, so that the library's
// arithmetic headers compile as plain C++ for host tests: the qualifiers
// become no-ops and the device multiply-high intrinsics get exact host
// definitions.
#pragma once
#include <stdint.h>
#define __host__
#define __device__
#define __global__
#define __forceinline__ inline
static inline uint64_t __umul64hi(uint64_t a, uint64_t b) { return (uint64_t)(((unsigned __int128)a * b) >> 64); }
static inline uint32_t __umulhi(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }
