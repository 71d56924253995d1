// Internal: device-side layout of a batch (job table, work items) and the
// launcher of the persistent batch kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "modarith.h"

namespace heconv {

enum : uint32_t { ITEM_FWD = 0, ITEM_MAC = 1, ITEM_INV = 2 };

// Counters of a batch launch sit 64 words (256 bytes) apart, one per line.
constexpr uint32_t CTR_STRIDE = 64;

// MAC tile of the batch kernel: 2 output channels x 2 rows per thread keeps
// the kernel at <= 128 VGPRs, so two 512-thread workgroups fit a CU.
constexpr int BATCH_MT = 2, BATCH_RT = 2;

struct BatchJob {
  uint64_t* in;        // [B][CB][S][2][L][N]
  const uint64_t* w;   // [M][CB][L][N]
  uint64_t* out;       // [B][M][S][2][L][N]
  uint32_t CB, S, M, rows;  // rows = B*S*2
  uint32_t n_mt, n_rt;      // MAC tiles over output channels and rows
  uint32_t n_fwd, n_mac, n_inv;
};

struct BatchItem {
  uint32_t jt;   // job << 2 | item type
  uint32_t idx;  // limb polynomial (FWD/INV) or MAC tile index
};

struct BatchLaunch {
  const BatchItem* items;
  uint32_t n_items;
  const BatchJob* jobs;
  uint32_t* ctr;    // (2 + 2 * n_jobs) * CTR_STRIDE words
  uint32_t n_ctr;
  const Tw* twf;
  const Tw* twi;
  const LimbConst* lcs;
  uint32_t L;
  uint32_t spin_limit;
  uint32_t grid;
};

hipError_t batch_occupancy(uint32_t logN, int* blocks_per_cu);
// A counter-reset kernel, then the persistent kernel, on stream st.
hipError_t batch_launch(uint32_t logN, const BatchLaunch& a, hipStream_t st);

}  // namespace heconv
