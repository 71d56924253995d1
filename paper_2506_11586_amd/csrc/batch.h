// Internal: device-side layout of a batch (job table, work lists) and the
// launcher of one chain of batch kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "modarith.h"

namespace heconv {

constexpr uint32_t BATCH_MAC_THREADS = 256;
constexpr uint32_t BATCH_XCDS = 8;              // workgroup b of a grid runs on XCD b mod 8
constexpr uint32_t BATCH_NO_JOB = 0xffffffffu;  // padding entry of a MAC work list

struct BatchJob {
  uint64_t* in;             // [B][CB][S][2][L][N]
  const uint64_t* w;        // [M][CB][L][N]
  uint64_t* out;            // [B][M][S][2][L][N]
  uint32_t CB, S, M, rows;  // rows = B*S*2
  uint32_t n_mt, n_rt;      // MAC tiles over output channels and rows
};

struct BatchItem {
  uint32_t job;
  uint32_t idx;  // limb polynomial (NTT phases) or MAC tile index
};

struct BatchPhase {
  const BatchItem* items;  // device
  uint32_t n;
};

// The three phases of one chain of jobs.
struct BatchChain {
  BatchPhase fwd, mac, inv;
};

struct BatchArgs {
  const BatchJob* jobs;
  const Tw* twf;
  const Tw* twi;
  const LimbConst* lcs;
  uint32_t L, N, logN;
  uint32_t loge_small, loge_large;  // NTT words per thread below / from 512 limb polys
  uint32_t mac_mt, mac_rt;          // MAC register tile, see batch_tile_supported
  uint32_t mac_lds;                 // 0, or LDS stages of the staged MAC (mac_tile_dma)
};

// Register tiles the batch MAC is built for: (4,4), (4,2), (2,4), (2,2).
bool batch_tile_supported(uint32_t mt, uint32_t rt);

// Forward-NTT grid, MAC grid, inverse-NTT grid of one chain, on stream st.
hipError_t batch_chain(const BatchChain& ch, const BatchArgs& a, hipStream_t st);

// One of the three grids of a chain (0 forward NTT, 1 MAC, 2 inverse NTT).
hipError_t batch_phase(const BatchChain& ch, const BatchArgs& a, int phase, hipStream_t st);

}  // namespace heconv
