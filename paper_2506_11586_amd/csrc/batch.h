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

// One MAC tile of a batch job for the streamed MAC, decoded on the host so
// that the kernel divides nothing: k-chunk kc (256 NTT points of limb
// kc >> (logN - 8)), output channels mt*MT.., rows rt*RT.., and the image b0
// and spatial tile s0 of its first row pair (row pair rt*RT/2 = b0*S + s0).
// (With the 2x2 wave grid, kc is a chunk of 64 points, limb kc >> (logN - 6),
// and the tile covers channels mt*2MT.. and rows rt*2RT.., first row pair
// rt*RT = b0*S + s0.)
struct MacItem {
  uint32_t job;  // BATCH_NO_JOB: padding (only after a workgroup's last tile)
  uint32_t kc, mt, rt, b0, s0;
};

struct BatchPhase {
  const BatchItem* items;  // device
  uint32_t n;              // items; for the streamed MAC, workgroups
  const MacItem* mitems;   // streamed MAC: per_wg consecutive tiles per workgroup
  uint32_t per_wg;
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
  uint32_t mac_lds;                 // 0, or LDS stages of the streamed MAC (mac_stream)
  uint32_t all_pm;                  // every q_l = 2^60 - delta, delta < 2^20 (the MAC's short fold)
  uint32_t mac_grid;                // streamed MAC on a 2x2 wave grid (mac_grid): tiles of 2*mac_mt x 2*mac_rt
};

// Register tiles the batch MAC is built for: with register loads (lds 0)
// (4,4), (4,2), (2,4), (2,2); streamed (lds 2-4) also (6,4), (8,4) and (4,8).
bool batch_tile_supported(uint32_t mt, uint32_t rt, uint32_t lds);

// Forward-NTT grid, MAC grid, inverse-NTT grid of one chain, on stream st.
hipError_t batch_chain(const BatchChain& ch, const BatchArgs& a, hipStream_t st);

// One of the three grids of a chain (0 forward NTT, 1 MAC, 2 inverse NTT).
hipError_t batch_phase(const BatchChain& ch, const BatchArgs& a, int phase, hipStream_t st);

}  // namespace heconv
