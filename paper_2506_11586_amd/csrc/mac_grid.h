// Streamed MAC with the workgroup's four waves as a 2 x 2 grid over one
// slice of 64 NTT points (device part, batch executor).
//
// mac_stream gives each wave its own 64 points, so the four waves of a
// workgroup load disjoint rows: per channel block a wave loads MT + RT rows
// for MT*RT products.  Here the four waves cover the same 64 points: wave w
// computes output channels (w & 1)*MT .. and rows (w >> 1)*RT .. of a
// (2MT) x (2RT) workgroup tile, reading the RT input rows it shares with the
// wave beside it and the MT weight rows it shares with the wave below from
// one LDS ring that the four waves fill together.  A block then moves
// 2(MT + RT) rows for 4*MT*RT products, half of what four separate waves
// load, which matters because the vector-memory data path, not the HBM, is
// what the batch MAC saturates.
//
// Same sums, accumulators, carries and folds as mac_stream (three
// accumulators, a carry every MAC3_CHUNK blocks kept whole in a00, the
// canonical fold at the tile's end).  The loads are direct buffer-to-LDS
// loads, P - 1 blocks ahead across tile boundaries; the 2(MT + RT)/2 row
// pairs of a block are spread over the waves (pair j by wave j mod 4).  One
// workgroup barrier per block: a wave waits for its own loads of block g,
// and after the barrier every wave's loads of block g are in LDS and every
// wave has finished reading block g - 1, whose stage the loads of block
// g + P - 1 then overwrite.  Every wave runs the same tiles and blocks, so
// every wave reaches every barrier.
#pragma once
#include "mac_stream.h"

namespace heconv {

template <int MT, int RT>
struct MacGridShape {
  static constexpr int PIN = RT, PW = MT, PAIRS = PIN + PW;  // row pairs of the workgroup tile
  static constexpr int ROWS = 2 * PAIRS;                     // rows of one LDS stage
  static constexpr int NW = (PAIRS + 3) / 4;                 // pairs loaded by one wave, at most
};

template <int MT, int RT>
struct MacGridLoad {
  __amdgpu_buffer_rsrc_t r[MacGridShape<MT, RT>::NW];
  uint32_t lane_off[MacGridShape<MT, RT>::NW];  // the lane's byte offset (second row for lanes 32-63)
  uint32_t step[MacGridShape<MT, RT>::NW];      // bytes from one channel block to the next
  uint32_t CB;
};

template <int MT, int RT>
struct MacGridStore {
  uint64_t obase[RT / 2];  // word offset of component a of each of the wave's row pairs, channel of its first column
  uint64_t mstride;
  uint32_t CB, l;
  uint32_t rvalid, mvalid;  // the wave's rows / channels inside the job
};

// Image and spatial tile of row pair `idx` of a tile whose first pair is (b0, s0).
__device__ __forceinline__ void mac_grid_pair(uint32_t b0, uint32_t s0, uint32_t S, uint32_t idx, uint32_t& b,
                                              uint32_t& s) {
  b = b0, s = s0 + idx;
  while (s >= S) s -= S, b++;
}

// Decode tile `it` (kc: a chunk of 64 NTT points, limb kc >> (logN - 6);
// mt, rt: tiles of 2*MT channels and 2*RT rows) for wave `wave` (0-3).
template <int MT, int RT>
__device__ __forceinline__ void mac_grid_decode(const MacItem& it, const BatchJob& jd, uint32_t L, uint32_t logN,
                                                uint32_t wave, uint32_t half, uint32_t lo16,
                                                MacGridLoad<MT, RT>* ld, MacGridStore<MT, RT>* sd) {
  using Sh = MacGridShape<MT, RT>;
  const uint32_t N = 1u << logN;
  const uint32_t l = it.kc >> (logN - 6);
  const uint64_t kofs = (uint64_t)l * N + ((uint64_t)(it.kc & ((N >> 6) - 1)) << 6);
  const uint64_t LN = (uint64_t)L << logN;
  const uint64_t in_cb = (uint64_t)jd.S * 2 * LN, mstride = in_cb;
  const uint32_t r0 = it.rt * 2 * RT, m0 = it.mt * 2 * MT;
  if (ld) {
#pragma unroll
    for (int k = 0; k < Sh::NW; k++) {
      const uint32_t j = wave + 4 * k;  // the workgroup pair this wave loads (j >= PAIRS: none)
      const uint32_t jj = j < Sh::PAIRS ? j : 0;
      if (jj < Sh::PIN) {
        uint32_t b, s;
        mac_grid_pair(it.b0, it.s0, jd.S, jj, b, s);
        const bool ok = r0 + 2 * jj < jd.rows;
        const uint64_t base = (((uint64_t)(ok ? b : 0) * jd.CB * jd.S + (ok ? s : 0)) * 2) * LN + kofs;
        ld->r[k] = mac_rsrc((const uint64_t*)jd.in + base, (uint64_t)jd.CB * in_cb * 8);
        ld->lane_off[k] = lo16 + half * (uint32_t)(LN * 8);
        ld->step[k] = (uint32_t)(in_cb * 8);
      } else {
        const uint32_t m = m0 + 2 * (jj - Sh::PIN);
        ld->r[k] = mac_rsrc(jd.w + ((uint64_t)(m < jd.M ? m : 0) * jd.CB) * LN + kofs, (uint64_t)2 * jd.CB * LN * 8);
        ld->lane_off[k] = lo16 + half * (m + 1 < jd.M ? (uint32_t)(jd.CB * LN * 8) : 0u);
        ld->step[k] = (uint32_t)(LN * 8);
      }
    }
    ld->CB = jd.CB;
  }
  if (sd) {
    const uint32_t wi = wave & 1, wj = wave >> 1;
#pragma unroll
    for (int p = 0; p < RT / 2; p++) {
      uint32_t b, s;
      const uint32_t idx = wj * (RT / 2) + p;
      mac_grid_pair(it.b0, it.s0, jd.S, idx, b, s);
      const bool ok = r0 + 2 * idx < jd.rows;
      sd->obase[p] = (((uint64_t)(ok ? b : 0) * jd.M * jd.S + (ok ? s : 0)) * 2) * LN + kofs +
                     (uint64_t)(m0 + wi * MT) * mstride;
    }
    sd->mstride = mstride;
    sd->CB = jd.CB;
    sd->l = l;
    const uint32_t rw = r0 + wj * RT, mw = m0 + wi * MT;
    sd->rvalid = rw >= jd.rows ? 0u : (jd.rows - rw >= (uint32_t)RT ? (1u << RT) - 1 : (1u << (jd.rows - rw)) - 1);
    sd->mvalid = mw >= jd.M ? 0u : (jd.M - mw >= (uint32_t)MT ? (1u << MT) - 1 : (1u << (jd.M - mw)) - 1);
  }
}

template <int MT, int RT, int THREADS, int P, bool PM, class Src>
__device__ __forceinline__ void mac_grid(const Src& src, const LimbConst* __restrict__ lcs, uint32_t L, uint32_t logN,
                                         uint64_t* lds, int tid) {
  static_assert(THREADS == 256 && MT % 2 == 0 && RT % 2 == 0 && P >= 2 && P <= 4, "four waves, rows in pairs");
  using Sh = MacGridShape<MT, RT>;
  constexpr int ROWS = Sh::ROWS;
  // loads per block of the wave with the fewest (every wave loads PAIRS / 4
  // or PAIRS / 4 + 1 row pairs)
  constexpr int MINE = Sh::PAIRS / 4;
  static_assert(MINE >= 1 && (P - 2) * MINE <= 63, "wait counts");
  // (tid < 256: the mask only tells the compiler that wave <= 3, so that the
  // per-wave load tests of tiles whose pairs divide by four fold away)
  const uint32_t wave = __builtin_amdgcn_readfirstlane((uint32_t)tid >> 6) & 3u, lane = (uint32_t)tid & 63;
  const uint32_t half = lane >> 5, lo16 = (lane & 31) * 16;
  const uint32_t wi = wave & 1, wj = wave >> 1;
  const uint32_t LN8 = (L << logN) * 8;

  const uint32_t nv = src.count();
  if (nv == 0) return;

  // load cursor: tile li, its block lcb, the stage it fills; it stays on the
  // stream's last block once that is issued (li = nv), so that every block
  // issues the same loads and the wait count is a constant (the P - 1
  // re-loads at the end fill stages that no block reads)
  uint32_t li = 0, lcb = 0, lst = 0;
  MacGridLoad<MT, RT> ld;
  auto load_tile = [&](uint32_t i) {
    MacItem it;
    BatchJob jd;
    src.get(i, it, jd);
    mac_grid_decode<MT, RT>(it, jd, L, logN, wave, half, lo16, &ld, (MacGridStore<MT, RT>*)nullptr);
  };
  auto issue_next = [&]() {
    uint64_t* st = lds + lst * ROWS * 64;
#pragma unroll
    for (int k = 0; k < Sh::NW; k++)
      if (wave + 4 * k < (uint32_t)Sh::PAIRS)
        mac_dma_load(ld.r[k], st + (wave + 4 * k) * 2 * 64, ld.lane_off[k], lcb * ld.step[k]);
    lst = lst + 1 == (uint32_t)P ? 0 : lst + 1;
    if (li < nv && ++lcb == ld.CB) {
      if (li + 1 < nv) {
        lcb = 0;
        load_tile(++li);
      } else {
        lcb = ld.CB - 1, li = nv;
      }
    }
  };

  uint32_t ci = 0;
  MacGridStore<MT, RT> sd;
  MacItem it0;
  BatchJob jd0;
  src.get(0, it0, jd0);
  gword* out = as_global(jd0.out);
  mac_grid_decode<MT, RT>(it0, jd0, L, logN, wave, half, lo16, (MacGridLoad<MT, RT>*)nullptr, &sd);
  LimbConst c = lcs[sd.l];

  load_tile(0);
#pragma unroll
  for (int s0 = 0; s0 < P - 1; s0++) issue_next();
  uint32_t gst = 0;  // the stage of the block being consumed
  for (;;) {         // tiles
    uint64_t a00[MT][RT], am[MT][RT], a11[MT][RT];
#pragma unroll
    for (int j = 0; j < MT; j++)
#pragma unroll
      for (int i = 0; i < RT; i++) a00[j][i] = am[j][i] = a11[j][i] = 0;
    for (uint32_t ccb = 0;;) {  // chunks of MAC3_CHUNK blocks
      const uint32_t nb = sd.CB - ccb < MAC3_CHUNK ? sd.CB - ccb : MAC3_CHUNK;
      for (uint32_t k = 0; k < nb; k++) {
        // own loads of block g (P - 2 blocks were issued after it; a wave with
        // more than MINE loads a block waits for a few more than it needs),
        // then every wave's, and every wave is past block g - 1
        wait_vmcnt<(P - 2) * MINE>();
        __builtin_amdgcn_s_barrier();
        __asm__ volatile("" ::: "memory");
        issue_next();  // block g + P - 1, into the stage block g - 1 used
        __builtin_amdgcn_sched_barrier(0);
        const uint64_t* st = lds + gst * ROWS * 64 + lane;
        gst = gst + 1 == (uint32_t)P ? 0 : gst + 1;
        Half30 xs[RT];
#pragma unroll
        for (int i = 0; i < RT; i++) xs[i] = split30(st[(wj * RT + i) * 64]);
#pragma unroll
        for (int j = 0; j < MT; j++) {
          const Half30 ws = split30(st[(2 * RT + wi * MT + j) * 64]);
#pragma unroll
          for (int i = 0; i < RT; i++) {
            a00[j][i] += (uint64_t)xs[i].lo * ws.lo;
            am[j][i] += (uint64_t)xs[i].lo * ws.hi;
            am[j][i] += (uint64_t)xs[i].hi * ws.lo;
            a11[j][i] += (uint64_t)xs[i].hi * ws.hi;
          }
        }
        __asm__ volatile("" ::: "memory");
      }
      ccb += nb;
      if (ccb == sd.CB) break;
#pragma unroll
      for (int j = 0; j < MT; j++)
#pragma unroll
        for (int i = 0; i < RT; i++) {
          const uint64_t x = PM ? fold3_pm<false>(a00[j][i], am[j][i], a11[j][i], (uint32_t)c.pmd, (uint32_t)c.c30)
                                : fold30(a00[j][i], am[j][i], 0, a11[j][i], c);
          a00[j][i] = x, am[j][i] = 0, a11[j][i] = 0;
        }
    }
#pragma unroll
    for (int j = 0; j < MT; j++)
#pragma unroll
      for (int i = 0; i < RT; i++) {
        const uint64_t r = PM ? fold3_pm<true>(a00[j][i], am[j][i], a11[j][i], (uint32_t)c.pmd, (uint32_t)c.c30)
                              : fold30(a00[j][i], am[j][i], 0, a11[j][i], c);
        if (((sd.rvalid >> i) & (sd.mvalid >> j) & 1u) != 0) {
          gword* o = out + uniform64(sd.obase[i / 2] + (uint64_t)(i & 1) * (LN8 / 8) + (uint64_t)j * sd.mstride);
          __builtin_nontemporal_store(r, &o[lane]);
        }
      }
    if (++ci == nv) break;
    MacItem it;
    BatchJob jd;
    src.get(ci, it, jd);
    out = as_global(jd.out);
    mac_grid_decode<MT, RT>(it, jd, L, logN, wave, half, lo16, (MacGridLoad<MT, RT>*)nullptr, &sd);
    c = lcs[sd.l];
  }
  wait_vmcnt<0>();
}

}  // namespace heconv
