// Streamed channel-block MAC (device part), for the batch executor and the
// per-layer MAC.
//
// A batch workgroup runs a short list of MAC tiles (consecutive tiles of one
// XCD's share, decoded on the host into MacItems; the per-layer kernel runs
// one tile decoded from its block index) as one continuous stream
// of channel blocks per wave: the direct buffer-to-LDS loads run P - 1
// blocks ahead of the products across tile boundaries, so the next tile's
// first blocks are in flight while the current tile's sums are folded and
// stored, and a tile costs no start-up latency and no integer division.
//
// Same sums as mac_tile (Out[(b,s,c), m] = sum_cb
// In[(b,s,c), cb] * W[cb, m] mod q at every NTT point, Sec. 6.2), with three
// accumulators per output instead of four: a00 += lo*lo, am += lo*hi +
// hi*lo, a11 += hi*hi over the operands' 30-bit halves.  The two cross
// products share am, so a fold comes every MAC3_CHUNK = 8 blocks (am then
// holds sixteen products below 2^60 plus the carry), and a tile of
// MT x RT outputs holds 6*MT*RT accumulator registers: 8 x 4 and 4 x 8 tiles
// fit, which load up to a quarter fewer operand rows per product than 4 x 4.
// The carried value between chunks is the unreduced fold X (below
// 2^60 + 2^45), kept whole in a00 (am and a11 restart at zero, so only a00
// is carried from chunk to chunk in registers).
//
// Wave layout (see mac_impl.h): each wave streams its own 64 NTT points
// of the tile through a private LDS ring of P stages of MT + RT rows (512
// bytes a row), one load instruction filling two rows (lanes 0-31 the first
// row's 512 bytes, lanes 32-63 the second's).  No workgroup barrier: a
// wave's loads into LDS count in its own vmcnt, and loads return in order,
// so block g is in LDS once at most (blocks issued after g) * PAIRS vector
// memory operations are outstanding.  The stores of a finished tile also
// count in vmcnt; the wait may then also wait for some of them (never too
// little).
#pragma once
#include "batch.h"
#include "mac_impl.h"

namespace heconv {

constexpr uint32_t MAC3_CHUNK = 8;

// The load side of one tile: buffer resources of its input and weight row
// pairs (a pair past the end reads pair 0: valid memory, never stored).
template <int MT, int RT>
struct MacLoad {
  __amdgpu_buffer_rsrc_t ib[RT / 2], wb[MT / 2];
  uint32_t w2[MT / 2];       // byte offset of a weight pair's second channel (0 past the end)
  uint32_t CB, in_step;      // blocks; bytes from one input block to the next
};

// The fold-and-store side of one tile.
template <int MT, int RT>
struct MacStore {
  uint64_t obase[RT / 2];    // word offset (from the job's out) of component a of each row pair, channel mt*MT
  uint64_t mstride;          // words from one output channel to the next
  uint32_t CB, l;
  uint32_t rvalid, mvalid;   // rows / output channels of the tile inside the job
};

// Decode tile `it` of job `jd` for the calling wave (all values uniform).
template <int MT, int RT>
__device__ __forceinline__ void mac_stream_decode(const MacItem& it, const BatchJob& jd, uint32_t L, uint32_t logN,
                                                  uint32_t wave, MacLoad<MT, RT>* ld, MacStore<MT, RT>* sd) {
  constexpr int PIN = RT / 2, PW = MT / 2;
  const uint32_t N = 1u << logN;
  const uint32_t l = it.kc >> (logN - 8);
  const uint64_t kofs = (uint64_t)l * N + ((uint64_t)(it.kc & ((N >> 8) - 1)) << 8) + wave * 64;
  const uint64_t LN = (uint64_t)L << logN;
  const uint64_t in_cb = (uint64_t)jd.S * 2 * LN;  // words from one input block to the next
  const uint64_t mstride = in_cb;                  // words from one output channel to the next
  uint32_t b = it.b0, s = it.s0;
#pragma unroll
  for (int p = 0; p < PIN; p++) {
    const bool ok = it.rt * RT + 2 * p < jd.rows;
    const uint64_t bp = ok ? b : 0, sp = ok ? s : 0;
    if (ld)
      ld->ib[p] = mac_rsrc((const uint64_t*)jd.in + ((bp * jd.CB * jd.S + sp) * 2) * LN + kofs,
                           (uint64_t)jd.CB * in_cb * 8);
    if (sd) sd->obase[p] = ((bp * jd.M * jd.S + sp) * 2) * LN + kofs + (uint64_t)it.mt * MT * mstride;
    if (++s == jd.S) s = 0, b++;
  }
  if (ld) {
#pragma unroll
    for (int p = 0; p < PW; p++) {
      const uint32_t m = it.mt * MT + 2 * p;
      ld->wb[p] = mac_rsrc(jd.w + ((uint64_t)(m < jd.M ? m : 0) * jd.CB) * LN + kofs, (uint64_t)2 * jd.CB * LN * 8);
      ld->w2[p] = m + 1 < jd.M ? (uint32_t)(jd.CB * LN * 8) : 0u;
    }
    ld->CB = jd.CB;
    ld->in_step = (uint32_t)(in_cb * 8);
  }
  if (sd) {
    sd->mstride = mstride;
    sd->CB = jd.CB;
    sd->l = l;
    const uint32_t r0 = it.rt * RT, m0 = it.mt * MT;
    sd->rvalid = r0 >= jd.rows ? 0u : (jd.rows - r0 >= (uint32_t)RT ? (1u << RT) - 1 : (1u << (jd.rows - r0)) - 1);
    sd->mvalid = m0 >= jd.M ? 0u : (jd.M - m0 >= (uint32_t)MT ? (1u << MT) - 1 : (1u << (jd.M - m0)) - 1);
  }
}

// Tile sources: count() tiles, get(i) the tile and its job.
// A batch workgroup's list: items[0 .. n), valid ones first.
struct MacListSrc {
  const MacItem* __restrict__ items;
  uint32_t n;
  const BatchJob* __restrict__ jobs;
  __device__ __forceinline__ uint32_t count() const {
    uint32_t nv = 0;
    while (nv < n && items[nv].job != BATCH_NO_JOB) nv++;
    return nv;
  }
  __device__ __forceinline__ void get(uint32_t i, MacItem& it, BatchJob& jd) const {
    it = items[i];
    jd = jobs[it.job];
  }
};

// One tile of one layer, decoded by the caller.
struct MacOneSrc {
  MacItem it;
  BatchJob jd;
  __device__ __forceinline__ uint32_t count() const { return 1; }
  __device__ __forceinline__ void get(uint32_t, MacItem& i, BatchJob& j) const { i = it, j = jd; }
};

// The source's tiles, for the calling wave's 64 points of each.  PM: every
// limb's prime is 2^60 - delta (fold3_pm), else the Shoup fold of any prime
// (fold30); a compile-time choice, so that the fold code has one path and
// the accumulators stay in their registers across it.
template <int MT, int RT, int THREADS, int P, bool PM, class Src>
__device__ __forceinline__ void mac_stream(const Src& src, const LimbConst* __restrict__ lcs, uint32_t L,
                                           uint32_t logN, uint64_t* lds, int tid) {
  static_assert(MT % 2 == 0 && RT % 2 == 0 && P >= 2 && P <= 4, "rows are loaded in pairs");
  constexpr int PIN = RT / 2, PW = MT / 2, PAIRS = PIN + PW, ROWS = MT + RT;
  const uint32_t wave = __builtin_amdgcn_readfirstlane((uint32_t)tid >> 6), lane = (uint32_t)tid & 63;
  const uint32_t half = lane >> 5, lo16 = (lane & 31) * 16;
  const uint32_t LN8 = (L << logN) * 8;
  const uint32_t in_lane = lo16 + half * LN8;
  uint64_t* ring = lds + (uint64_t)wave * P * ROWS * 64;

  const uint32_t nv = src.count();
  if (nv == 0) return;

  // load cursor: tile li, its block lcb, the stage it fills.  Once the
  // stream's last block is issued the cursor stays on it (li = nv): every
  // block issues the same PAIRS loads, so block g is in LDS once at most
  // (P - 1) * PAIRS are outstanding, a constant; the P - 1 re-loads at the end
  // fill stages that no block reads.
  uint32_t li = 0, lcb = 0, lst = 0;
  MacLoad<MT, RT> ld;
  uint32_t w_lane[PW];
  auto load_tile = [&](uint32_t i) {
    MacItem it;
    BatchJob jd;
    src.get(i, it, jd);
    mac_stream_decode<MT, RT>(it, jd, L, logN, wave, &ld, (MacStore<MT, RT>*)nullptr);
#pragma unroll
    for (int p = 0; p < PW; p++) w_lane[p] = lo16 + half * ld.w2[p];
  };
  auto issue_next = [&]() {
    uint64_t* st = ring + lst * ROWS * 64;
#pragma unroll
    for (int p = 0; p < PIN; p++) mac_dma_load(ld.ib[p], st + (2 * p) * 64, in_lane, lcb * ld.in_step);
#pragma unroll
    for (int p = 0; p < PW; p++) mac_dma_load(ld.wb[p], st + (RT + 2 * p) * 64, w_lane[p], lcb * LN8);
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

  // compute cursor: tile ci
  uint32_t ci = 0;
  MacStore<MT, RT> sd;
  MacItem it0;
  BatchJob jd0;
  src.get(0, it0, jd0);
  gword* out = as_global(jd0.out);
  mac_stream_decode<MT, RT>(it0, jd0, L, logN, wave, (MacLoad<MT, RT>*)nullptr, &sd);
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
        issue_next();
        wait_vmcnt<(P - 1) * PAIRS>();  // P - 1 blocks were issued after this one
        __asm__ volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        const uint64_t* st = ring + gst * ROWS * 64 + lane;
        gst = gst + 1 == (uint32_t)P ? 0 : gst + 1;
        Half30 xs[RT];
#pragma unroll
        for (int i = 0; i < RT; i++) xs[i] = split30(st[i * 64]);
#pragma unroll
        for (int j = 0; j < MT; j++) {
          const Half30 ws = split30(st[(RT + j) * 64]);
#pragma unroll
          for (int i = 0; i < RT; i++) {
            a00[j][i] += (uint64_t)xs[i].lo * ws.lo;
            am[j][i] += (uint64_t)xs[i].lo * ws.hi;
            am[j][i] += (uint64_t)xs[i].hi * ws.lo;
            a11[j][i] += (uint64_t)xs[i].hi * ws.hi;
          }
        }
        // the next load into this stage must not pass the reads above
        __asm__ volatile("" ::: "memory");
      }
      ccb += nb;
      if (ccb == sd.CB) break;
      // carry the chunk's sum into the next chunk's accumulators
#pragma unroll
      for (int j = 0; j < MT; j++)
#pragma unroll
        for (int i = 0; i < RT; i++) {
          const uint64_t x = PM ? fold3_pm<false>(a00[j][i], am[j][i], a11[j][i], (uint32_t)c.pmd, (uint32_t)c.c30)
                                : fold30(a00[j][i], am[j][i], 0, a11[j][i], c);
          a00[j][i] = x, am[j][i] = 0, a11[j][i] = 0;
        }
    }
    // the tile's sums, reduced and stored (non-temporal: streamed past the
    // caches, which keep the weights)
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
    mac_stream_decode<MT, RT>(it, jd, L, logN, wave, (MacLoad<MT, RT>*)nullptr, &sd);
    c = lcs[sd.l];
  }
  wait_vmcnt<0>();  // no load into LDS outlives the wave
}

}  // namespace heconv
