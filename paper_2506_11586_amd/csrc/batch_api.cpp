// C ABI of the batch executor: validates jobs, builds the work lists, keeps
// the job table on the device, and launches the three batch kernels of each
// chain -- eagerly or as one captured hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <new>
#include <numeric>
#include <vector>

#include "batch.h"
#include "ctx.h"
#include "heconv.h"

using heconv::BatchChain;
using heconv::BatchItem;
using heconv::BatchJob;
using heconv::MacItem;

// Groups of jobs ("chains"): one for HE_SCHED_ONE_CHAIN, two run on two
// streams for HE_SCHED_TWO_CHAINS, up to BATCH_MAX_GROUPS run as a pipeline
// for the pipelined schedules (each group's forward NTTs and MAC tiles on the
// caller's stream, its inverse NTTs on a second stream once its MAC is done).
constexpr uint32_t BATCH_MAX_GROUPS = 8;

struct he_batch {
  const he_ctx* ctx = nullptr;
  uint32_t schedule = HE_SCHED_ONE_CHAIN;
  uint32_t n_chains = 1;  // groups of jobs
  uint32_t mac_mt = 4, mac_rt = 4;
  uint32_t mac_lds = 0;
  uint32_t mac_tiles = 1;  // streamed MAC: tiles per workgroup
  uint32_t mac_grid = 0;   // streamed MAC on a 2x2 wave grid
  uint64_t n_items = 0;
  BatchJob* d_jobs = nullptr;
  BatchItem* d_items = nullptr;
  MacItem* d_mitems = nullptr;  // streamed MAC tiles (mac_lds >= 2)
  BatchChain chains[BATCH_MAX_GROUPS] = {};
  hipStream_t side = nullptr, cap0 = nullptr, cap1 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  hipEvent_t mac_done[BATCH_MAX_GROUPS] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void free_batch(he_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (hipStream_t s : {b->side, b->cap0, b->cap1})
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t e : {b->fork, b->join})
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : b->mac_done)
    if (e) (void)hipEventDestroy(e);
  if (b->d_jobs) (void)hipFree(b->d_jobs);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_mitems) (void)hipFree(b->d_mitems);
  delete b;
}

heconv::BatchArgs args_of(const he_batch* b) {
  const he_ctx* c = b->ctx;
  return heconv::BatchArgs{b->d_jobs, c->d_fwd, c->d_inv, c->d_lc, c->L, c->N, c->logN,
                           c->tune.ntt_loge_small, c->tune.ntt_loge_large, b->mac_mt, b->mac_rt, b->mac_lds,
                           c->all_pm ? 1u : 0u, b->mac_grid};
}

bool pipelined(const he_batch* b) { return b->schedule == HE_SCHED_PIPELINED_4 || b->schedule == HE_SCHED_PIPELINED_8; }

// All chains on `main` (chain 1, if any, on `second`, forked from and
// joined back into `main` with events).  Pipelined: group g's forward NTTs
// and MAC tiles on `main`, its inverse NTTs on `second` after an event
// recorded behind its MAC, so they overlap group g+1's MAC.
hipError_t enqueue(const he_batch* b, hipStream_t main, hipStream_t second) {
  const heconv::BatchArgs a = args_of(b);
  if (pipelined(b)) {
    hipError_t e = hipEventRecord(b->fork, main);
    if (e == hipSuccess) e = hipStreamWaitEvent(second, b->fork, 0);
    for (uint32_t g = 0; g < b->n_chains && e == hipSuccess; g++) {
      e = heconv::batch_phase(b->chains[g], a, 0, main);
      if (e == hipSuccess) e = heconv::batch_phase(b->chains[g], a, 1, main);
      if (e == hipSuccess) e = hipEventRecord(b->mac_done[g], main);
      if (e == hipSuccess) e = hipStreamWaitEvent(second, b->mac_done[g], 0);
      if (e == hipSuccess) e = heconv::batch_phase(b->chains[g], a, 2, second);
    }
    if (e == hipSuccess) e = hipEventRecord(b->join, second);
    if (e == hipSuccess) e = hipStreamWaitEvent(main, b->join, 0);
    return e;
  }
  if (b->n_chains == 1) return heconv::batch_chain(b->chains[0], a, main);
  hipError_t e = hipEventRecord(b->fork, main);
  if (e == hipSuccess) e = hipStreamWaitEvent(second, b->fork, 0);
  if (e == hipSuccess) e = heconv::batch_chain(b->chains[0], a, main);
  if (e == hipSuccess) e = heconv::batch_chain(b->chains[1], a, second);
  if (e == hipSuccess) e = hipEventRecord(b->join, second);
  if (e == hipSuccess) e = hipStreamWaitEvent(main, b->join, 0);
  return e;
}

}  // namespace

extern "C" {

he_status he_batch_create(const he_ctx* c, const he_job* jobs, uint32_t n_jobs, uint32_t schedule, he_batch** out) {
  if (out) *out = nullptr;
  if (!c || !jobs || !out || n_jobs == 0 || n_jobs >= (1u << 24)) return HE_EINVAL;
  if (schedule != HE_SCHED_ONE_CHAIN && schedule != HE_SCHED_TWO_CHAINS && schedule != HE_SCHED_PIPELINED_4 &&
      schedule != HE_SCHED_PIPELINED_8)
    return HE_EINVAL;
  he_batch* b = new (std::nothrow) he_batch;
  if (!b) return HE_ENOMEM;
  b->ctx = c;
  b->schedule = schedule;
  if (schedule == HE_SCHED_TWO_CHAINS) b->n_chains = n_jobs > 1 ? 2 : 1;
  if (schedule == HE_SCHED_PIPELINED_4) b->n_chains = std::min<uint32_t>(n_jobs, 4);
  if (schedule == HE_SCHED_PIPELINED_8) b->n_chains = std::min<uint32_t>(n_jobs, 8);

  // validate, and pick the MAC tile: the context's tile when the batch
  // kernel is built for it, else (2,2) when a job has fewer than 4 output
  // channels, (4,2) when a job has fewer than 4 ciphertext rows (a job of
  // one spatial tile and one image has 2), else (6,4) for the streamed MAC
  // when every job has at least 6 output channels, else (4,4)
  std::vector<heconv::Geo> geo(n_jobs);
  bool few_rows = false, few_m = false, narrow = false;
  for (uint32_t j = 0; j < n_jobs; j++) {
    const he_job& jb = jobs[j];
    if (!heconv::geo_of(jb.desc, c->N, geo[j]) || !heconv::mac_offsets_fit(geo[j], c->L, c->N)) {
      free_batch(b);
      return HE_ESHAPE;
    }
    if (jb.B == 0 || !jb.d_in || !jb.d_wntt || !jb.d_out) {
      free_batch(b);
      return HE_EINVAL;
    }
    few_rows |= (uint64_t)jb.B * geo[j].S * 2 < 4;
    few_m |= jb.desc.M < 4;
    narrow |= jb.desc.M < 6;
  }
  // the LDS-staged MAC when the context asks for it and every job fits it
  bool dma = c->tune.mac_lds >= 2;
  for (uint32_t j = 0; j < n_jobs; j++) dma &= heconv::mac_dma_fits(geo[j].CB, c->L, c->N);
  b->mac_lds = dma ? c->tune.mac_lds : 0;
  b->mac_tiles = c->tune.mac_tiles ? c->tune.mac_tiles : 4;
  if (heconv::batch_tile_supported(c->tune.mac_mt, c->tune.mac_rt, b->mac_lds)) {
    b->mac_mt = c->tune.mac_mt, b->mac_rt = c->tune.mac_rt;
  } else if (few_m) {
    b->mac_mt = b->mac_rt = 2;
  } else if (few_rows) {
    b->mac_mt = 4, b->mac_rt = 2;
  } else {
    b->mac_mt = b->mac_lds >= 2 && !narrow ? 6 : 4, b->mac_rt = 4;
  }
  // the 2x2 wave grid when asked for and every job fills the waves' rows
  // and channels (2*mac_rt rows, 2*mac_mt channels); by default with the
  // 4x4 tile per wave (an 8x8 workgroup tile)
  auto fills = [&](uint32_t mt, uint32_t rt) {
    bool f = true;
    for (uint32_t j = 0; j < n_jobs; j++)
      f &= (uint64_t)jobs[j].B * geo[j].S * 2 >= 2 * rt && jobs[j].desc.M >= 2 * mt;
    return f;
  };
  if (b->mac_lds >= 2 && c->tune.mac_grid) {
    if (!heconv::batch_tile_supported(c->tune.mac_mt, c->tune.mac_rt, b->mac_lds) && !few_rows && !few_m && fills(4, 4))
      b->mac_mt = b->mac_rt = 4;
    b->mac_grid = b->mac_mt != 8 && b->mac_rt != 8 && fills(b->mac_mt, b->mac_rt) ? 1 : 0;
  }

  const uint64_t n_kc = (uint64_t)c->L * c->N / heconv::BATCH_MAC_THREADS;
  std::vector<BatchJob> dj(n_jobs);
  std::vector<uint64_t> n_fwd(n_jobs), n_mac(n_jobs), n_inv(n_jobs), wbytes(n_jobs);
  for (uint32_t j = 0; j < n_jobs; j++) {
    const he_job& jb = jobs[j];
    const heconv::Geo& g = geo[j];
    const uint64_t rows = (uint64_t)jb.B * g.S * 2;
    // MAC tiles: the 2x2 wave grid's cover 2*mac_mt channels x 2*mac_rt rows
    // of 64 points, the others mac_mt x mac_rt of 256
    const uint32_t gm = b->mac_grid ? 2 : 1;
    const uint64_t n_mt = (jb.desc.M + gm * b->mac_mt - 1) / (gm * b->mac_mt),
                   n_rt = (rows + gm * b->mac_rt - 1) / (gm * b->mac_rt);
    n_fwd[j] = (uint64_t)jb.B * g.CB * g.S * 2 * c->L;
    n_mac[j] = (b->mac_grid ? n_kc * 4 : n_kc) * n_mt * n_rt;
    n_inv[j] = (uint64_t)jb.B * jb.desc.M * g.S * 2 * c->L;
    wbytes[j] = (uint64_t)jb.desc.M * g.CB * c->L * c->N * 8;
    if (rows > 0xffffffffull || n_fwd[j] > 0x7fffffffull || n_mac[j] > 0x7fffffffull || n_inv[j] > 0x7fffffffull) {
      free_batch(b);
      return HE_ESHAPE;
    }
    dj[j] = BatchJob{jb.d_in, jb.d_wntt, jb.d_out, g.CB, g.S, jb.desc.M, (uint32_t)rows, (uint32_t)n_mt,
                     (uint32_t)n_rt};
  }

  std::vector<uint32_t> chain_of(n_jobs, 0);
  if (pipelined(b)) {
    // groups of consecutive jobs with about equal MAC work (weight bytes plus
    // the bytes of every image's inputs and outputs): group g ends once the
    // running total passes (g+1)/G of the whole
    std::vector<uint64_t> cost(n_jobs);
    uint64_t total = 0;
    for (uint32_t j = 0; j < n_jobs; j++) {
      cost[j] = wbytes[j] + (uint64_t)jobs[j].B * (geo[j].CB + jobs[j].desc.M) * geo[j].S * 2 * c->L * c->N * 8;
      total += cost[j];
    }
    uint64_t run = 0;
    uint32_t g = 0;
    for (uint32_t j = 0; j < n_jobs; j++) {
      chain_of[j] = g;
      run += cost[j];
      const uint32_t left = n_jobs - 1 - j, groups_left = b->n_chains - 1 - g;
      if (g + 1 < b->n_chains && (left == groups_left || (long double)run * b->n_chains >= (long double)total * (g + 1)))
        g++;
    }
    b->n_chains = g + 1;
  } else {
    // chain assignment: largest weight streams first, each to the chain with
    // fewer weight bytes so far (both chains then stream about equally)
    std::vector<uint32_t> order(n_jobs);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return wbytes[x] > wbytes[y]; });
    uint64_t load[2] = {0, 0};
    for (uint32_t j : order) {
      const uint32_t ch = (b->n_chains == 2 && load[1] < load[0]) ? 1 : 0;
      chain_of[j] = ch;
      load[ch] += wbytes[j];
    }
  }

  // work lists, chain by chain: forward NTT items, MAC tiles, inverse NTT items
  std::vector<BatchItem> items;
  std::vector<MacItem> mitems;  // streamed MAC: mac_tiles per workgroup
  uint64_t off[BATCH_MAX_GROUPS][3] = {}, cnt[BATCH_MAX_GROUPS][3] = {}, moff_of[BATCH_MAX_GROUPS] = {};
  const std::vector<uint64_t>* counts[3] = {&n_fwd, &n_mac, &n_inv};
  for (uint32_t ch = 0; ch < b->n_chains; ch++) {
    for (int ph = 0; ph < 3; ph++) {
      off[ch][ph] = items.size();
      if (ph == 1 && b->mac_lds >= 2) {
        // streamed MAC: XCD x takes the x-th eighth of every job's tiles, as
        // below.  Its list is cut into mac_tiles segments of W tiles, and its
        // workgroup i runs tile i of each segment in turn (valid ones
        // first): the workgroups advance through the segments together, so
        // the tiles running at one time stay a contiguous stretch of the
        // list and share their input and weight words in the XCD's L2 (a
        // workgroup taking consecutive tiles would reuse a weight row only
        // one tile later, after the L2 has evicted it).  The workgroups of
        // the eight lists are interleaved (workgroup 8i+x runs on XCD x).
        const uint32_t T = b->mac_tiles;
        std::vector<MacItem> per[heconv::BATCH_XCDS];
        for (uint32_t j = 0; j < n_jobs; j++) {
          if (chain_of[j] != ch) continue;
          const uint64_t n = n_mac[j];
          const uint32_t n_rt = dj[j].n_rt, per_chunk = dj[j].n_mt * dj[j].n_rt, S = dj[j].S;
          for (uint32_t x = 0; x < heconv::BATCH_XCDS; x++)
            for (uint64_t i = n * x / heconv::BATCH_XCDS; i < n * (x + 1) / heconv::BATCH_XCDS; i++) {
              const uint32_t kc = (uint32_t)(i / per_chunk), rem = (uint32_t)(i % per_chunk);
              const uint32_t mt = rem / n_rt, rt = rem % n_rt, bs0 = rt * b->mac_rt * (b->mac_grid ? 2 : 1) / 2;
              per[x].push_back(MacItem{j, kc, mt, rt, bs0 / S, bs0 % S});
            }
        }
        size_t wgs = 0;  // W: workgroups per XCD
        for (const auto& v : per) wgs = std::max(wgs, (v.size() + T - 1) / T);
        const uint64_t moff = mitems.size();
        for (size_t w = 0; w < wgs; w++)
          for (const auto& v : per)
            for (uint32_t t = 0; t < T; t++) {
              const size_t i = w + t * wgs;
              mitems.push_back(i < v.size() ? v[i] : MacItem{heconv::BATCH_NO_JOB, 0, 0, 0, 0, 0});
            }
        // the phase's workgroup count; its tiles start at mitems[moff] (kept in off/cnt below)
        moff_of[ch] = moff;
        cnt[ch][ph] = wgs * heconv::BATCH_XCDS;
        if (cnt[ch][ph] > heconv::grid_max_blocks(heconv::BATCH_MAC_THREADS)) {
          free_batch(b);
          return HE_ESHAPE;
        }
        continue;
      }
      if (ph == 1) {
        // MAC tiles: XCD x takes the x-th eighth of every job's tiles (tiles
        // are k-chunk-major, so that is a contiguous range of k-chunks); the
        // eight lists are interleaved (entry 8i+x runs on XCD x) and padded
        // to equal length
        std::vector<BatchItem> per[heconv::BATCH_XCDS];
        for (uint32_t j = 0; j < n_jobs; j++) {
          if (chain_of[j] != ch) continue;
          const uint64_t T = n_mac[j];
          for (uint32_t x = 0; x < heconv::BATCH_XCDS; x++)
            for (uint64_t i = T * x / heconv::BATCH_XCDS; i < T * (x + 1) / heconv::BATCH_XCDS; i++)
              per[x].push_back(BatchItem{j, (uint32_t)i});
        }
        size_t len = 0;
        for (const auto& v : per) len = std::max(len, v.size());
        for (size_t i = 0; i < len; i++)
          for (const auto& v : per) items.push_back(i < v.size() ? v[i] : BatchItem{heconv::BATCH_NO_JOB, 0});
      } else {
        for (uint32_t j = 0; j < n_jobs; j++) {
          if (chain_of[j] != ch) continue;
          for (uint64_t i = 0; i < (*counts[ph])[j]; i++) items.push_back(BatchItem{j, (uint32_t)i});
        }
      }
      cnt[ch][ph] = items.size() - off[ch][ph];
      // NTT grids use workgroups of up to 1024 threads, the MAC grid 256
      if (cnt[ch][ph] > heconv::grid_max_blocks(ph == 1 ? heconv::BATCH_MAC_THREADS : 1024)) {
        free_batch(b);
        return HE_ESHAPE;
      }
    }
  }
  b->n_items = items.size() + mitems.size();
  if (hipMalloc(&b->d_jobs, sizeof(BatchJob) * n_jobs) != hipSuccess ||
      hipMalloc(&b->d_items, sizeof(BatchItem) * std::max<size_t>(1, items.size())) != hipSuccess ||
      (!mitems.empty() && hipMalloc(&b->d_mitems, sizeof(MacItem) * mitems.size()) != hipSuccess)) {
    free_batch(b);
    return HE_ENOMEM;
  }
  if (hipMemcpy(b->d_jobs, dj.data(), sizeof(BatchJob) * n_jobs, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice) != hipSuccess ||
      (!mitems.empty() &&
       hipMemcpy(b->d_mitems, mitems.data(), sizeof(MacItem) * mitems.size(), hipMemcpyHostToDevice) != hipSuccess)) {
    free_batch(b);
    return HE_EDEVICE;
  }
  for (uint32_t ch = 0; ch < b->n_chains; ch++) {
    heconv::BatchPhase* ph[3] = {&b->chains[ch].fwd, &b->chains[ch].mac, &b->chains[ch].inv};
    for (int p = 0; p < 3; p++)
      *ph[p] = heconv::BatchPhase{b->d_items + off[ch][p], (uint32_t)cnt[ch][p], nullptr, 0};
    if (b->mac_lds >= 2) {
      b->chains[ch].mac.items = nullptr;
      b->chains[ch].mac.mitems = b->d_mitems ? b->d_mitems + moff_of[ch] : nullptr;
      b->chains[ch].mac.per_wg = b->mac_tiles;
    }
  }
  if ((b->n_chains == 2 || pipelined(b)) &&
      (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
       hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
       hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess)) {
    free_batch(b);
    return HE_EDEVICE;
  }
  for (uint32_t g = 0; pipelined(b) && g < b->n_chains; g++)
    if (hipEventCreateWithFlags(&b->mac_done[g], hipEventDisableTiming) != hipSuccess) {
      free_batch(b);
      return HE_EDEVICE;
    }
  *out = b;
  return HE_OK;
}

he_status he_batch_launch(he_batch* b, void* stream, int use_graph) {
  if (!b) return HE_EINVAL;
  if (!use_graph) return enqueue(b, (hipStream_t)stream, b->side) == hipSuccess ? HE_OK : HE_EDEVICE;
  if (!b->exec) {
    // capture every kernel of the batch once, on private streams; the
    // instantiated graph is then replayed on the caller's stream
    if (!b->cap0 && hipStreamCreateWithFlags(&b->cap0, hipStreamNonBlocking) != hipSuccess) return HE_EDEVICE;
    if ((b->n_chains == 2 || pipelined(b)) && !b->cap1 &&
        hipStreamCreateWithFlags(&b->cap1, hipStreamNonBlocking) != hipSuccess)
      return HE_EDEVICE;
    if (hipStreamBeginCapture(b->cap0, hipStreamCaptureModeThreadLocal) != hipSuccess) return HE_EDEVICE;
    const hipError_t le = enqueue(b, b->cap0, b->cap1);
    const hipError_t ce = hipStreamEndCapture(b->cap0, &b->graph);
    if (le != hipSuccess || ce != hipSuccess) return HE_EDEVICE;
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) return HE_EDEVICE;
  }
  return hipGraphLaunch(b->exec, (hipStream_t)stream) == hipSuccess ? HE_OK : HE_EDEVICE;
}

he_status he_batch_launch_timed(he_batch* b, void* stream, float* ms) {
  if (!b || !ms) return HE_EINVAL;
  hipStream_t main = (hipStream_t)stream;
  const heconv::BatchArgs a = args_of(b);
  if (pipelined(b)) {
    // per group: events around its forward and MAC grids on `main` and its
    // inverse grid on the side stream; the sums per stream are reported
    hipEvent_t ev[BATCH_MAX_GROUPS][5] = {};
    he_status s = HE_OK;
    for (uint32_t g = 0; g < b->n_chains && !s; g++)
      for (int k = 0; k < 5 && !s; k++)
        if (hipEventCreate(&ev[g][k]) != hipSuccess) s = HE_EDEVICE;
    if (!s && (hipEventRecord(b->fork, main) != hipSuccess || hipStreamWaitEvent(b->side, b->fork, 0) != hipSuccess))
      s = HE_EDEVICE;
    for (uint32_t g = 0; g < b->n_chains && !s; g++) {
      if (hipEventRecord(ev[g][0], main) != hipSuccess || heconv::batch_phase(b->chains[g], a, 0, main) != hipSuccess ||
          hipEventRecord(ev[g][1], main) != hipSuccess || heconv::batch_phase(b->chains[g], a, 1, main) != hipSuccess ||
          hipEventRecord(ev[g][2], main) != hipSuccess || hipStreamWaitEvent(b->side, ev[g][2], 0) != hipSuccess ||
          hipEventRecord(ev[g][3], b->side) != hipSuccess ||
          heconv::batch_phase(b->chains[g], a, 2, b->side) != hipSuccess ||
          hipEventRecord(ev[g][4], b->side) != hipSuccess)
        s = HE_EDEVICE;
    }
    if (!s && (hipEventRecord(b->join, b->side) != hipSuccess || hipStreamWaitEvent(main, b->join, 0) != hipSuccess))
      s = HE_EDEVICE;
    if (!s && hipStreamSynchronize(main) != hipSuccess) s = HE_EDEVICE;
    for (int k = 0; k < 6; k++) ms[k] = 0;
    for (uint32_t g = 0; g < b->n_chains && !s; g++) {
      float f = 0, m = 0, v = 0;
      if (hipEventElapsedTime(&f, ev[g][0], ev[g][1]) != hipSuccess ||
          hipEventElapsedTime(&m, ev[g][1], ev[g][2]) != hipSuccess ||
          hipEventElapsedTime(&v, ev[g][3], ev[g][4]) != hipSuccess)
        s = HE_EDEVICE;
      ms[0] += f, ms[1] += m, ms[5] += v;
    }
    for (auto& row : ev)
      for (hipEvent_t e : row)
        if (e) (void)hipEventDestroy(e);
    return s;
  }
  hipEvent_t ev[2][4] = {};
  he_status s = HE_OK;
  for (uint32_t c = 0; c < b->n_chains && !s; c++)
    for (int k = 0; k < 4 && !s; k++)
      if (hipEventCreate(&ev[c][k]) != hipSuccess) s = HE_EDEVICE;
  if (!s && b->n_chains == 2 &&
      (hipEventRecord(b->fork, main) != hipSuccess || hipStreamWaitEvent(b->side, b->fork, 0) != hipSuccess))
    s = HE_EDEVICE;
  for (uint32_t c = 0; c < b->n_chains && !s; c++) {
    hipStream_t st = c == 0 ? main : b->side;
    if (hipEventRecord(ev[c][0], st) != hipSuccess) s = HE_EDEVICE;
    for (int p = 0; p < 3 && !s; p++)
      if (heconv::batch_phase(b->chains[c], a, p, st) != hipSuccess || hipEventRecord(ev[c][p + 1], st) != hipSuccess)
        s = HE_EDEVICE;
  }
  if (!s && b->n_chains == 2 &&
      (hipEventRecord(b->join, b->side) != hipSuccess || hipStreamWaitEvent(main, b->join, 0) != hipSuccess))
    s = HE_EDEVICE;
  if (!s && hipStreamSynchronize(main) != hipSuccess) s = HE_EDEVICE;
  for (uint32_t c = 0; c < 2; c++)
    for (int p = 0; p < 3; p++) {
      float t = 0;
      if (!s && c < b->n_chains && hipEventElapsedTime(&t, ev[c][p], ev[c][p + 1]) != hipSuccess) s = HE_EDEVICE;
      if (c < b->n_chains) ms[3 * c + p] = t;
    }
  for (auto& row : ev)
    for (hipEvent_t e : row)
      if (e) (void)hipEventDestroy(e);
  return s;
}

he_status he_batch_status(he_batch* b, void* stream) {
  if (!b) return HE_EINVAL;
  return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? HE_OK : HE_EDEVICE;
}

he_status he_batch_info(const he_batch* b, uint64_t* n_items, uint32_t* n_chains) {
  if (!b) return HE_EINVAL;
  if (n_items) *n_items = b->n_items;
  if (n_chains) *n_chains = pipelined(b) ? 2 : b->n_chains;
  return HE_OK;
}

he_status he_batch_mac_form(const he_batch* b, uint32_t* mt, uint32_t* rt, uint32_t* lds, uint32_t* tiles,
                            uint32_t* grid) {
  if (!b) return HE_EINVAL;
  if (mt) *mt = b->mac_mt;
  if (rt) *rt = b->mac_rt;
  if (lds) *lds = b->mac_lds;
  if (tiles) *tiles = b->mac_lds >= 2 ? b->mac_tiles : 1;
  if (grid) *grid = b->mac_grid;
  return HE_OK;
}

void he_batch_destroy(he_batch* b) { free_batch(b); }

}  // extern "C"
