// C ABI of the batch executor: validates jobs, builds the work list, keeps
// the job table on the device, and launches (optionally as a captured
// hipGraph) the persistent batch kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <new>
#include <vector>

#include "batch.h"
#include "ctx.h"
#include "heconv.h"

using heconv::BatchItem;
using heconv::BatchJob;

struct he_batch {
  const he_ctx* ctx = nullptr;
  std::vector<BatchJob> jobs;
  BatchJob* d_jobs = nullptr;
  BatchItem* d_items = nullptr;
  uint32_t* d_ctr = nullptr;
  uint32_t n_items = 0, n_ctr = 0, grid = 0, spin_limit = 1u << 20;
  uint32_t n_jobs = 0;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void free_batch(he_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->d_jobs) (void)hipFree(b->d_jobs);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_ctr) (void)hipFree(b->d_ctr);
  delete b;
}

void emit(std::vector<BatchItem>& v, uint32_t j, uint32_t type, uint32_t count) {
  for (uint32_t i = 0; i < count; i++) v.push_back(BatchItem{(j << 2) | type, i});
}

heconv::BatchLaunch launch_args(const he_batch* b) {
  const he_ctx* c = b->ctx;
  return heconv::BatchLaunch{b->d_items, b->n_items, b->d_jobs, b->d_ctr, b->n_ctr, c->d_fwd,
                             c->d_inv,   c->d_lc,    c->L,      b->spin_limit, b->grid};
}

}  // namespace

extern "C" {

he_status he_batch_create(const he_ctx* c, const he_job* jobs, uint32_t n_jobs, uint32_t schedule, he_batch** out) {
  // The persistent executor is switched off: its kernel hung on the GPU
  // (see the notes on the batch executor in the design document).
  if (out) *out = nullptr;
  return HE_EINVAL;
  if (!c || !jobs || !out || n_jobs == 0 || n_jobs >= (1u << 20)) return HE_EINVAL;
  if (schedule != HE_SCHED_PIPELINED && schedule != HE_SCHED_PHASED) return HE_EINVAL;
  *out = nullptr;
  const uint64_t T = c->N / 16, n_kc = (uint64_t)c->L * c->N / T;
  he_batch* b = new (std::nothrow) he_batch;
  if (!b) return HE_ENOMEM;
  b->ctx = c;
  uint64_t total = 0;
  for (uint32_t j = 0; j < n_jobs; j++) {
    const he_job& jb = jobs[j];
    heconv::Geo g;
    if (!heconv::geo_of(jb.desc, c->N, g)) {
      free_batch(b);
      return HE_ESHAPE;
    }
    if (jb.B == 0 || !jb.d_in || !jb.d_wntt || !jb.d_out) {
      free_batch(b);
      return HE_EINVAL;
    }
    BatchJob d{};
    d.in = jb.d_in, d.w = jb.d_wntt, d.out = jb.d_out;
    const uint64_t rows = (uint64_t)jb.B * g.S * 2;
    const uint64_t n_mt = (jb.desc.M + heconv::BATCH_MT - 1) / heconv::BATCH_MT;
    const uint64_t n_rt = (rows + heconv::BATCH_RT - 1) / heconv::BATCH_RT;
    const uint64_t n_fwd = (uint64_t)jb.B * g.CB * g.S * 2 * c->L;
    const uint64_t n_mac = n_kc * n_mt * n_rt;
    const uint64_t n_inv = (uint64_t)jb.B * jb.desc.M * g.S * 2 * c->L;
    if (rows > 0xffffffffull || n_fwd > 0xffffffffull || n_mac > 0xffffffffull || n_inv > 0xffffffffull) {
      free_batch(b);
      return HE_ESHAPE;
    }
    d.CB = g.CB, d.S = g.S, d.M = jb.desc.M, d.rows = (uint32_t)rows;
    d.n_mt = (uint32_t)n_mt, d.n_rt = (uint32_t)n_rt;
    d.n_fwd = (uint32_t)n_fwd, d.n_mac = (uint32_t)n_mac, d.n_inv = (uint32_t)n_inv;
    total += n_fwd + n_mac + n_inv;
    b->jobs.push_back(d);
  }
  if (total >= 0xffffffffull) {
    free_batch(b);
    return HE_ESHAPE;
  }
  // work list: every item's prerequisites come before it
  std::vector<BatchItem> items;
  items.reserve(total);
  if (schedule == HE_SCHED_PHASED) {
    for (uint32_t j = 0; j < n_jobs; j++) emit(items, j, heconv::ITEM_FWD, b->jobs[j].n_fwd);
    for (uint32_t j = 0; j < n_jobs; j++) emit(items, j, heconv::ITEM_MAC, b->jobs[j].n_mac);
    for (uint32_t j = 0; j < n_jobs; j++) emit(items, j, heconv::ITEM_INV, b->jobs[j].n_inv);
  } else {
    // software pipeline over jobs: forward NTTs of job s, MACs of job s-1
    // and inverse NTTs of job s-2 are adjacent in the list, so VALU-bound
    // transforms and HBM-bound MACs of different jobs run side by side
    for (uint32_t s = 0; s < n_jobs + 2; s++) {
      if (s < n_jobs) emit(items, s, heconv::ITEM_FWD, b->jobs[s].n_fwd);
      if (s >= 1 && s - 1 < n_jobs) emit(items, s - 1, heconv::ITEM_MAC, b->jobs[s - 1].n_mac);
      if (s >= 2 && s - 2 < n_jobs) emit(items, s - 2, heconv::ITEM_INV, b->jobs[s - 2].n_inv);
    }
  }
  b->n_items = (uint32_t)items.size();
  b->n_jobs = n_jobs;
  b->n_ctr = (2 + 2 * n_jobs) * heconv::CTR_STRIDE;
  int per_cu = 0, cus = 0;
  if (heconv::batch_occupancy(c->logN, &per_cu) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) {
    free_batch(b);
    return HE_EDEVICE;
  }
  b->grid = (uint32_t)std::max<int64_t>(1, std::min<int64_t>((int64_t)per_cu * cus, b->n_items));
  if (hipMalloc(&b->d_jobs, sizeof(BatchJob) * n_jobs) != hipSuccess ||
      hipMalloc(&b->d_items, sizeof(BatchItem) * items.size()) != hipSuccess ||
      hipMalloc(&b->d_ctr, sizeof(uint32_t) * b->n_ctr) != hipSuccess) {
    free_batch(b);
    return HE_ENOMEM;
  }
  if (hipMemcpy(b->d_jobs, b->jobs.data(), sizeof(BatchJob) * n_jobs, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice) != hipSuccess) {
    free_batch(b);
    return HE_EDEVICE;
  }
  *out = b;
  return HE_OK;
}

he_status he_batch_launch(he_batch* b, void* stream, int use_graph) {
  if (!b) return HE_EINVAL;
  const heconv::BatchLaunch a = launch_args(b);
  if (!use_graph) return heconv::batch_launch(b->ctx->logN, a, (hipStream_t)stream) == hipSuccess ? HE_OK : HE_EDEVICE;
  if (!b->exec) {
    // capture the reset kernel and the persistent kernel once, on a
    // private stream; the instantiated graph is replayed on any stream
    if (!b->cap && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) return HE_EDEVICE;
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return HE_EDEVICE;
    const hipError_t le = heconv::batch_launch(b->ctx->logN, a, b->cap);
    const hipError_t ce = hipStreamEndCapture(b->cap, &b->graph);
    if (le != hipSuccess || ce != hipSuccess) return HE_EDEVICE;
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) return HE_EDEVICE;
  }
  return hipGraphLaunch(b->exec, (hipStream_t)stream) == hipSuccess ? HE_OK : HE_EDEVICE;
}

he_status he_batch_status(he_batch* b, void* stream) {
  if (!b) return HE_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return HE_EDEVICE;
  uint32_t err = 0;
  if (hipMemcpy(&err, b->d_ctr + heconv::CTR_STRIDE, sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return HE_EDEVICE;
  return err ? HE_EDEVICE : HE_OK;
}

he_status he_batch_counters(he_batch* b, void* stream, uint32_t* out, uint32_t n) {
  if (!b || !out || n < 4 + 2 * b->n_jobs) return HE_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return HE_EDEVICE;
  std::vector<uint32_t> h(b->n_ctr);
  if (hipMemcpy(h.data(), b->d_ctr, sizeof(uint32_t) * b->n_ctr, hipMemcpyDeviceToHost) != hipSuccess)
    return HE_EDEVICE;
  const uint32_t S = heconv::CTR_STRIDE;
  out[0] = h[0], out[1] = h[S], out[2] = h[S + 1], out[3] = h[S + 2];
  for (uint32_t j = 0; j < b->n_jobs; j++) {
    out[4 + 2 * j] = h[(2 + 2 * j) * S];
    out[5 + 2 * j] = h[(3 + 2 * j) * S];
  }
  return HE_OK;
}

he_status he_batch_info(const he_batch* b, uint64_t* n_items, uint32_t* n_workgroups) {
  if (!b) return HE_EINVAL;
  if (n_items) *n_items = b->n_items;
  if (n_workgroups) *n_workgroups = b->grid;
  return HE_OK;
}

he_status he_batch_set_spin_limit(he_batch* b, uint32_t limit) {
  if (!b || limit == 0) return HE_EINVAL;
  if (b->exec) return HE_EBUSY;  // already captured with the old bound
  b->spin_limit = limit;
  return HE_OK;
}

void he_batch_destroy(he_batch* b) { free_batch(b); }

}  // extern "C"
