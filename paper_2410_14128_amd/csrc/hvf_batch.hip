// Batched launches: descriptor tables on the device, graph capture and replay, tuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "hvf_internal.h"

namespace hvf {
hvf_status launch_trace_batch(const BatchItem* d_items, const uint32_t* d_dinfo, uint32_t nitems, uint32_t total,
                              int max_depth, int kinds, uint32_t* d_counter, uint32_t refill, uint32_t inner, unsigned grid,
                              hipStream_t s);
hvf_status batch_grid(uint32_t nitems, int max_depth, int kinds, int blocks_per_cu, unsigned* grid);
}  // namespace hvf

struct hvf_batch {
  std::vector<hvf::BatchItem> items;
  std::vector<uint32_t> dinfo;
  hvf::BatchItem* d_items = nullptr;
  uint32_t* d_dinfo = nullptr;
  uint32_t* d_counter = nullptr;
  uint32_t total = 0;
  int max_depth = 1;
  int kinds = 0;  // hvf::batch_kernel_code of its volumes: picks the kernel
  hvf_batch_opts opts{16, 8, 0, 1};
  unsigned grid = 0;
  hipStream_t cap = nullptr;  // private stream used for graph capture
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

hvf_status fail(hvf_status s, const std::string& m) {
  hvf_set_error(m);
  return s;
}
hvf_status hipf(hipError_t e, const char* what) {
  hvf_set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? HVF_E_NOMEM : HVF_E_DEVICE;
}

hvf_status check_opts(const hvf_batch_opts& o) {
  if (o.refill < 1 || o.refill > 64 || o.inner < 1 || o.inner > 4096 || o.blocks_per_cu < 0 || o.blocks_per_cu > 64 ||
      o.use_graph < 0 || o.use_graph > 1)
    return fail(HVF_E_INPUT, "batch option out of range");
  return HVF_OK;
}

void drop_graph(hvf_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

hvf_status launch(hvf_batch* b, hipStream_t s) {
  return hvf::launch_trace_batch(b->d_items, b->d_dinfo, (uint32_t)b->items.size(), b->total, b->max_depth, b->kinds,
                                 b->d_counter, (uint32_t)b->opts.refill, (uint32_t)b->opts.inner, b->grid, s);
}

// Capture counter reset + kernel into a graph on the private stream.
hvf_status capture(hvf_batch* b) {
  drop_graph(b);
  hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hipf(e, "hipStreamBeginCapture");
  hvf_status st = launch(b, b->cap);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->cap, &g);
  if (st != HVF_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hipf(e, "hipStreamEndCapture");
  b->graph = g;
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(b);
    return hipf(e, "hipGraphInstantiate");
  }
  return HVF_OK;
}

hvf_status configure(hvf_batch* b) {
  hvf_status st = hvf::batch_grid((uint32_t)b->items.size(), b->max_depth, b->kinds, b->opts.blocks_per_cu, &b->grid);
  if (st != HVF_OK) return st;
  if (b->opts.use_graph) return capture(b);
  drop_graph(b);
  return HVF_OK;
}

}  // namespace

extern "C" {

hvf_status hvf_batch_create(hvf_volume* const* vols, const hvf_ray* const* d_rays, const size_t* n,
                            hvf_hit* const* d_hits, size_t m, const hvf_batch_opts* opts, hvf_batch** out) {
  if (!out || !vols || !d_rays || !n || !d_hits) return fail(HVF_E_INPUT, "null argument");
  if (m < 1 || m > (size_t)hvf::HVF_BATCH_MAX_ITEMS) return fail(HVF_E_INPUT, "a batch holds 1..256 ray batches");
  hvf_batch_opts o = opts ? *opts : hvf_batch_opts{16, 8, 0, 1};
  hvf_status st = check_opts(o);
  if (st != HVF_OK) return st;
  hvf_batch* b = new (std::nothrow) hvf_batch();
  if (!b) return fail(HVF_E_NOMEM, "host allocation failed");
  b->opts = o;
  uint64_t total = 0;
  int common = -1;  // the kernel family every volume shares, else -1
  bool regions = false;  // some volume has per-depth regions
  for (size_t i = 0; i < m; ++i) {
    if (!vols[i] || (n[i] && (!d_rays[i] || !d_hits[i]))) {
      delete b;
      return fail(HVF_E_INPUT, "null volume or buffer in batch " + std::to_string(i));
    }
    st = hvf_upload(vols[i], nullptr);
    if (st != HVF_OK) {
      delete b;
      return st;
    }
    const hvf::DevFormat F = hvf::make_devformat(vols[i]->layout, vols[i]->spec, vols[i]->dbuf);
    hvf::BatchItem it{};
    it.buf = F.buf;
    it.rays = d_rays[i];
    it.hits = d_hits[i];
    it.pop_lut = F.pop_lut;
    it.first = (uint32_t)total;
    it.n = (uint32_t)n[i];
    for (int a = 0; a < 3; ++a) it.ext[a] = F.ext[a];
    it.ndepth = F.ndepth;
    it.stacked = F.stacked;
    it.rtab = hvf::device_region_table(vols[i]);
    regions = regions || vols[i]->built.regions;
    b->max_depth = std::max(b->max_depth, F.ndepth);
    b->kinds = std::max(b->kinds, hvf::batch_kinds(vols[i]->spec, vols[i]->layout));
    const int f = hvf::volume_family(vols[i]->spec, vols[i]->layout);
    common = (i == 0 || common == f) ? f : -1;
    b->items.push_back(it);
    b->dinfo.insert(b->dinfo.end(), F.dinfo, F.dinfo + HVF_MAX_DEPTH);
    total += n[i];
  }
  if (total >= (1ull << 31)) {
    delete b;
    return fail(HVF_E_INPUT, "a batched launch holds fewer than 2^31 rays");
  }
  b->total = (uint32_t)total;
  b->kinds = hvf::batch_kernel_code(b->kinds, common, regions);
  hipError_t e = hipMalloc(&b->d_items, b->items.size() * sizeof(hvf::BatchItem));
  if (e == hipSuccess) e = hipMalloc(&b->d_dinfo, b->dinfo.size() * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&b->d_counter, 64 * sizeof(uint32_t));
  if (e == hipSuccess)
    e = hipMemcpy(b->d_items, b->items.data(), b->items.size() * sizeof(hvf::BatchItem), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_dinfo, b->dinfo.data(), b->dinfo.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    st = hipf(e, "batch setup");
    hvf_batch_free(b);
    return st;
  }
  st = configure(b);
  if (st != HVF_OK) {
    hvf_batch_free(b);
    return st;
  }
  *out = b;
  return HVF_OK;
}

hvf_status hvf_batch_run(hvf_batch* b, void* stream) {
  if (!b) return fail(HVF_E_INPUT, "null batch");
  if (b->total == 0) return HVF_OK;
  if (b->exec) {
    const hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    return e == hipSuccess ? HVF_OK : hipf(e, "hipGraphLaunch");
  }
  return launch(b, (hipStream_t)stream);
}

hvf_status hvf_batch_autotune(hvf_batch* b, void* stream, hvf_batch_opts* out) {
  if (!b) return fail(HVF_E_INPUT, "null batch");
  hipStream_t s = (hipStream_t)stream;
  const hvf_batch_opts keep = b->opts;
  std::vector<hvf_batch_opts> cand;
  for (int refill : {4, 16, 32})
    for (int inner : {2, 8, 32})
      for (int bpc : {0, 4}) cand.push_back(hvf_batch_opts{refill, inner, bpc, keep.use_graph});
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(HVF_E_DEVICE, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(HVF_E_DEVICE, "hipEventCreate failed");
  }
  float best = 1e30f;
  hvf_batch_opts pick = keep;
  hvf_status st = HVF_OK;
  for (const hvf_batch_opts& c : cand) {
    b->opts = c;
    st = configure(b);
    if (st != HVF_OK) break;
    st = hvf_batch_run(b, stream);  // warm-up
    float ms = 0.0f;
    const int reps = 3;
    bool ok = st == HVF_OK && hipEventRecord(e0, s) == hipSuccess;
    for (int r = 0; r < reps && ok; ++r) ok = hvf_batch_run(b, stream) == HVF_OK;
    ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
         hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    if (!ok) {
      st = (st != HVF_OK) ? st : fail(HVF_E_DEVICE, "batch autotune timing failed");
      break;
    }
    if (ms / reps < best) {
      best = ms / reps;
      pick = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->opts = (st == HVF_OK) ? pick : keep;
  const hvf_status st2 = configure(b);
  if (st != HVF_OK) return st;
  if (st2 != HVF_OK) return st2;
  if (out) *out = b->opts;
  return HVF_OK;
}

void hvf_batch_free(hvf_batch* b) {
  if (!b) return;
  if (b->cap) (void)hipStreamSynchronize(b->cap);
  (void)hipDeviceSynchronize();
  drop_graph(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_dinfo) (void)hipFree(b->d_dinfo);
  if (b->d_counter) (void)hipFree(b->d_counter);
  delete b;
}

}  // extern "C"
