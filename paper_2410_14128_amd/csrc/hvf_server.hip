// Serving: resident volumes, memory-gated admission, continuous batching on the device.
//
// Requests (a volume id and a host ray array) queue in arrival order. An engine thread
// admits them while request slots and device memory allow (each admitted request holds
// 48 bytes per ray of a fixed device arena, and the same of a pinned staging arena),
// and packs every admitted, not yet launched request into the next "step": one batched
// persistent launch (the kernel of hvf_batch) on one of several streams, bracketed by
// the ray upload and the hit download. Requests that arrive while steps run are admitted
// into the following step, so work of different requests overlaps on the device. When a
// step's event completes, its requests' hits are copied to the callers' arrays, their
// memory and slots are returned, and their latency (submission to completion) recorded.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hvf_internal.h"

namespace hvf {
hvf_status launch_trace_batch(const BatchItem* d_items, const uint32_t* d_dinfo, uint32_t nitems, uint32_t total,
                              int max_depth, int kinds, uint32_t* d_counter, uint32_t refill, uint32_t inner, unsigned grid,
                              hipStream_t s);
hvf_status batch_grid(uint32_t nitems, int max_depth, int kinds, int blocks_per_cu, unsigned* grid);
}  // namespace hvf

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

// First-fit allocator over [0, size) with coalescing; 256-byte granules.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  size_t size_, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

struct Request {
  uint64_t id = 0;
  int vol = 0;
  size_t n = 0;
  const hvf_ray* src = nullptr;  // caller's host rays (valid until completion)
  hvf_hit* out = nullptr;        // caller's host hit array; null: kept in staging until released
  bool src_pinned = false;       // rays are in pinned host memory: DMA without staging
  bool released = false;
  size_t off = 0;             // arena offset (rays, then hits)
  Clock::time_point t_submit, t_admit, t_done;
  bool done = false;
  hvf_status status = HVF_OK;
};

struct Step {
  hipStream_t stream = nullptr;
  hipEvent_t done_ev = nullptr;
  hvf::BatchItem* d_items = nullptr;
  uint32_t* d_dinfo = nullptr;
  uint32_t* d_counter = nullptr;
  hvf::BatchItem* h_items = nullptr;  // pinned
  uint32_t* h_dinfo = nullptr;        // pinned
  std::vector<std::shared_ptr<Request>> reqs;
  bool busy = false;
};

}  // namespace

struct hvf_server {
  size_t budget = 0;
  int max_slots = 1;
  int max_steps = 1;
  hvf_batch_opts opts{16, 8, 0, 0};
  uint8_t* d_arena = nullptr;  // device
  uint8_t* h_arena = nullptr;  // pinned host staging, same offsets
  std::unique_ptr<Arena> arena;
  std::vector<hvf_volume*> vols;  // capacity reserved at creation: never reallocated
  std::vector<Step> steps;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<std::shared_ptr<Request>> pending;
  std::vector<std::shared_ptr<Request>> admitted;  // admitted, not yet launched
  std::unordered_map<uint64_t, std::shared_ptr<Request>> all;
  std::vector<double> lat;
  uint64_t next_id = 1;
  int slots_used = 0;
  uint64_t rays_done = 0, admission_waits = 0, steps_launched = 0, max_step_requests = 0;
  bool have_first = false;
  Clock::time_point t_first, t_last;
  bool stop = false;
  int fail_steps = 0;  // testing: steps still to fail at launch (hvf_server_fail_steps)
  hvf_status fault = HVF_OK;
  std::string fault_msg;
  std::thread engine;
  int device = 0;
};

namespace {

hvf_status fail(hvf_status s, const std::string& m) {
  hvf_set_error(m);
  return s;
}

size_t req_bytes(size_t n) {
  return std::max<size_t>(256, ((n * sizeof(hvf_ray) + 255) & ~(size_t)255) + n * sizeof(hvf_hit));
}

// Launch one step with the given requests (engine thread, lock not held).
hvf_status launch_step(hvf_server* S, Step& st) {
  const size_t m = st.reqs.size();
  uint64_t total = 0;
  int max_depth = 1;
  int kinds = 0;
  int common = -1;  // the kernel family every request's volume shares, else -1
  bool regions = false;  // some request's volume has per-depth regions
  for (size_t i = 0; i < m; ++i) {
    Request& r = *st.reqs[i];
    hvf_volume* v = S->vols[r.vol];
    regions = regions || v->built.regions;
    kinds = std::max(kinds, hvf::batch_kinds(v->spec, v->layout));
    const int f = hvf::volume_family(v->spec, v->layout);
    common = (i == 0 || common == f) ? f : -1;
    const hvf::DevFormat F = hvf::make_devformat(v->layout, v->spec, v->dbuf);
    uint8_t* hr = S->h_arena + r.off;
    if (r.n && !r.src_pinned) std::memcpy(hr, r.src, r.n * sizeof(hvf_ray));
    const size_t hit_off = r.off + ((r.n * sizeof(hvf_ray) + 255) & ~(size_t)255);
    hvf::BatchItem it{};
    it.buf = F.buf;
    it.rays = S->d_arena + r.off;
    it.hits = S->d_arena + hit_off;
    it.pop_lut = F.pop_lut;
    it.first = (uint32_t)total;
    it.n = (uint32_t)r.n;
    for (int a = 0; a < 3; ++a) it.ext[a] = F.ext[a];
    it.ndepth = F.ndepth;
    it.stacked = F.stacked;
    it.rtab = hvf::device_region_table(v);
    st.h_items[i] = it;
    std::memcpy(st.h_dinfo + i * HVF_MAX_DEPTH, F.dinfo, sizeof(F.dinfo));
    max_depth = std::max(max_depth, F.ndepth);
    total += r.n;
  }
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < m && e == hipSuccess; ++i) {
    const Request& r = *st.reqs[i];
    const void* from = r.src_pinned ? (const void*)r.src : (const void*)(S->h_arena + r.off);
    e = hipMemcpyAsync(S->d_arena + r.off, from, r.n * sizeof(hvf_ray), hipMemcpyHostToDevice, st.stream);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(st.d_items, st.h_items, m * sizeof(hvf::BatchItem), hipMemcpyHostToDevice, st.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(st.d_dinfo, st.h_dinfo, m * HVF_MAX_DEPTH * sizeof(uint32_t), hipMemcpyHostToDevice, st.stream);
  if (e != hipSuccess) return fail(HVF_E_DEVICE, std::string("server upload: ") + hipGetErrorString(e));
  unsigned grid = 0;
  kinds = hvf::batch_kernel_code(kinds, common, regions);
  hvf_status s = hvf::batch_grid((uint32_t)m, max_depth, kinds, S->opts.blocks_per_cu, &grid);
  if (s != HVF_OK) return s;
  if (total)
    s = hvf::launch_trace_batch(st.d_items, st.d_dinfo, (uint32_t)m, (uint32_t)total, max_depth, kinds, st.d_counter,
                                (uint32_t)S->opts.refill, (uint32_t)S->opts.inner, grid, st.stream);
  if (s != HVF_OK) return s;
  for (size_t i = 0; i < m && e == hipSuccess; ++i) {
    const Request& r = *st.reqs[i];
    const size_t hit_off = r.off + ((r.n * sizeof(hvf_ray) + 255) & ~(size_t)255);
    e = hipMemcpyAsync(S->h_arena + hit_off, S->d_arena + hit_off, r.n * sizeof(hvf_hit), hipMemcpyDeviceToHost,
                       st.stream);
  }
  if (e == hipSuccess) e = hipEventRecord(st.done_ev, st.stream);
  if (e != hipSuccess) return fail(HVF_E_DEVICE, std::string("server step: ") + hipGetErrorString(e));
  return HVF_OK;
}

void engine_loop(hvf_server* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    bool progressed = false;
    // 1. Completions.
    for (Step& st : S->steps) {
      if (!st.busy) continue;
      const hipError_t q = hipEventQuery(st.done_ev);
      if (q == hipErrorNotReady) continue;
      const auto now = Clock::now();
      for (auto& rp : st.reqs) {
        Request& r = *rp;
        if (q == hipSuccess) {
          const size_t hit_off = r.off + ((r.n * sizeof(hvf_ray) + 255) & ~(size_t)255);
          if (r.out) std::memcpy(r.out, S->h_arena + hit_off, r.n * sizeof(hvf_hit));
        } else {
          r.status = HVF_E_DEVICE;
        }
        r.t_done = now;
        r.done = true;
        if (r.out || r.released) S->arena->release(r.off, req_bytes(r.n));  // else held until released
        S->slots_used -= 1;
        S->lat.push_back(ms_between(r.t_submit, r.t_done));
        S->rays_done += r.n;
        S->t_last = now;
      }
      if (q != hipSuccess) {
        S->fault = HVF_E_DEVICE;
        S->fault_msg = std::string("server step failed: ") + hipGetErrorString(q);
      }
      st.reqs.clear();
      st.busy = false;
      progressed = true;
      S->cv_done.notify_all();
    }
    // 2. Admission in arrival order, gated by slots and memory.
    while (!S->pending.empty() && S->slots_used < S->max_slots) {
      auto& r = S->pending.front();
      size_t off = 0;
      if (!S->arena->alloc(req_bytes(r->n), &off)) {
        ++S->admission_waits;
        break;
      }
      r->off = off;
      r->t_admit = Clock::now();
      S->slots_used += 1;
      S->admitted.push_back(r);
      S->pending.pop_front();
      progressed = true;
    }
    // 3. Launch every admitted request as one step on a free stream.
    if (!S->admitted.empty()) {
      for (Step& st : S->steps) {
        if (st.busy) continue;
        const size_t take = std::min<size_t>(S->admitted.size(), hvf::HVF_BATCH_MAX_ITEMS);
        st.reqs.assign(S->admitted.begin(), S->admitted.begin() + take);
        S->admitted.erase(S->admitted.begin(), S->admitted.begin() + take);
        st.busy = true;
        S->steps_launched += 1;
        S->max_step_requests = std::max<uint64_t>(S->max_step_requests, take);
        const bool inject = S->fail_steps > 0;
        if (inject) --S->fail_steps;
        lk.unlock();
        const hvf_status s = inject ? fail(HVF_E_DEVICE, "injected step failure (hvf_server_fail_steps)")
                                    : launch_step(S, st);
        lk.lock();
        if (s != HVF_OK) {
          // Nothing was recorded on done_ev: finish the step's requests here with the
          // error, after the copies it may have enqueued (their staging ranges are freed).
          (void)hipStreamSynchronize(st.stream);
          const auto now = Clock::now();
          for (auto& rp : st.reqs) {
            Request& r = *rp;
            r.status = s;
            r.t_done = now;
            r.done = true;
            if (r.out || r.released) S->arena->release(r.off, req_bytes(r.n));  // else held until released
            S->slots_used -= 1;
          }
          st.reqs.clear();
          st.busy = false;
          S->fault = s;
          S->fault_msg = hvf_last_error();
          S->cv_done.notify_all();
        }
        progressed = true;
        break;
      }
    }
    if (S->stop && S->pending.empty() && S->admitted.empty()) {
      bool any = false;
      for (Step& st : S->steps) any = any || st.busy;
      if (!any) break;
    }
    if (!progressed) {
      bool any_busy = false;
      for (Step& st : S->steps) any_busy = any_busy || st.busy;
      if (any_busy)
        S->cv.wait_for(lk, std::chrono::microseconds(20));
      else
        S->cv.wait(lk);
    }
  }
}

}  // namespace

extern "C" {

hvf_status hvf_server_create(size_t mem_budget_bytes, int max_slots, int max_steps, const hvf_batch_opts* opts,
                             hvf_server** out) {
  if (!out) return fail(HVF_E_INPUT, "null output pointer");
  if (mem_budget_bytes < 4096 || max_slots < 1 || max_steps < 1 || max_steps > 8)
    return fail(HVF_E_INPUT, "budget >= 4096 bytes, slots >= 1, 1 <= in-flight steps <= 8");
  hvf_server* S = new (std::nothrow) hvf_server();
  if (!S) return fail(HVF_E_NOMEM, "host allocation failed");
  S->budget = (mem_budget_bytes + 255) & ~(size_t)255;
  S->vols.reserve(HVF_SERVER_MAX_VOLUMES);
  S->max_slots = max_slots;
  S->max_steps = max_steps;
  if (opts) S->opts = *opts;
  if (S->opts.refill < 1 || S->opts.refill > 64 || S->opts.inner < 1) {
    delete S;
    return fail(HVF_E_INPUT, "batch option out of range");
  }
  (void)hipGetDevice(&S->device);
  hipError_t e = hipMalloc(&S->d_arena, S->budget);
  if (e == hipSuccess) e = hipHostMalloc(&S->h_arena, S->budget, hipHostMallocDefault);
  S->arena.reset(new Arena(S->budget));
  S->steps.resize(max_steps);
  for (Step& st : S->steps) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&st.done_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&st.d_items, hvf::HVF_BATCH_MAX_ITEMS * sizeof(hvf::BatchItem));
    if (e == hipSuccess) e = hipMalloc(&st.d_dinfo, hvf::HVF_BATCH_MAX_ITEMS * HVF_MAX_DEPTH * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&st.d_counter, 64 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipHostMalloc(&st.h_items, hvf::HVF_BATCH_MAX_ITEMS * sizeof(hvf::BatchItem), hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc(&st.h_dinfo, hvf::HVF_BATCH_MAX_ITEMS * HVF_MAX_DEPTH * sizeof(uint32_t), hipHostMallocDefault);
  }
  if (e != hipSuccess) {
    const std::string msg = std::string("server setup: ") + hipGetErrorString(e);
    hvf_server_destroy(S);
    return fail(e == hipErrorOutOfMemory ? HVF_E_NOMEM : HVF_E_DEVICE, msg);
  }
  S->engine = std::thread(engine_loop, S);
  *out = S;
  return HVF_OK;
}

hvf_status hvf_server_add_volume(hvf_server* S, hvf_volume* v, int* vol_id) {
  if (!S || !v || !vol_id) return fail(HVF_E_INPUT, "null argument");
  hvf_status st = hvf_upload(v, nullptr);
  if (st != HVF_OK) return st;
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->vols.size() >= HVF_SERVER_MAX_VOLUMES) return fail(HVF_E_INPUT, "too many volumes");
  S->vols.push_back(v);
  *vol_id = (int)S->vols.size() - 1;
  return HVF_OK;
}

hvf_status hvf_server_submit(hvf_server* S, int vol_id, const hvf_ray* rays, size_t n, hvf_hit* hits,
                             uint64_t* req_id) {
  if (!S || !req_id || (n && !rays)) return fail(HVF_E_INPUT, "null argument");
  auto r = std::make_shared<Request>();
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->fault != HVF_OK) return fail(S->fault, S->fault_msg);
  if (vol_id < 0 || vol_id >= (int)S->vols.size()) return fail(HVF_E_INPUT, "unknown volume id");
  if (req_bytes(n) > S->budget)
    return fail(HVF_E_NOMEM, "request needs " + std::to_string(req_bytes(n)) + " bytes, above the server budget");
  if (n >= (1ull << 31)) return fail(HVF_E_INPUT, "request too large");
  r->id = S->next_id++;
  r->vol = vol_id;
  r->n = n;
  r->out = hits;
  r->src = rays;
  if (n) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, rays) == hipSuccess && attr.type == hipMemoryTypeHost) r->src_pinned = true;
    (void)hipGetLastError();  // a pageable pointer is not an error here
  }
  if (!S->have_first) {
    S->have_first = true;
    S->t_first = r->t_submit;
  }
  S->all[r->id] = r;
  S->pending.push_back(r);
  *req_id = r->id;
  S->cv.notify_all();
  return HVF_OK;
}

hvf_status hvf_server_poll(hvf_server* S, uint64_t req_id, int* done, double* latency_ms) {
  if (!S || !done) return fail(HVF_E_INPUT, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(req_id);
  if (it == S->all.end()) return fail(HVF_E_INPUT, "unknown request id");
  *done = it->second->done ? 1 : 0;
  if (it->second->done && latency_ms) *latency_ms = ms_between(it->second->t_submit, it->second->t_done);
  if (it->second->done && it->second->status != HVF_OK) return fail(it->second->status, "request failed on the device");
  return HVF_OK;
}

hvf_status hvf_server_wait(hvf_server* S, uint64_t req_id, double* latency_ms) {
  if (!S) return fail(HVF_E_INPUT, "null server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->all.find(req_id);
  if (it == S->all.end()) return fail(HVF_E_INPUT, "unknown request id");
  auto r = it->second;
  S->cv_done.wait(lk, [&] { return r->done || S->fault != HVF_OK; });
  if (!r->done) return fail(S->fault, S->fault_msg);
  if (latency_ms) *latency_ms = ms_between(r->t_submit, r->t_done);
  return r->status == HVF_OK ? HVF_OK : fail(r->status, "request failed on the device");
}

hvf_status hvf_server_result(hvf_server* S, uint64_t req_id, const hvf_hit** hits) {
  if (!S || !hits) return fail(HVF_E_INPUT, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(req_id);
  if (it == S->all.end()) return fail(HVF_E_INPUT, "unknown request id");
  const Request& r = *it->second;
  if (!r.done) return fail(HVF_E_STATE, "request not complete");
  if (r.out || r.released) return fail(HVF_E_STATE, "request results are not held by the server");
  *hits = reinterpret_cast<const hvf_hit*>(S->h_arena + r.off + ((r.n * sizeof(hvf_ray) + 255) & ~(size_t)255));
  return HVF_OK;
}

hvf_status hvf_server_release(hvf_server* S, uint64_t req_id) {
  if (!S) return fail(HVF_E_INPUT, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(req_id);
  if (it == S->all.end()) return fail(HVF_E_INPUT, "unknown request id");
  Request& r = *it->second;
  if (!r.done) return fail(HVF_E_STATE, "request not complete");
  if (!r.out && !r.released) S->arena->release(r.off, req_bytes(r.n));
  r.released = true;
  S->all.erase(it);
  S->cv.notify_all();
  return HVF_OK;
}

hvf_status hvf_server_fail_steps(hvf_server* S, int n) {
  if (!S || n < 0) return fail(HVF_E_INPUT, "null server or negative count");
  std::lock_guard<std::mutex> lk(S->mu);
  S->fail_steps = n;
  return HVF_OK;
}

hvf_status hvf_server_drain(hvf_server* S) {
  if (!S) return fail(HVF_E_INPUT, "null server");
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_done.wait(lk, [&] {
    if (S->fault != HVF_OK) return true;
    if (!S->pending.empty() || !S->admitted.empty()) return false;
    for (const Step& st : S->steps)
      if (st.busy) return false;
    return true;
  });
  return S->fault == HVF_OK ? HVF_OK : fail(S->fault, S->fault_msg);
}

hvf_status hvf_server_stats(hvf_server* S, hvf_serve_stats* out) {
  if (!S || !out) return fail(HVF_E_INPUT, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  hvf_serve_stats st;
  std::memset(&st, 0, sizeof(st));
  std::vector<double> l = S->lat;
  std::sort(l.begin(), l.end());
  st.completed = l.size();
  auto pct = [&](double p) {
    if (l.empty()) return 0.0;
    const size_t k = (size_t)std::min<double>((double)l.size() - 1, std::ceil(p * (double)l.size()) - 1);
    return l[k];
  };
  st.p50_ms = pct(0.50);
  st.p99_ms = pct(0.99);
  double sum = 0;
  for (double x : l) sum += x;
  st.mean_ms = l.empty() ? 0.0 : sum / (double)l.size();
  st.max_ms = l.empty() ? 0.0 : l.back();
  st.rays = S->rays_done;
  const double span = S->have_first && st.completed ? ms_between(S->t_first, S->t_last) : 0.0;
  st.span_ms = span;
  st.mrays_s = span > 0 ? (double)S->rays_done / span / 1e3 : 0.0;
  st.steps = S->steps_launched;
  st.admission_waits = S->admission_waits;
  st.peak_bytes = S->arena->peak();
  st.budget_bytes = S->budget;
  st.max_step_requests = S->max_step_requests;
  *out = st;
  return HVF_OK;
}

void hvf_server_destroy(hvf_server* S) {
  if (!S) return;
  if (S->engine.joinable()) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stop = true;
      S->cv.notify_all();
    }
    S->engine.join();
  }
  for (Step& st : S->steps) {
    if (st.stream) (void)hipStreamSynchronize(st.stream);
    if (st.done_ev) (void)hipEventDestroy(st.done_ev);
    if (st.stream) (void)hipStreamDestroy(st.stream);
    if (st.d_items) (void)hipFree(st.d_items);
    if (st.d_dinfo) (void)hipFree(st.d_dinfo);
    if (st.d_counter) (void)hipFree(st.d_counter);
    if (st.h_items) (void)hipHostFree(st.h_items);
    if (st.h_dinfo) (void)hipHostFree(st.h_dinfo);
  }
  if (S->d_arena) (void)hipFree(S->d_arena);
  if (S->h_arena) (void)hipHostFree(S->h_arena);
  delete S;
}

}  // extern "C"
