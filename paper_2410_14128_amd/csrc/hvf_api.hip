// C-ABI entry points: build, upload, trace, info, save/load, errors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hvf_internal.h"

namespace hvf {
hvf_status launch_trace(const DevFormat& F, int family, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits,
                        bool interleave, hipStream_t s);
hvf_status launch_trace_count(const DevFormat& F, bool paper, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits, uint32_t* d_log,
                              uint32_t cap, uint32_t* d_count, uint32_t* d_steps, hipStream_t s);
hvf_status launch_trace_persistent(const DevFormat& F, int family, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits,
                                   uint32_t* d_counter, uint32_t refill, uint32_t inner, unsigned grid, hipStream_t s);
hvf_status persistent_grid(const DevFormat& F, int blocks_per_cu, unsigned* grid);
hvf_status launch_trace_split(const DevFormat& F, int family, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits,
                              uint32_t budget, uint32_t klog2, uint32_t rounds, uint32_t* scratch, hipStream_t s);
hvf_status launch_trace_steal(const DevFormat& F, int family, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits,
                              uint32_t period, float minlen, uint32_t min_idle, bool interleave, uint32_t rays_per_wave,
                              hipStream_t s);
hipError_t scratch_alloc(void** p, size_t bytes, hipStream_t s);
hvf_status launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t s);
hvf_status trace_sorted(const DevFormat& F, int family, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits,
                        const hvf_schedule& sc, hipStream_t s);
}

namespace {
thread_local std::string g_err;

hvf_status fail(hvf_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

hvf_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return (e == hipErrorOutOfMemory) ? HVF_E_NOMEM : HVF_E_DEVICE;
}

uint64_t fnv64(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

const char MAGIC[8] = {'H', 'V', 'F', 'W', 'O', 'R', 'D', '1'};
}  // namespace

void hvf_set_error(const std::string& s) { g_err = s; }

extern "C" {

const char* hvf_last_error(void) { return g_err.c_str(); }

const char* hvf_status_string(hvf_status s) {
  switch (s) {
    case HVF_OK: return "ok";
    case HVF_E_SPEC: return "malformed format spec";
    case HVF_E_INPUT: return "invalid input";
    case HVF_E_OVERFLOW: return "format exceeds 2^32 words";
    case HVF_E_NOMEM: return "out of memory";
    case HVF_E_DEVICE: return "HIP device error";
    case HVF_E_UNSUPPORTED: return "unsupported format";
    case HVF_E_STATE: return "invalid state";
  }
  return "unknown status";
}

hvf_status hvf_build(const char* format_spec, const uint64_t* morton, size_t n, hvf_volume** out) {
  if (!out) return fail(HVF_E_INPUT, "null output handle pointer");
  hvf::Spec spec;
  std::string err;
  hvf_status st = hvf::parse_spec(format_spec, spec, err);
  if (st != HVF_OK) return fail(st, err);
  hvf_volume* v = new (std::nothrow) hvf_volume();
  if (!v) return fail(HVF_E_NOMEM, "host allocation failed");
  v->spec = spec;
  if (spec.paper) {
    v->layout = hvf::make_paper_layout(spec);
    st = hvf::build_paper_words(v->spec, v->layout, morton, n, v->built, err);
  } else {
    v->layout = hvf::make_layout(spec);
    st = hvf::build_words(v->spec, v->layout, morton, n, v->built, err);
    if (st == HVF_OK && v->built.regions && !v->spec.regions) {
      // the builder chose per-depth regions (the format needs 2^32 words or more): the spec
      // says so, so a saved file loads the same way
      v->spec.regions = true;
      v->spec.text += " --depth-buffers";
    }
  }
  if (st != HVF_OK) {
    delete v;
    return fail(st, err);
  }
  *out = v;
  return HVF_OK;
}

hvf_status hvf_upload(hvf_volume* v, void* stream) {
  if (!v) return fail(HVF_E_INPUT, "null volume");
  std::lock_guard<std::mutex> g(v->dev_mu);
  if (v->dbuf) return HVF_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  const size_t nw = v->built.words.size(), bytes = nw * sizeof(uint32_t);
  uint32_t* p = nullptr;
  // Four spare zero words after the buffer: the kernels read 8 bytes at any word index.
  // With per-depth regions, the table of region starts follows (hvf::device_region_table).
  hvf::DevFormat R{};
  hvf::set_regions(R, v->built);
  const size_t alloc_words =
      v->built.regions ? hvf::region_table_word(nw) + 2 * HVF_MAX_DEPTH : nw + HVF_BUFFER_PAD_WORDS;
  e = hipMalloc(&p, alloc_words * sizeof(uint32_t));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc of the word buffer");
  e = hipMemsetAsync(p + nw, 0, HVF_BUFFER_PAD_WORDS * sizeof(uint32_t), (hipStream_t)stream);
  if (e == hipSuccess && v->built.regions)
    e = hipMemcpyAsync(p + hvf::region_table_word(nw), R.rbase, sizeof(R.rbase), hipMemcpyHostToDevice,
                       (hipStream_t)stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p, v->built.words.data(), bytes, hipMemcpyHostToDevice, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) {
    (void)hipFree(p);
    return hip_fail(e, "upload of the word buffer");
  }
  v->dbuf = p;
  v->device = dev;
  return HVF_OK;
}

namespace {
hvf_status check_sched(const hvf_schedule& sc) {
  if (sc.persistent < 0 || sc.persistent > 1 || sc.refill < 1 || sc.refill > 64 || sc.inner < 1 || sc.inner > 4096 ||
      sc.sort < 0 || sc.sort > 1 || sc.sort_bits < 0 || sc.sort_bits > 16 || sc.blocks_per_cu < 0 ||
      sc.blocks_per_cu > 64 || sc.stack_depth < 0 || sc.stack_depth > HVF_MAX_DEPTH || sc.lds_depths < 0 ||
      sc.lds_depths > HVF_MAX_DEPTH || sc.split < 0 || sc.split > 64 || (sc.split & (sc.split - 1)) != 0 ||
      sc.split == 1 || (sc.split && (sc.split_budget < 1 || sc.split_budget > (1 << 20))) || sc.split_rounds < 0 ||
      sc.split_rounds > (int)hvf::HVF_SPLIT_MAX_ROUNDS || (sc.split_rounds && !sc.split) || sc.steal < 0 ||
      sc.steal > 64 || (sc.steal & (sc.steal - 1)) != 0 || (sc.steal && (sc.steal_len < 1 || sc.steal_len > (1 << 20) || sc.steal_idle < 1 || sc.steal_idle > 64)) || sc.interleave < 0 || sc.interleave > 1 || sc.rays_per_wave < 0 ||
      sc.rays_per_wave > 64)
    return fail(HVF_E_INPUT, "schedule field out of range");
  if (sc.rays_per_wave && sc.rays_per_wave < 64 && !(sc.steal && sc.interleave))
    return fail(HVF_E_INPUT, "fewer than 64 rays per wave needs the stealing schedule with interleaved rays");
  if (sc.split && (sc.persistent || sc.sort))
    return fail(HVF_E_INPUT, "the split schedule runs without persistent lanes and without sorting");
  if (sc.steal && (sc.persistent || sc.sort || sc.split))
    return fail(HVF_E_INPUT, "the stealing schedule runs without persistent lanes, sorting or splitting");
  if (sc.interleave && (sc.persistent || sc.sort || sc.split))
    return fail(HVF_E_INPUT, "interleaved rays need one lane per ray: no persistent lanes, sorting or splitting");
  return HVF_OK;
}
}  // namespace

hvf_status hvf_trace_sched(hvf_volume* v, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits, const hvf_schedule* sched,
                           void* stream) {
  if (!v) return fail(HVF_E_INPUT, "null volume");
  const hvf_schedule sc = sched ? *sched : v->sched;
  hvf_status st = check_sched(sc);
  if (st != HVF_OK) return st;
  if (n == 0) return HVF_OK;
  if (!d_rays || !d_hits) return fail(HVF_E_INPUT, "null ray or hit buffer");
  st = hvf_upload(v, stream);
  if (st != HVF_OK) return st;
  if (v->spec.paper && (sc.stack_depth > 0 || sc.lds_depths > 0))
    return fail(HVF_E_INPUT, "short stacks and staged depths need the library's own layout, not --paper-layout");
  hvf::DevFormat F = hvf::make_devformat(v->layout, v->spec, v->dbuf);
  hvf::set_regions(F, v->built);
  if (sc.stack_depth > 0) hvf::set_stacked(F, hvf::stacked_mask(v->layout, v->spec.restart_sv, sc.stack_depth));
  if (!hvf::lds_prefix_words(v->layout, v->built, sc.lds_depths, &F.lds_words))
    return fail(HVF_E_INPUT, "the top " + std::to_string(sc.lds_depths) + " depths exceed the LDS prefix limit of " +
                                 std::to_string(hvf::HVF_LDS_PREFIX_MAX_WORDS) + " words");
  hipStream_t s = (hipStream_t)stream;
  const int family = hvf::volume_family(v->spec, v->layout);
  if (sc.sort) return hvf::trace_sorted(F, family, d_rays, n, d_hits, sc, s);
  if (sc.steal)
    return hvf::launch_trace_steal(F, family, d_rays, n, d_hits, (uint32_t)sc.steal, (float)sc.steal_len,
                                   (uint32_t)sc.steal_idle, sc.interleave != 0, (uint32_t)sc.rays_per_wave, s);
  if (sc.split) {
    const uint32_t budget = (uint32_t)sc.split_budget, klog2 = (uint32_t)__builtin_ctz((unsigned)sc.split),
                   rounds = (uint32_t)sc.split_rounds;
    // The legacy default stream runs its calls in order, so they share the volume's survivor
    // list; a call there that finds the list held by another host thread, and every call on
    // another stream, takes stream-ordered scratch of its own.
    if (s == nullptr) {
      std::unique_lock<std::mutex> g(v->split_mu, std::try_to_lock);
      if (g.owns_lock()) {
        const size_t need = hvf::split_scratch_words(n, rounds);
        if (need > v->split_words) {
          if (v->split_buf) (void)hipFreeAsync(v->split_buf, s);
          v->split_buf = nullptr;
          v->split_words = 0;
          const hipError_t e = hvf::scratch_alloc(reinterpret_cast<void**>(&v->split_buf), need * sizeof(uint32_t), s);
          if (e != hipSuccess) {
            v->split_buf = nullptr;
            return hip_fail(e, "allocation of the split schedule's survivor list");
          }
          v->split_words = need;
        }
        return hvf::launch_trace_split(F, family, d_rays, n, d_hits, budget, klog2, rounds, v->split_buf, s);
      }
    }
    return hvf::launch_trace_split(F, family, d_rays, n, d_hits, budget, klog2, rounds, nullptr, s);
  }
  uint32_t* counter = nullptr;
  if (sc.persistent) {
    {
      std::lock_guard<std::mutex> g(v->dev_mu);
      if (!v->dcounters) {
        hipError_t e = hipMalloc(&v->dcounters, HVF_NUM_COUNTERS * 2 * sizeof(uint32_t));
        if (e != hipSuccess) {
          v->dcounters = nullptr;
          return hip_fail(e, "hipMalloc of ray counters");
        }
      }
    }
    counter = v->dcounters + 2 * (v->counter_next.fetch_add(1) % HVF_NUM_COUNTERS);
  }
  if (!sc.persistent) return hvf::launch_trace(F, family, d_rays, n, d_hits, sc.interleave != 0, s);
  unsigned grid = 0;
  st = hvf::persistent_grid(F, sc.blocks_per_cu, &grid);
  if (st != HVF_OK) return st;
  st = hvf::launch_fill_u32(counter, 0u, 1, s);
  if (st != HVF_OK) return st;
  return hvf::launch_trace_persistent(F, family, d_rays, n, d_hits, counter, (uint32_t)sc.refill, (uint32_t)sc.inner,
                                      grid, s);
}

// The allocation-free split trace: survivor lists in a fixed device array. Host code never
// passes the array's name to a kernel: each device's address comes from hipGetSymbolAddress
// on its first call there, with that device current.
namespace {
constexpr size_t NOALLOC_WORDS = hvf::HVF_SPLIT_HEAD_WORDS + 4 * (size_t)HVF_NOALLOC_MAX_RAYS;
__device__ __align__(256) uint32_t scratch[NOALLOC_WORDS];
constexpr int NOALLOC_MAX_DEVICES = 64;
std::once_flag g_noalloc_once[NOALLOC_MAX_DEVICES];
uint32_t* g_noalloc_ptr[NOALLOC_MAX_DEVICES];
hipError_t g_noalloc_err[NOALLOC_MAX_DEVICES];
}  // namespace

hvf_status hvf_trace_split_noalloc(hvf_volume* v, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits,
                                   const hvf_schedule* sched, void* stream) {
  if (!v) return fail(HVF_E_INPUT, "null volume");
  if (!sched || sched->split == 0) return fail(HVF_E_INPUT, "the allocation-free trace needs a split schedule");
  const hvf_schedule sc = *sched;
  hvf_status st = check_sched(sc);
  if (st != HVF_OK) return st;
  if (n > HVF_NOALLOC_MAX_RAYS)
    return fail(HVF_E_INPUT, "the allocation-free trace takes at most " + std::to_string(HVF_NOALLOC_MAX_RAYS) +
                                 " rays per call, got " + std::to_string(n));
  if (n == 0) return HVF_OK;
  if (!d_rays || !d_hits) return fail(HVF_E_INPUT, "null ray or hit buffer");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  {
    std::lock_guard<std::mutex> g(v->dev_mu);
    if (!v->dbuf) return fail(HVF_E_STATE, "the allocation-free trace needs an uploaded volume (hvf_upload)");
  }
  if (v->device != dev) return fail(HVF_E_STATE, "the volume was uploaded to another device");
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(HVF_E_DEVICE, "device index out of range");
  std::call_once(g_noalloc_once[dev], [dev] {
    void* p = nullptr;
    g_noalloc_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_noalloc_ptr[dev] = g_noalloc_err[dev] == hipSuccess ? static_cast<uint32_t*>(p) : nullptr;
  });
  if (g_noalloc_err[dev] != hipSuccess || !g_noalloc_ptr[dev])
    return hip_fail(g_noalloc_err[dev] != hipSuccess ? g_noalloc_err[dev] : hipErrorInvalidSymbol,
                    "hipGetSymbolAddress of the allocation-free scratch");
  if (v->spec.paper && (sc.stack_depth > 0 || sc.lds_depths > 0))
    return fail(HVF_E_INPUT, "short stacks and staged depths need the library's own layout, not --paper-layout");
  hvf::DevFormat F = hvf::make_devformat(v->layout, v->spec, v->dbuf);
  hvf::set_regions(F, v->built);
  if (sc.stack_depth > 0) hvf::set_stacked(F, hvf::stacked_mask(v->layout, v->spec.restart_sv, sc.stack_depth));
  if (!hvf::lds_prefix_words(v->layout, v->built, sc.lds_depths, &F.lds_words))
    return fail(HVF_E_INPUT, "the top " + std::to_string(sc.lds_depths) + " depths exceed the LDS prefix limit of " +
                                 std::to_string(hvf::HVF_LDS_PREFIX_MAX_WORDS) + " words");
  static_assert(hvf::HVF_SPLIT_HEAD_WORDS + 4 * (size_t)HVF_NOALLOC_MAX_RAYS == NOALLOC_WORDS, "scratch size");
  // split_scratch_words(n, rounds) <= NOALLOC_WORDS for every n <= HVF_NOALLOC_MAX_RAYS.
  const uint32_t klog2 = (uint32_t)__builtin_ctz((unsigned)sc.split);
  return hvf::launch_trace_split(F, hvf::volume_family(v->spec, v->layout), d_rays, n, d_hits, (uint32_t)sc.split_budget, klog2,
                                 (uint32_t)sc.split_rounds, g_noalloc_ptr[dev], (hipStream_t)stream);
}

hvf_status hvf_autotune(hvf_volume* v, const hvf_ray* d_sample, size_t n, hvf_hit* d_hits, hvf_schedule* out,
                        void* stream) {
  if (!v || !d_sample || !d_hits || n == 0) return fail(HVF_E_INPUT, "autotune needs a volume and a non-empty sample");
  hipStream_t s = (hipStream_t)stream;
  std::vector<hvf_schedule> cand;
  cand.push_back(hvf_schedule{0, 16, 8, 0, 4, 0, 0, 0});
  const int nd = (int)v->layout.d.size();
  const bool own_layout = !v->spec.paper;  // short stacks and staged depths need it
  for (int sd : {2, 4})
    if (own_layout && sd < nd) cand.push_back(hvf_schedule{0, 16, 8, 0, 4, 0, sd, 0});
  for (int bpc : {0, 2, 4})
    for (int refill : {8, 32})
      for (int inner : {4, 16}) cand.push_back(hvf_schedule{1, refill, inner, 0, 4, bpc, 0, 0});
  for (int bits : {2, 4, 6}) cand.push_back(hvf_schedule{0, 16, 8, 1, bits, 0, 0, 0});
  // Split: K is an upper bound (the second launch cuts no more segments than its grid has
  // lanes), so K = 64 stands for every K the survivor count allows.
  const int split_cand[][3] = {{4, 64, 0}, {16, 64, 0}, {64, 32, 0}, {64, 64, 0}, {64, 128, 0}, {64, 48, 1}, {64, 64, 1}};
  for (const auto& c : split_cand) cand.push_back(hvf_schedule{0, 16, 8, 0, 4, 0, 0, 0, c[0], c[1], c[2]});
  // Stealing: (period, length in voxels, idle lanes).
  const int steal_cand[][3] = {{1, 2, 16}, {2, 2, 8}, {2, 8, 1}, {4, 8, 1}, {1, 8, 32}};
  for (int il : {0, 1}) {
    if (il) cand.push_back(hvf_schedule{0, 16, 8, 0, 4, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1});
    for (const auto& c : steal_cand)
      cand.push_back(hvf_schedule{0, 16, 8, 0, 4, 0, 0, 0, 0, 0, 0, c[0], c[1], c[2], il});
  }
  // Fewer rays per wave (interleaved, stealing): more waves for launches of few rays.
  for (int rpw : {32, 16}) cand.push_back(hvf_schedule{0, 16, 8, 0, 4, 0, 0, 0, 0, 0, 0, 1, 2, 16, 1, rpw});
  hvf_schedule best = cand[0];
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(HVF_E_DEVICE, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(HVF_E_DEVICE, "hipEventCreate failed");
  }
  hvf_status st = HVF_OK;
  // Mean time of `reps` launches of schedule c after one warm-up launch (uploads on first use).
  auto time_one = [&](const hvf_schedule& c, int reps) -> float {
    st = hvf_trace_sched(v, d_sample, n, d_hits, &c, stream);
    if (st != HVF_OK) return 0.0f;
    float tot = 0.0f;
    bool ok = hipEventRecord(e0, s) == hipSuccess;
    for (int r = 0; r < reps && st == HVF_OK; ++r) st = hvf_trace_sched(v, d_sample, n, d_hits, &c, stream);
    ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
         hipEventElapsedTime(&tot, e0, e1) == hipSuccess;
    if (st == HVF_OK && !ok) st = fail(HVF_E_DEVICE, "event timing failed during autotune");
    return tot / (float)reps;
  };
  // Round one: every candidate once. Round two: the default, the best three of round one
  // and the best one with the deepest LDS prefixes that fit, re-timed in interleaved
  // passes; the lowest median wins, and it replaces the default only when it is at least
  // 3% faster (timing noise must not pick a schedule).
  std::vector<std::pair<float, size_t>> r1;
  for (size_t i = 0; i < cand.size() && st == HVF_OK; ++i) r1.push_back({time_one(cand[i], 3), i});
  if (st == HVF_OK) {
    std::sort(r1.begin(), r1.end());
    std::vector<hvf_schedule> fin;
    fin.push_back(cand[0]);
    for (size_t k = 0; k < r1.size() && fin.size() < 4; ++k)
      if (r1[k].second != 0) fin.push_back(cand[r1[k].second]);
    const hvf_schedule top = cand[r1[0].second];
    uint32_t last = 0;
    int tried = 0;
    for (int k = nd; own_layout && k >= 1 && tried < 3; --k) {
      uint32_t w = 0;
      if (!hvf::lds_prefix_words(v->layout, v->built, k, &w) || w == 0 || w == last) continue;
      last = w;
      ++tried;
      hvf_schedule c = top;
      c.lds_depths = k;
      fin.push_back(c);
    }
    const int passes = 3;
    std::vector<std::vector<float>> t(fin.size());
    for (int pass = 0; pass < passes && st == HVF_OK; ++pass)
      for (size_t i = 0; i < fin.size() && st == HVF_OK; ++i) t[i].push_back(time_one(fin[i], 3));
    if (st == HVF_OK) {
      auto median = [](std::vector<float> x) {
        std::sort(x.begin(), x.end());
        return x[x.size() / 2];
      };
      size_t bi = 0;
      float bm = median(t[0]);
      const float base_ms = bm;
      for (size_t i = 1; i < fin.size(); ++i) {
        const float m = median(t[i]);
        if (m < bm) {
          bm = m;
          bi = i;
        }
      }
      if (bm > 0.97f * base_ms) bi = 0;
      best = fin[bi];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != HVF_OK) return st;
  v->sched = best;
  if (out) *out = best;
  return HVF_OK;
}

hvf_status hvf_trace(hvf_volume* v, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits, void* stream) {
  return hvf_trace_sched(v, d_rays, n, d_hits, nullptr, stream);
}

hvf_status hvf_get_schedule(const hvf_volume* v, hvf_schedule* out) {
  if (!v || !out) return fail(HVF_E_INPUT, "null argument");
  *out = v->sched;
  return HVF_OK;
}

hvf_status hvf_set_schedule(hvf_volume* v, const hvf_schedule* sched) {
  if (!v || !sched) return fail(HVF_E_INPUT, "null argument");
  hvf_status st = check_sched(*sched);
  if (st != HVF_OK) return st;
  v->sched = *sched;
  return HVF_OK;
}

hvf_status hvf_trace_count(hvf_volume* v, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits, uint32_t* d_log,
                           uint32_t cap, uint32_t* d_count, uint32_t* d_steps, void* stream) {
  if (!v) return fail(HVF_E_INPUT, "null volume");
  if (n == 0) return HVF_OK;
  if (!d_rays || !d_hits || !d_count || (cap && !d_log)) return fail(HVF_E_INPUT, "null buffer");
  hvf_status st = hvf_upload(v, stream);
  if (st != HVF_OK) return st;
  hvf::DevFormat F = hvf::make_devformat(v->layout, v->spec, v->dbuf);
  hvf::set_regions(F, v->built);
  if (v->built.regions && v->built.words.size() >= (1ull << 32))
    return fail(HVF_E_UNSUPPORTED, "the counting trace logs 32-bit word indices: buffers of 2^32 words or more are not counted");
  return hvf::launch_trace_count(F, v->spec.paper, d_rays, n, d_hits, d_log, cap, d_count, d_steps,
                                 (hipStream_t)stream);
}

hvf_status hvf_trace_host(hvf_volume* v, const hvf_ray* rays, size_t n, hvf_hit* hits) {
  if (!v) return fail(HVF_E_INPUT, "null volume");
  if (n == 0) return HVF_OK;
  if (!rays || !hits) return fail(HVF_E_INPUT, "null ray or hit array");
  hvf_ray* dr = nullptr;
  hvf_hit* dh = nullptr;
  hipError_t e = hipMalloc(&dr, n * sizeof(hvf_ray));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc rays");
  e = hipMalloc(&dh, n * sizeof(hvf_hit));
  if (e != hipSuccess) {
    (void)hipFree(dr);
    return hip_fail(e, "hipMalloc hits");
  }
  hvf_status st = HVF_OK;
  e = hipMemcpy(dr, rays, n * sizeof(hvf_ray), hipMemcpyHostToDevice);
  if (e != hipSuccess) st = hip_fail(e, "copy rays");
  if (st == HVF_OK) st = hvf_trace(v, dr, n, dh, nullptr);
  if (st == HVF_OK) {
    e = hipMemcpy(hits, dh, n * sizeof(hvf_hit), hipMemcpyDeviceToHost);
    if (e != hipSuccess) st = hip_fail(e, "copy hits");
  }
  (void)hipFree(dr);
  (void)hipFree(dh);
  return st;
}

}  // extern "C"

namespace hvf {
hvf_status host_words(const hvf_volume* v) {
  std::lock_guard<std::mutex> g(v->host_mu);
  if (!v->host_pending) return HVF_OK;
  hvf_volume* m = const_cast<hvf_volume*>(v);
  try {
    m->built.words.assign(v->pending_words, 0u);
  } catch (const std::bad_alloc&) {
    return fail(HVF_E_NOMEM, "host allocation failed");
  }
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  const bool other = e == hipSuccess && cur != v->device;
  if (other) e = hipSetDevice(v->device);
  if (e == hipSuccess)
    e = hipMemcpy(m->built.words.data(), v->dbuf, v->pending_words * sizeof(uint32_t), hipMemcpyDeviceToHost);
  if (other) (void)hipSetDevice(cur);
  if (e != hipSuccess) {
    m->built.words.clear();
    return hip_fail(e, "download of the word buffer");
  }
  m->host_pending = false;
  return HVF_OK;
}

size_t word_count(const hvf_volume* v) {
  std::lock_guard<std::mutex> g(v->host_mu);
  return v->host_pending ? v->pending_words : v->built.words.size();
}
}  // namespace hvf

extern "C" {

hvf_status hvf_info_get(const hvf_volume* v, hvf_info* out) {
  if (!v || !out) return fail(HVF_E_INPUT, "null argument");
  hvf_info I;
  std::memset(&I, 0, sizeof(I));
  I.num_levels = (int32_t)v->spec.lv.size();
  for (int k = 0; k < I.num_levels; ++k) {
    const int kind = v->spec.lv[k].kind;
    I.kinds[k] = kind == hvf::LK_RAW ? (v->spec.lv[k].maxd ? 'D' : 'R') : kind == hvf::LK_SVO ? 'S' : 'G';
    I.level_maxdist[k] = v->spec.lv[k].maxd;
    for (int a = 0; a < 3; ++a) I.level_exp[k][a] = v->spec.lv[k].e[a];
    I.level_nodes[k] = v->built.level_nodes.empty() ? 0 : v->built.level_nodes[k];
  }
  for (int a = 0; a < 3; ++a) I.extent_log2[a] = v->spec.ext[a];
  I.whole_level_dedup = v->spec.wld ? 1 : 0;
  I.num_depths = (int32_t)v->layout.d.size();
  I.num_words = hvf::word_count(v);
  for (size_t d = 0; d < v->layout.d.size() && d < HVF_MAX_DEPTH; ++d) {
    I.depth_nodes[d] = d < v->built.depth_nodes.size() ? v->built.depth_nodes[d] : 0;
    I.depth_offset[d] = d < v->built.depth_offset.size() ? v->built.depth_offset[d] : 0;
  }
  I.num_voxels = v->built.nvox;
  I.kernel_family = hvf::family_value(hvf::volume_family(v->spec, v->layout));
  I.depth_buffers = v->built.regions ? 1 : 0;
  I.paper_layout = v->spec.paper ? 1 : 0;
  *out = I;
  return HVF_OK;
}

hvf_status hvf_words(const hvf_volume* v, uint32_t* words, size_t cap, size_t* n_words) {
  if (!v || !n_words) return fail(HVF_E_INPUT, "null argument");
  if (words) {
    const hvf_status st = hvf::host_words(v);
    if (st != HVF_OK) return st;
  }
  const size_t n = hvf::word_count(v);
  if (words) std::memcpy(words, v->built.words.data(), (cap < n ? cap : n) * sizeof(uint32_t));
  *n_words = n;
  return HVF_OK;
}

namespace {
// Reads/writes that fold every byte into a running FNV-1a checksum.
struct HashedFile {
  FILE* f;
  uint64_t h = 1469598103934665603ull;
  bool ok = true;
  void put(const void* p, size_t n) {
    if (ok && n) ok = std::fwrite(p, 1, n, f) == n;
    h = fnv64(p, n, h);
  }
  void get(void* p, size_t n) {
    if (ok && n) ok = std::fread(p, 1, n, f) == n;
    if (ok) h = fnv64(p, n, h);
  }
};
}  // namespace

hvf_status hvf_save(const hvf_volume* v, const char* path) {
  if (!v || !path) return fail(HVF_E_INPUT, "null argument");
  const hvf_status hst = hvf::host_words(v);
  if (hst != HVF_OK) return hst;
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(HVF_E_INPUT, std::string("cannot open ") + path);
  const hvf::Built& B = v->built;
  const uint64_t slen = v->spec.text.size(), nw = B.words.size(), nd = B.depth_nodes.size(),
                 nl = B.level_nodes.size();
  HashedFile w{f};
  w.put(MAGIC, 8);
  w.put(&slen, 8);
  w.put(v->spec.text.data(), slen);
  w.put(&nw, 8);
  w.put(&B.nvox, 8);
  w.put(&nd, 8);
  w.put(&nl, 8);
  w.put(B.depth_nodes.data(), 8 * nd);
  w.put(B.depth_offset.data(), 8 * nd);
  w.put(B.depth_words.data(), 8 * nd);
  w.put(B.level_nodes.data(), 8 * nl);
  w.put(B.words.data(), 4 * nw);
  const uint64_t sum = w.h;
  bool ok = w.ok && std::fwrite(&sum, 8, 1, f) == 1;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? HVF_OK : fail(HVF_E_INPUT, std::string("write failed: ") + path);
}

hvf_status hvf_load(const char* path, hvf_volume** out) {
  if (!path || !out) return fail(HVF_E_INPUT, "null argument");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(HVF_E_INPUT, std::string("cannot open ") + path);
  char magic[8];
  uint64_t slen = 0, nw = 0, nd = 0, nl = 0, sum = 0;
  hvf_volume* v = new (std::nothrow) hvf_volume();
  HashedFile r{f};
  bool ok = v != nullptr;
  if (ok) {
    r.get(magic, 8);
    ok = r.ok && std::memcmp(magic, MAGIC, 8) == 0;
  }
  if (ok) {
    r.get(&slen, 8);
    ok = r.ok && slen < 4096;
  }
  std::string text(ok ? slen : 0, '\0');
  if (ok) {
    r.get(&text[0], slen);
    r.get(&nw, 8);
    r.get(&v->built.nvox, 8);
    r.get(&nd, 8);
    r.get(&nl, 8);
    ok = r.ok && nw >= 1 && nw < (1ull << 40) && nd <= HVF_MAX_DEPTH && nl <= HVF_MAX_LEVELS;
  }
  if (ok) {
    v->built.depth_nodes.resize(nd);
    v->built.depth_offset.resize(nd);
    v->built.depth_words.resize(nd);
    v->built.level_nodes.resize(nl);
    r.get(v->built.depth_nodes.data(), 8 * nd);
    r.get(v->built.depth_offset.data(), 8 * nd);
    r.get(v->built.depth_words.data(), 8 * nd);
    r.get(v->built.level_nodes.data(), 8 * nl);
    ok = r.ok;
  }
  if (ok) {
    try {
      v->built.words.resize(nw);
    } catch (const std::bad_alloc&) {
      ok = false;
    }
    if (ok) r.get(v->built.words.data(), 4 * nw);
    ok = ok && r.ok && std::fread(&sum, 8, 1, f) == 1 && sum == r.h;
  }
  std::fclose(f);
  std::string err;
  if (ok) {
    hvf_status st = hvf::parse_spec(text.c_str(), v->spec, err);
    ok = (st == HVF_OK);
    if (ok) {
      v->layout = v->spec.paper ? hvf::make_paper_layout(v->spec) : hvf::make_layout(v->spec);
      ok = v->layout.d.size() == nd && v->spec.lv.size() == nl && (nw < (1ull << 32) || v->spec.regions);
      v->built.regions = v->spec.regions;
      if (ok) ok = hvf::validate_words(v->layout, v->built, err);
    }
  }
  if (!ok) {
    delete v;
    return fail(HVF_E_INPUT, std::string("not a valid volume file: ") + path + (err.empty() ? "" : " (" + err + ")"));
  }
  *out = v;
  return HVF_OK;
}

void hvf_free(hvf_volume* v) {
  if (!v) return;
  if (v->dbuf || v->dcounters || v->split_buf) {
    int cur = 0;
    const bool other = hipGetDevice(&cur) == hipSuccess && v->device >= 0 && cur != v->device;
    if (other) (void)hipSetDevice(v->device);
    if (v->split_buf) (void)hipFreeAsync(v->split_buf, nullptr);  // after the calls that used it
    if (v->dbuf) (void)hipFree(v->dbuf);
    if (v->dcounters) (void)hipFree(v->dcounters);
    if (other) (void)hipSetDevice(cur);
  }
  delete v;
}

}  // extern "C"
