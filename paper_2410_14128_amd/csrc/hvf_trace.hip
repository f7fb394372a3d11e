// Ray traversal of hybrid voxel formats on gfx950 (one lane per ray, wave64).
//
// The paper's per-level intersection functions (Sec. 4.2: Raw levels by DDA, SVO and SVDAG
// levels by pre-order traversal with a per-thread stack, visiting non-empty hit children
// in order of hit time and handing each to the next level) are folded into one flat loop
// over "node depths". Every iteration a lane does exactly one of:
//   * test the child cell of its current node that holds the ray at time t;
//   * descend into it (push the node on the lane's stack, enter the child, refine the
//     cell position by comparing mid-plane crossing times with t);
//   * report the hit (last level, occupied voxel);
//   * advance to the next cell at the current scale (least far-plane time, all axes
//     crossing at that time step together) and pop every node the new cell left.
// Because the crossing time of a plane depends only on the plane coordinate, a coarse
// cell's visit interval is exactly the union of its children's, so this walk visits the
// same voxels, in the same order, as a flat DDA over the finest grid.
//
// Memory: the format is one uint32 buffer in HBM; per-depth tables live in scalar
// registers as 4-bit fields; the node stack is in LDS, one 8-byte slot per depth per lane.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "hvf_internal.h"

namespace hvf {
namespace {

constexpr int BLOCK = 256;
constexpr uint32_t MAX_ITERS = 1u << 22;  // guard; a correct walk needs far fewer

struct Lane {
  float o[3], inv[3];
  bool par[3], neg[3];
  int vo[3];
  float t0, t1;
};

__device__ __forceinline__ float fmax_fx(float a, float b) { return a < b ? b : a; }
__device__ __forceinline__ float fmin_fx(float a, float b) { return b < a ? b : a; }

// Crossing time of the integer plane p on axis a: two rounded fp32 ops, never fused.
__device__ __forceinline__ float plane_t(const Lane& L, int a, int p) { return ((float)p - L.o[a]) * L.inv[a]; }

// Ray setup and clip against [0, 2^ext) (the root volume). False on a miss.
__device__ __forceinline__ bool setup(const float4 r0, const float4 r1, const int32_t ext[3], Lane& L) {
  const float o[3] = {r0.x, r0.y, r0.z}, d[3] = {r1.x, r1.y, r1.z};
  bool ok = true, anyn = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ok = ok && isfinite(o[a]) && isfinite(d[a]);
    L.o[a] = o[a];
    L.inv[a] = 1.0f / d[a];
    L.par[a] = !isfinite(L.inv[a]);
    L.neg[a] = d[a] < 0.0f;
    L.vo[a] = 0;
    if (L.par[a]) {
      const bool in = (o[a] >= 0.0f) && (o[a] < (float)(1 << ext[a]));
      ok = ok && in;
      if (in) L.vo[a] = (int)floorf(o[a]);
    } else {
      anyn = true;
    }
  }
  if (!(ok && anyn)) return false;
  bool first = true;
  float tn = 0.0f, tf = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (L.par[a]) continue;
    const int N = 1 << ext[a];
    const float ne = plane_t(L, a, L.neg[a] ? N : 0);
    const float fa = plane_t(L, a, L.neg[a] ? 0 : N);
    tn = first ? ne : fmax_fx(tn, ne);
    tf = first ? fa : fmin_fx(tf, fa);
    first = false;
  }
  L.t0 = fmax_fx(r0.w, tn);
  L.t1 = fmin_fx(r1.w, tf);
  return L.t0 < L.t1;
}

// Narrow coordinate p (aligned to 2^hi) to the 2^lo-aligned cell that holds the ray at
// time t on axis a: one mid-plane comparison per bit.
__device__ __forceinline__ int refine(const Lane& L, int a, int p, int hi, int lo, float t) {
  for (int b = hi - 1; b >= lo; --b) {
    const int mid = p + (1 << b);
    bool up;
    if (L.par[a]) {
      up = L.vo[a] >= mid;
    } else {
      const float tm = plane_t(L, a, mid);
      up = L.neg[a] ? (t < tm) : (tm <= t);
    }
    p = up ? mid : p;
  }
  return p;
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ __forceinline__ uint32_t tab(uint64_t t, int d) { return (uint32_t)(t >> (4 * d)) & 15u; }

// Memory policies. Plain: just load. Counting: also log every word index a lane reads
// (the byte accounting of the roofline counts distinct words / 64-byte sectors per ray).
struct Plain {
  __device__ __forceinline__ void note(uint32_t, uint32_t) {}
};
struct Counting {
  uint32_t* log;  // this lane's log: cap entries
  uint32_t cap;
  uint32_t k = 0;
  __device__ __forceinline__ void note(uint32_t idx, uint32_t nwords) {
    for (uint32_t w = 0; w < nwords; ++w) {
      if (k < cap) log[k] = idx + w;
      ++k;
    }
  }
};

// Trace one lane's ray; writes the result to *out.
template <class Mem>
__device__ __forceinline__ void walk(const DevFormat& F, const Lane& L, uint2* stk, int4& out, Mem& mem) {
  const uint32_t* __restrict__ buf = F.buf;
  const uint32_t root = buf[0];  // word 0: pointer to the root sub-volume; 0 = empty
  mem.note(0, 1);
  if (root == 0) return;
  int p[3];
  const int cs0 = (int)tab(F.cs_tab, 0);
#pragma unroll
  for (int a = 0; a < 3; ++a) p[a] = refine(L, a, 0, F.ext[a], cs0, L.t0);
  int d = 0;
  uint32_t base = root, valid = 0xFFu;
  {
    const uint32_t hk = tab(F.hk_tab, 0);
    if (hk == HK_SVO) {
      const uint2 h = *reinterpret_cast<const uint2*>(buf + root);
      mem.note(root, 2);
      base = h.x;
      valid = h.y & 0xFFu;
    } else if (hk == HK_DAG) {
      valid = buf[root] & 0xFFu;
      mem.note(root, 1);
      base = root + 1;
    }
  }
  float t = L.t0;
  for (uint32_t it = 0; it < MAX_ITERS; ++it) {
    const uint32_t nk = tab(F.nk_tab, d);
    const int cs = (int)tab(F.cs_tab, d);
    bool occ;
    uint32_t child = 0;
    if (nk <= NK_RAW_BITS) {
      int wx, wy, wz;
      if (d == 0) {
        wx = F.top_w[0];
        wy = F.top_w[1];
        wz = F.top_w[2];
      } else {
        wx = wy = wz = (int)tab(F.w_tab, d);
      }
      const uint32_t cx = ((uint32_t)p[0] >> cs) & ((1u << wx) - 1u);
      const uint32_t cy = ((uint32_t)p[1] >> cs) & ((1u << wy) - 1u);
      const uint32_t cz = ((uint32_t)p[2] >> cs) & ((1u << wz) - 1u);
      if (nk == NK_RAW_PTR) {
        const uint32_t ix = base + (cx | (cy << wx) | (cz << (wx + wy)));
        child = buf[ix];
        mem.note(ix, 1);
        occ = child != 0u;
      } else {
        uint32_t word_ix, bit;
        if (F.bits_linear) {
          const uint64_t b64 = (uint64_t)cx | ((uint64_t)cy << wx) | ((uint64_t)cz << (wx + wy));
          word_ix = (uint32_t)(b64 >> 5);
          bit = (uint32_t)b64 & 31u;
        } else if (wx <= 10) {
          const uint32_t m = spread10(cx) | (spread10(cy) << 1) | (spread10(cz) << 2);
          word_ix = m >> 5;
          bit = m & 31u;
        } else {
          const uint64_t m = (uint64_t)(spread10(cx) | (spread10(cy) << 1) | (spread10(cz) << 2)) |
                             ((uint64_t)(spread10(cx >> 10) | (spread10(cy >> 10) << 1) | (spread10(cz >> 10) << 2)) << 30);
          word_ix = (uint32_t)(m >> 5);
          bit = (uint32_t)m & 31u;
        }
        occ = (buf[base + word_ix] >> bit) & 1u;
        mem.note(base + word_ix, 1);
      }
    } else {
      const uint32_t oct = (((uint32_t)p[0] >> cs) & 1u) | ((((uint32_t)p[1] >> cs) & 1u) << 1) |
                           ((((uint32_t)p[2] >> cs) & 1u) << 2);
      occ = (valid >> oct) & 1u;
      if (occ && nk != NK_OCT_FINAL) {
        const uint32_t rank = __popc(valid & ((1u << oct) - 1u));
        if (nk == NK_SVO_INNER) {
          child = base + 2u * rank;
        } else {
          child = buf[base + rank];
          mem.note(base + rank, 1);
        }
      }
    }
    if (occ) {
      if (nk == NK_RAW_BITS || nk == NK_OCT_FINAL) {
        // An occupied single voxel: report it if the ray really spends time in it.
        float e = L.t0, x = L.t1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          if (L.par[a]) continue;
          e = fmax_fx(e, plane_t(L, a, L.neg[a] ? p[a] + 1 : p[a]));
          x = fmin_fx(x, plane_t(L, a, L.neg[a] ? p[a] : p[a] + 1));
        }
        if (e < x) {
          out = make_int4(p[0], p[1], p[2], __float_as_int(e));
          return;
        }
      } else {
        stk[d * BLOCK] = make_uint2(base, valid);
        ++d;
        const uint32_t hk = tab(F.hk_tab, d);
        if (hk == HK_RAW) {
          base = child;
        } else if (hk == HK_SVO) {
          const uint2 h = *reinterpret_cast<const uint2*>(buf + child);
          mem.note(child, 2);
          base = h.x;
          valid = h.y & 0xFFu;
        } else {
          valid = buf[child] & 0xFFu;
          mem.note(child, 1);
          base = child + 1u;
        }
        const int ncs = (int)tab(F.cs_tab, d);
#pragma unroll
        for (int a = 0; a < 3; ++a) p[a] = refine(L, a, p[a], cs, ncs, t);
        continue;
      }
    }
    // Advance to the next cell of side 2^cs.
    const int step = 1 << cs;
    float tf[3];
    float m = 0.0f;
    bool first = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      tf[a] = 0.0f;
      if (L.par[a]) continue;
      tf[a] = plane_t(L, a, L.neg[a] ? p[a] : p[a] + step);
      m = first ? tf[a] : fmin_fx(m, tf[a]);
      first = false;
    }
    if (!(m < L.t1)) return;  // leaves the clipped ray interval: miss
    t = m;
    int diff = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (L.par[a] || tf[a] != m) continue;
      const int np = p[a] + (L.neg[a] ? -step : step);
      diff |= np ^ p[a];
      p[a] = np;
    }
    if (d > 0) {
      const int h = 31 - __clz(diff);
      int nd = d;
      while (nd > 0 && h >= (int)(tab(F.cs_tab, nd) + tab(F.w_tab, nd))) --nd;
      if (nd != d) {
        d = nd;
        const uint2 s = stk[d * BLOCK];
        base = s.x;
        valid = s.y;
        const int mask = ~((1 << (int)tab(F.cs_tab, d)) - 1);
        p[0] &= mask;
        p[1] &= mask;
        p[2] &= mask;
      }
    }
  }
  out = make_int4(-2, -2, -2, 0);  // iteration guard tripped: reported, never silent
}

__global__ __launch_bounds__(BLOCK) void trace_kernel(const DevFormat F, const float4* __restrict__ rays,
                                                      int4* __restrict__ hits, uint32_t n) {
  extern __shared__ uint2 stk_all[];
  const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  const float4 r0 = rays[2 * (size_t)i], r1 = rays[2 * (size_t)i + 1];
  int4 out = make_int4(-1, -1, -1, __float_as_int(INFINITY));
  Lane L;
  Plain mem;
  if (setup(r0, r1, F.ext, L)) walk(F, L, stk_all + threadIdx.x, out, mem);
  hits[i] = out;
}

// Same traversal, logging the word index of every format load: log[i * cap + k] for the
// first cap loads of ray i; count[i] = number of loads (may exceed cap).
__global__ __launch_bounds__(BLOCK) void trace_count_kernel(const DevFormat F, const float4* __restrict__ rays,
                                                            int4* __restrict__ hits, uint32_t n,
                                                            uint32_t* __restrict__ log, uint32_t cap,
                                                            uint32_t* __restrict__ count) {
  extern __shared__ uint2 stk_all[];
  const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  const float4 r0 = rays[2 * (size_t)i], r1 = rays[2 * (size_t)i + 1];
  int4 out = make_int4(-1, -1, -1, __float_as_int(INFINITY));
  Lane L;
  Counting mem{log + (size_t)i * cap, cap};
  if (setup(r0, r1, F.ext, L)) walk(F, L, stk_all + threadIdx.x, out, mem);
  hits[i] = out;
  count[i] = mem.k;
}

}  // namespace

hvf_status launch_trace(const DevFormat& F, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits, hipStream_t s) {
  if (n == 0) return HVF_OK;
  if (n >= (1ull << 32)) {
    hvf_set_error("at most 2^32 - 1 rays per call");
    return HVF_E_INPUT;
  }
  const unsigned grid = (unsigned)((n + BLOCK - 1) / BLOCK);
  const size_t lds = (size_t)F.ndepth * BLOCK * sizeof(uint2);
  hipLaunchKernelGGL(trace_kernel, dim3(grid), dim3(BLOCK), lds, s, F, reinterpret_cast<const float4*>(d_rays),
                     reinterpret_cast<int4*>(d_hits), (uint32_t)n);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    hvf_set_error(std::string("trace launch failed: ") + hipGetErrorString(e));
    return HVF_E_DEVICE;
  }
  return HVF_OK;
}

hvf_status launch_trace_count(const DevFormat& F, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits, uint32_t* d_log,
                              uint32_t cap, uint32_t* d_count, hipStream_t s) {
  if (n == 0) return HVF_OK;
  if (n >= (1ull << 32)) {
    hvf_set_error("at most 2^32 - 1 rays per call");
    return HVF_E_INPUT;
  }
  const unsigned grid = (unsigned)((n + BLOCK - 1) / BLOCK);
  const size_t lds = (size_t)F.ndepth * BLOCK * sizeof(uint2);
  hipLaunchKernelGGL(trace_count_kernel, dim3(grid), dim3(BLOCK), lds, s, F, reinterpret_cast<const float4*>(d_rays),
                     reinterpret_cast<int4*>(d_hits), (uint32_t)n, d_log, cap, d_count);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    hvf_set_error(std::string("counting trace launch failed: ") + hipGetErrorString(e));
    return HVF_E_DEVICE;
  }
  return HVF_OK;
}

}  // namespace hvf
