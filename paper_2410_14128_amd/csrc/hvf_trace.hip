// Ray traversal of hybrid voxel formats on gfx950 (one lane per ray, wave64).
//
// The paper's per-level intersection functions (Sec. 4.2: Raw levels by DDA, SVO and SVDAG
// levels by pre-order traversal with a per-thread stack, visiting non-empty hit children
// in order of hit time and handing each to the next level) are folded into one flat loop
// over "node depths". Every step a lane does exactly one of:
//   * test the child cell of its current node that holds the ray at time t;
//   * descend into it (push the node on the lane's stack, enter the child, narrow the
//     cell position by comparing mid-plane crossing times with t);
//   * report the hit (last level, occupied voxel);
//   * advance to the next cell at the current scale (least far-plane time, every axis
//     crossing at that time steps together) and pop every node the new cell left.
// Because the crossing time of a plane depends only on the plane coordinate, a coarse
// cell's visit interval is exactly the union of its children's, so this walk visits the
// same voxels, in the same order, as a flat DDA over the finest grid.
//
// Memory: the format is one uint32 buffer in HBM; a per-depth descriptor table and the
// node stack (one 8-byte slot per depth per lane) live in LDS; the current depth's
// descriptor, node header and, inside a brick, the 64-bit block mask live in registers.
//
// Kernels: trace_kernel (one ray per lane), trace_persistent_kernel (a fixed grid whose
// waves refill idle lanes from a global ray counter when a ballot shows enough idle
// lanes), trace_count_kernel (trace_kernel plus a log of every format word read).
#include <hip/hip_runtime.h>

#include <cmath>
#include <hipcub/hipcub.hpp>
#include <mutex>
#include <string>

#include "hvf_internal.h"

namespace hvf {
namespace {

constexpr int BLOCK = 256;
constexpr uint32_t MAX_STEPS = 1u << 22;  // guard; a correct walk needs far fewer

__device__ __forceinline__ float fmax_fx(float a, float b) { return a < b ? b : a; }
__device__ __forceinline__ float fmin_fx(float a, float b) { return b < a ? b : a; }

__device__ __forceinline__ uint32_t bf(uint32_t v, uint32_t off, uint32_t w) {
  return __builtin_amdgcn_ubfe(v, off, w);
}
__device__ __forceinline__ uint32_t di_nk(uint32_t i) { return i & 15u; }
__device__ __forceinline__ uint32_t di_hk(uint32_t i) { return bf(i, 4, 4); }
__device__ __forceinline__ int di_cs(uint32_t i) { return (int)bf(i, 8, 4); }
__device__ __forceinline__ int di_w(uint32_t i, int a) { return (int)bf(i, 12 + 4 * a, 4); }

// After setup, an axis the ray is parallel to (1/d_a not finite) carries o_a = floor(o_a)
// + 0.5 and 1/d_a = +inf, and its sign bit is clear. Its plane time (p - o_a) * inf is
// then -inf for every plane p <= floor(o_a) and +inf for every plane above (never NaN: p
// is an integer, o_a is not), so the generic tests below need no parallel-axis case: a
// mid-plane test "T(mid) <= t" says whether floor(o_a) lies in the upper half, and a far
// plane is never crossed.
struct Ray {
  float o[3], inv[3];
  uint32_t neg, par;  // bit a set: d_a < 0 (clear on parallel axes) / axis a parallel
  float t0, t1;
  __device__ __forceinline__ bool is_par(int a) const { return (par >> a) & 1u; }
  __device__ __forceinline__ bool is_neg(int a) const { return (neg >> a) & 1u; }
  // Crossing time of the integer plane p on axis a: two rounded fp32 ops, never fused.
  __device__ __forceinline__ float T(int a, int p) const { return ((float)p - o[a]) * inv[a]; }
};

// Ray setup and clip against [0, 2^ext) (the root volume). False on a miss.
__device__ __forceinline__ bool setup(const float4 r0, const float4 r1, const int32_t ext[3], Ray& R) {
  const float o[3] = {r0.x, r0.y, r0.z}, d[3] = {r1.x, r1.y, r1.z};
  bool ok = true;
  R.neg = R.par = 0;
  float po[3];  // o_a as a parallel axis carries it after the clip
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ok = ok && isfinite(o[a]) && isfinite(d[a]);
    R.o[a] = o[a];
    R.inv[a] = 1.0f / d[a];
    const bool par = !isfinite(R.inv[a]);
    R.par |= (uint32_t)par << a;
    R.neg |= (uint32_t)(d[a] < 0.0f) << a;
    po[a] = 0.5f;
    if (par) {
      const bool in = (o[a] >= 0.0f) && (o[a] < (float)(1 << ext[a]));
      ok = ok && in;
      if (in) po[a] = floorf(o[a]) + 0.5f;  // exact: floor(o_a) < 2^21
    }
  }
  if (!ok || R.par == 7u) return false;
  bool first = true;
  float tn = 0.0f, tf = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (R.is_par(a)) continue;
    const int N = 1 << ext[a];
    const float ne = R.T(a, R.is_neg(a) ? N : 0);
    const float fa = R.T(a, R.is_neg(a) ? 0 : N);
    tn = first ? ne : fmax_fx(tn, ne);
    tf = first ? fa : fmin_fx(tf, fa);
    first = false;
  }
  R.t0 = fmax_fx(r0.w, tn);
  R.t1 = fmin_fx(r1.w, tf);
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (R.is_par(a)) {
      R.o[a] = po[a];
      R.inv[a] = INFINITY;
    }
  R.neg &= ~R.par;
  return R.t0 < R.t1;
}

// Narrow the cell position p (aligned to 2^hi on every axis) to the 2^lo-aligned cell
// that holds the ray at time t: one mid-plane comparison per bit and axis. For d > 0 the
// upper half holds the ray iff T(mid) <= t; for d < 0 iff t < T(mid); on a parallel axis
// the same test compares floor(o) with mid (see Ray). No per-lane branch is taken.
__device__ __forceinline__ void refine3(const Ray& R, int p[3], int hi, int lo, float t) {
  for (int b = hi - 1; b >= lo; --b) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int mid = p[a] + (1 << b);
      const bool up = (R.T(a, mid) <= t) != R.is_neg(a);
      p[a] = up ? mid : p[a];
    }
  }
}

// Memory policies. Plain: just load. Counting: also log every word index a lane reads
// (the byte accounting of the roofline counts distinct words / 64-byte sectors per ray).
struct Plain {
  __device__ __forceinline__ void note(uint32_t, uint32_t) {}
};
struct Counting {
  uint32_t* log;  // this lane's log: cap entries
  uint32_t cap;
  uint32_t k;
  __device__ __forceinline__ void note(uint32_t idx, uint32_t nwords) {
    for (uint32_t w = 0; w < nwords; ++w) {
      if (k < cap) log[k] = idx + w;
      ++k;
    }
  }
};

// Format words are read through explicitly global pointers (and the staged prefix through
// explicitly LDS ones), so the compiler emits global_load / ds_read and never merges the
// two into a generic (flat) access.
typedef const __attribute__((address_space(1))) uint32_t gword;
typedef const __attribute__((address_space(3))) uint32_t lword;
__device__ __forceinline__ gword* as_global(const uint32_t* p) { return (gword*)p; }
__device__ __forceinline__ lword* as_lds(const uint32_t* p) { return (lword*)p; }
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <class I>
__device__ __forceinline__ uint2 ld2(gword* buf, I ix) {
  const u32x2 v = *reinterpret_cast<const __attribute__((address_space(1))) u32x2*>(buf + ix);
  return make_uint2(v.x, v.y);
}
template <class I>
__device__ __forceinline__ uint4 ld4(gword* buf, I ix) {
  const u32x4 v = *reinterpret_cast<const __attribute__((address_space(1))) u32x4*>(buf + ix);
  return make_uint4(v.x, v.y, v.z, v.w);
}

enum : int { RUN = 0, DONE = 1 };

// Template flag of the trace kernels: the top depths are staged in LDS.
constexpr uint32_t FAM_PRE = 1u << 31;

// The format a lane walks: word buffer, pop table, per-axis extents and the per-depth
// descriptor table (in LDS). Uniform across a launch for single-volume kernels; per lane
// in the batched kernel. The first npre words of the buffer (the top depths: nodes are
// stored depth by depth) may be staged in LDS at pre; reads below npre go there.
struct Fmt {
  gword* buf;
  uint64_t pop_lut;
  const uint32_t* dtab;
  const uint64_t* rtab;  // per-depth region starts (buffers with per-depth regions), or null
  int ext[3];
  uint32_t stacked;  // depths with a node-stack slot
  lword* pre;
  uint32_t npre;
  // Kernels are compiled twice, with and without a staged prefix (FAM_PRE), so reads in
  // the common unstaged case carry no per-lane test.
  // ix: a word index, 32-bit, or 64-bit in buffers with per-depth regions.
  // Start of depth d's region; 0 where a batch item without regions leaves the table null.
  __device__ __forceinline__ uint64_t region(int d) const { return rtab ? rtab[d] : 0ull; }
  template <uint32_t FAM, class I>
  __device__ __forceinline__ uint32_t w1(I ix) const {
    if ((FAM & FAM_PRE) && ix < npre) return pre[ix];
    return buf[ix];
  }
  template <uint32_t FAM, class I>
  __device__ __forceinline__ uint2 w2(I ix) const {
    if ((FAM & FAM_PRE) && ix + 2u <= npre) return make_uint2(pre[ix], pre[ix + 1u]);
    return ld2(buf, ix);
  }
  template <uint32_t FAM, class I>
  __device__ __forceinline__ uint4 w4(I ix) const {
    if ((FAM & FAM_PRE) && ix + 4u <= npre) return make_uint4(pre[ix], pre[ix + 1u], pre[ix + 2u], pre[ix + 3u]);
    return ld4(buf, ix);
  }
};

// LDS words of the per-depth tables: descriptors, then the 64-bit region starts.
constexpr int DTAB_WORDS = 3 * HVF_MAX_DEPTH;

// Index of a word of the current depth: rb + ix in buffers with per-depth regions (rb, the
// start of the depth's region), else ix.
template <uint32_t FAM>
__device__ __forceinline__ auto gx(uint32_t ix, uint64_t rb) {
  if constexpr ((FAM & FAM_REGIONS) != 0u)
    return rb + (uint64_t)ix;
  else
    return ix;
}

// Every depth stacked (the default): the slot of depth d is d.
constexpr uint32_t ALL_STACKED = 0xFFFFFFFFu;

// Stack slot of depth d: the number of stacked depths above it.
__device__ __forceinline__ uint32_t slot_of(uint32_t stacked, int d) { return __popc(stacked & ((1u << d) - 1u)); }

__device__ __forceinline__ Fmt fmt_of(const DevFormat& F, const uint32_t* dtab, const uint32_t* pre) {
  Fmt f;
  f.pre = as_lds(pre);
  f.npre = pre ? F.lds_words : 0u;
  f.buf = as_global(F.buf);
  f.pop_lut = F.pop_lut;
  f.dtab = dtab;
  f.rtab = reinterpret_cast<const uint64_t*>(dtab + HVF_MAX_DEPTH);
  f.ext[0] = F.ext[0];
  f.ext[1] = F.ext[1];
  f.ext[2] = F.ext[2];
  f.stacked = F.stacked;
  return f;
}

// The per-lane walk state.
struct Walk {
  Ray R;
  float t;
  int p[3];
  int d;
  uint32_t info;  // descriptor of depth d
  uint32_t base, valid;
  uint32_t steps;
  uint64_t rb;  // start of depth d's region (buffers with per-depth regions; else unused)
  // Distance-field skipping at the current depth: every cell whose L1 distance (in cells
  // of this depth) from the anchor cell a[] is below reach is known to be empty. The
  // anchor is the last empty cell read; any change of depth clears reach. Along a ray
  // each axis coordinate moves monotonically away from the anchor, so once a cell is
  // outside that ball every later cell is too.
  int a[3];
  uint32_t reach;

  // Enter the node at pointer ptr whose depth descriptor is nd: returns its header
  // (base, valid). m: the 64-bit block mask the parent's test read (used by HK_MASK).
  template <uint32_t FAM, class Mem>
  __device__ __forceinline__ static uint2 enter(const Fmt& F, uint32_t nd, uint32_t ptr, uint2 m, uint64_t rb,
                                                Mem& mem) {
    const uint32_t hk = di_hk(nd);
    constexpr uint32_t LOADS = fam_hk(HK_DAG) | fam_hk(HK_SVO) | fam_hk(HK_MASKLOAD);
    // One 8-byte load serves every header kind read at the pointer: an SVDAG node's mask
    // word (the node also holds at least one child word, so the load stays inside it), an
    // SVO node's two words, a one-block brick's mask.
    uint2 h = make_uint2(0u, 0u);
    constexpr uint32_t LOAD_KINDS = (1u << HK_DAG) | (1u << HK_SVO) | (1u << HK_MASKLOAD);
    if ((FAM & LOADS) && ((LOAD_KINDS >> hk) & 1u)) {
      h = F.template w2<FAM>(gx<FAM>(ptr, rb));
      mem.note((uint32_t)gx<FAM>(ptr, rb), hk == HK_DAG ? 1u : 2u);
    }
    uint32_t b = h.x, v = h.y;  // HK_MASKLOAD
    if (FAM & fam_hk(HK_SVO)) v = (hk == HK_SVO) ? (h.y & 0xFFu) : v;
    if (FAM & fam_hk(HK_DAG)) {
      b = (hk == HK_DAG) ? ptr + 1u : b;
      v = (hk == HK_DAG) ? (h.x & 0xFFu) : v;
    }
    if (FAM & fam_hk(HK_MASK)) {
      b = (hk == HK_MASK) ? m.x : b;
      v = (hk == HK_MASK) ? m.y : v;
    }
    if (FAM & fam_hk(HK_RAW)) {
      b = (hk == HK_RAW) ? ptr : b;
      v = (hk == HK_RAW) ? 0u : v;
    }
    return make_uint2(b, v);
  }

  // Pointer (and, for SVDAG descriptors, the child's header) of the occupied child `lin`
  // of an octree node with header (base, valid).
  template <uint32_t FAM, class Mem>
  __device__ __forceinline__ static void octree_child(const Fmt& F, uint32_t nk, uint32_t lin,
                                                      uint32_t base, uint32_t valid, uint32_t& child, uint2& cm,
                                                      uint64_t rb, Mem& mem) {
    const uint32_t rank = __popc(valid & ((1u << lin) - 1u));
    if ((FAM & fam_nk(NK_SVO_INNER)) && nk == NK_SVO_INNER) {
      child = base + 2u * rank;
    } else if ((FAM & fam_nk(NK_DAG_INNER)) && nk == NK_DAG_INNER) {
      const uint2 dsc = F.template w2<FAM>(gx<FAM>(base + 2u * rank, rb));  // (child pointer, child masks)
      mem.note((uint32_t)gx<FAM>(base + 2u * rank, rb), 2);
      child = dsc.x;
      cm = make_uint2(dsc.x + 1u, dsc.y & 0xFFu);
    } else {
      child = F.template w1<FAM>(gx<FAM>(base + rank, rb));
      mem.note((uint32_t)gx<FAM>(base + rank, rb), 1);
    }
  }

  // Far-plane crossing times of the current cell (side 2^cs) per axis (+inf on parallel
  // axes) and their minimum.
  __device__ __forceinline__ void far_times(int cs, float tf[3], float& m) const {
    const int stepv = 1 << cs;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      tf[a] = R.T(a, R.is_neg(a) ? p[a] : p[a] + stepv);  // +inf on a parallel axis
    }
    m = fmin_fx(fmin_fx(tf[0], tf[1]), tf[2]);
  }

  // Index of the child cell holding the ray: the cell position's bits [c, c + w_a) per axis,
  // x lowest. Octree-only families have w = 1 at every depth and cubic families one w for
  // all three axes, known at compile time or read once.
  template <uint32_t FAM>
  __device__ __forceinline__ uint32_t cell_lin(uint32_t in) const {
    const int c = di_cs(in);
    constexpr uint32_t F0 = FAM & ~FAM_PRE;
    if (fam_w1(F0)) return bf((uint32_t)p[0], c, 1) | (bf((uint32_t)p[1], c, 1) << 1) | (bf((uint32_t)p[2], c, 1) << 2);
    if (fam_cubic(F0)) {
      const uint32_t w = bf(in, 12, 4);
      return bf((uint32_t)p[0], c, w) | (bf((uint32_t)p[1], c, w) << w) | (bf((uint32_t)p[2], c, w) << (2 * w));
    }
    const uint32_t wx = bf(in, 12, 4), wy = bf(in, 16, 4), wz = bf(in, 20, 4);
    return bf((uint32_t)p[0], c, wx) | (bf((uint32_t)p[1], c, wy) << wx) | (bf((uint32_t)p[2], c, wz) << (wx + wy));
  }

  // Start the walk of a ray that passed setup. Returns DONE if the volume is empty.
  template <uint32_t FAM, class Mem>
  __device__ __forceinline__ int start(const Fmt& F, Mem& mem) {
    const uint32_t* dtab = F.dtab;
    const uint32_t root = F.template w1<FAM>(0u);  // word 0: pointer to the root sub-volume; 0 = empty
    mem.note(0, 1);
    if (root == 0u) return DONE;
    d = 0;
    info = dtab[0];
    rb = (FAM & FAM_REGIONS) ? F.region(0) : 0ull;
    const int cs = di_cs(info);
#pragma unroll
    for (int a = 0; a < 3; ++a) p[a] = 0;
    // The root node may be non-cubic: narrow each axis from its own extent.
    for (int b = max(F.ext[0], max(F.ext[1], F.ext[2])) - 1; b >= cs; --b) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (b >= F.ext[a]) continue;
        const int mid = p[a] + (1 << b);
        const bool up = (R.T(a, mid) <= R.t0) != R.is_neg(a);
        p[a] = up ? mid : p[a];
      }
    }
    const uint2 h = enter<FAM>(F, info, root, make_uint2(0u, 0u), rb, mem);
    base = h.x;
    valid = h.y;
    t = R.t0;
    steps = 0;
    reach = 0;
    return RUN;
  }

  // One step. On DONE, out holds the result (a miss leaves it untouched). GUARD: count this
  // walk's steps against MAX_STEPS (callers that pass false keep a guard of their own).
  template <uint32_t FAM, bool GUARD = true, class Mem>
  __device__ __forceinline__ int step(const Fmt& F, uint2* stk, int4& out, Mem& mem) {
    const uint32_t* dtab = F.dtab;
    if (GUARD && ++steps > MAX_STEPS) {
      out = make_int4(-2, -2, -2, 0);  // guard tripped: reported, never silent
      return DONE;
    }
    const uint32_t nk = di_nk(info);
    const int cs = di_cs(info);
    // Child cell of the current node holding the ray (octree nodes: w = 1, the octant).
    const uint32_t lin = cell_lin<FAM>(info);
    // Register test: a voxel's bit in the block mask (base:valid) or an octree child's valid bit.
    const uint32_t word = ((FAM & fam_nk(NK_CELLS)) && nk == NK_CELLS && lin < 32u) ? base : valid;
    bool occ = ((word >> (lin & 31u)) & 1u) != 0u;
    uint32_t child = 0u;
    uint2 cm = make_uint2(0u, 0u);
    float tf[3], m;
    constexpr uint32_t OCT = fam_nk(NK_SVO_INNER) | fam_nk(NK_OCT_PTR) | fam_nk(NK_DAG_INNER) | fam_nk(NK_OCT_FINAL) |
                             fam_nk(NK_PSVO_TERM) | fam_nk(NK_PDAG_TERM);
    const bool dfk = ((FAM & fam_nk(NK_DF_PTR)) && nk == NK_DF_PTR) || ((FAM & fam_nk(NK_DF_BLOCKS)) && nk == NK_DF_BLOCKS) ||
                     ((FAM & fam_nk(NK_PDF_PTR)) && nk == NK_PDF_PTR) || ((FAM & fam_nk(NK_PDF_VOX)) && nk == NK_PDF_VOX);
    const uint32_t rank = (FAM & OCT) ? (uint32_t)__popc(valid & ((1u << lin) - 1u)) : 0u;
    if (dfk) {
      // Cell positions at this depth are multiples of 2^cs, so the shift is exact.
      const uint32_t l1 = (uint32_t)(abs(p[0] - a[0]) + abs(p[1] - a[1]) + abs(p[2] - a[2])) >> cs;
      occ = false;
      if (l1 >= reach) {  // not known to be empty: read the cell
        uint32_t dist;
        if ((FAM & fam_nk(NK_DF_PTR)) && nk == NK_DF_PTR) {
          child = F.template w1<FAM>(gx<FAM>(base + lin, rb));
          mem.note((uint32_t)gx<FAM>(base + lin, rb), 1);
          occ = (child & DF_EMPTY) == 0u;
          dist = child & ~DF_EMPTY;
        } else if ((FAM & (fam_nk(NK_PDF_PTR) | fam_nk(NK_PDF_VOX))) && (nk == NK_PDF_PTR || nk == NK_PDF_VOX)) {
          const uint2 q = F.template w2<FAM>(gx<FAM>(base + 2u * lin, rb));  // (terminating integer, distance)
          mem.note((uint32_t)gx<FAM>(base + 2u * lin, rb), 2);
          child = q.x;
          occ = q.x != 0u;
          dist = q.y;
        } else {
          const uint4 q = F.template w4<FAM>(gx<FAM>(base + 4u * lin, rb));
          mem.note((uint32_t)gx<FAM>(base + 4u * lin, rb), 4);
          cm = make_uint2(q.x, q.y);
          occ = (q.x | q.y) != 0u;
          dist = q.z;
        }
        if (!occ) {
          reach = dist;
          a[0] = p[0];
          a[1] = p[1];
          a[2] = p[2];
        }
      }
    } else {
      // One 8-byte read serves every kind whose test or descent reads memory: a pointer-grid
      // cell, a block mask, or the occupied octree child's pointer or (pointer, masks)
      // descriptor. The device buffer ends with spare zero words, so a read that starts at
      // its last word stays inside the allocation.
      // Each kind is tested only in families that compile it in, so the families of the
      // library's own layout carry no test for the paper layout's kinds.
      const bool rawk = ((FAM & fam_nk(NK_RAW_PTR)) && nk == NK_RAW_PTR) ||
                        ((FAM & fam_nk(NK_PRAW_VOX)) && nk == NK_PRAW_VOX);
      const bool blk = (FAM & fam_nk(NK_BLOCKS)) && nk == NK_BLOCKS;
      const bool optr = ((FAM & fam_nk(NK_OCT_PTR)) && nk == NK_OCT_PTR) ||
                        ((FAM & fam_nk(NK_PDAG_TERM)) && nk == NK_PDAG_TERM);
      const bool dagi = ((FAM & fam_nk(NK_DAG_INNER)) && nk == NK_DAG_INNER) ||
                        ((FAM & fam_nk(NK_PSVO_TERM)) && nk == NK_PSVO_TERM);
      const uint32_t idx = rawk ? lin : (blk ? 2u * lin : (dagi ? 2u * rank : rank));
      uint2 q = make_uint2(0u, 0u);
      if (rawk || blk || ((optr || dagi) && occ)) {
        q = F.template w2<FAM>(gx<FAM>(base + idx, rb));
        mem.note((uint32_t)gx<FAM>(base + idx, rb), (blk || (FAM & fam_nk(NK_DAG_INNER) && nk == NK_DAG_INNER)) ? 2u : 1u);
      }
      child = q.x;
      cm = blk ? q : make_uint2(q.x + 1u, q.y & 0xFFu);
      if (rawk) occ = child != 0u;
      if (blk) occ = (cm.x | cm.y) != 0u;
      if ((FAM & fam_nk(NK_SVO_INNER)) && nk == NK_SVO_INNER) child = base + 2u * rank;
      if ((FAM & fam_nk(NK_PDAG_TERM)) && nk == NK_PDAG_TERM && occ) {  // the leaf word holds the pointer
        child = F.template w1<FAM>(gx<FAM>(child, rb));
        mem.note((uint32_t)gx<FAM>(q.x, rb), 1);
      }
    }
    const bool fin = ((FAM & fam_nk(NK_CELLS)) && nk == NK_CELLS) || ((FAM & fam_nk(NK_OCT_FINAL)) && nk == NK_OCT_FINAL) ||
                     ((FAM & fam_nk(NK_PRAW_VOX)) && nk == NK_PRAW_VOX) || ((FAM & fam_nk(NK_PDF_VOX)) && nk == NK_PDF_VOX);
    const bool desc = occ && !fin;
    // One set of plane times serves both ends of the step: a descent's first mid-plane test
    // (planes p + 2^(cs-1)) and an advance's far planes (p + 2^cs on axes the ray walks up,
    // p on the others).
    const int stepv = 1 << cs, half = stepv >> 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) tf[a] = R.T(a, p[a] + (desc ? half : (R.is_neg(a) ? 0 : stepv)));
    if (desc) {
      if (F.stacked == ALL_STACKED)  // uniform: every depth has a slot, slot = depth
        stk[d * BLOCK] = make_uint2(base, valid);
      else if ((F.stacked >> d) & 1u)
        stk[slot_of(F.stacked, d) * BLOCK] = make_uint2(base, valid);
      ++d;
      reach = 0;
      info = dtab[d];
      if (FAM & FAM_REGIONS) rb = F.region(d);
      const uint2 h = enter<FAM>(F, info, child, cm, rb, mem);
      base = h.x;
      valid = h.y;
      // The child cell holding the ray at t: the first bit from the mid-plane times above,
      // the rest (descents of more than one bit per axis) by refine3.
#pragma unroll
      for (int a = 0; a < 3; ++a) p[a] += ((tf[a] <= t) != R.is_neg(a)) ? half : 0;
      refine3(R, p, cs - 1, di_cs(info), t);
      return RUN;
    }
    m = fmin_fx(fmin_fx(tf[0], tf[1]), tf[2]);
    // An occupied single voxel. The walk's t is always the entry time of its current cell:
    // the root cell is entered at t0, an advance enters the next cell at the crossing time
    // of the plane between them, and a descent picks the child holding the ray at t, whose
    // near planes are crossed no later than t. So the voxel's visit interval is
    // [t, min(t1, m)) and t < t1 always holds: it is visited iff t < m, and its entry
    // time is t itself.
    // One exit test for both ends of a walk: the hit, or leaving the clipped ray interval
    // (a miss, which leaves out untouched).
    const bool hit = occ && t < m;
    if (hit) out = make_int4(p[0], p[1], p[2], __float_as_int(t));
    if (hit || !(m < R.t1)) return DONE;
    t = m;
    uint32_t dd = 0u;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int np = p[a] + (R.is_neg(a) ? -stepv : stepv);
      const bool mv = (tf[a] == m);
      dd |= mv ? (uint32_t)(np ^ p[a]) : 0u;
      p[a] = mv ? np : p[a];
    }
    // Pop to the deepest node that still contains the new cell (the root always does; at
    // depth 0 the min keeps nd = 0). Some axis always steps, so dd != 0.
    const int hb = 31 - __clz(dd);
    const int nd = min(d, (int)((F.pop_lut >> (4 * hb)) & 15u));
    if (nd != d) pop_to<FAM>(F, stk, nd, mem);
    return RUN;
  }

  // Exit time of the ancestor node at depth k (1 <= k <= d) of the current cell: the least
  // far-plane time of that node's cell, of side 2^cs(k - 1). Also the walk's position just
  // after leaving it (q: that cell advanced along every axis crossing at the exit time, as
  // an advance does) and the depth nd < k of the deepest node holding the new cell (from
  // the pop table). Only meaningful when the exit time is below t1 (the new cell is then
  // inside the root).
  __device__ __forceinline__ float node_exit(const Fmt& F, int k, int q[3], int& nd) const {
    const int cs = di_cs(F.dtab[k - 1]);
    const int side = 1 << cs, mask = ~(side - 1);
    float tf[3];
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      c[a] = p[a] & mask;
      tf[a] = R.T(a, R.is_neg(a) ? c[a] : c[a] + side);
    }
    const float m = fmin_fx(fmin_fx(tf[0], tf[1]), tf[2]);
    uint32_t dd = 0u;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int np = c[a] + (R.is_neg(a) ? -side : side);
      const bool mv = (tf[a] == m);
      dd |= mv ? (uint32_t)(np ^ c[a]) : 0u;
      q[a] = mv ? np : c[a];
    }
    const int hb = 31 - __clz(dd);
    nd = min(k - 1, (int)((F.pop_lut >> (4 * hb)) & 15u));
    return m;
  }

  // Leave the current node for its ancestor at depth nd < d that contains the new cell:
  // restore the deepest stacked ancestor r <= nd, then descend again along p (every
  // ancestor of the current cell exists, so each child on the way is occupied).
  template <uint32_t FAM, class Mem>
  __device__ __forceinline__ void pop_to(const Fmt& F, uint2* stk, int nd, Mem& mem) {
    const uint32_t* dtab = F.dtab;
    if (F.stacked == ALL_STACKED) {  // uniform: the ancestor's own slot holds it
      const uint2 sv = stk[nd * BLOCK];
      base = sv.x;
      valid = sv.y;
      info = dtab[nd];
      if (FAM & FAM_REGIONS) rb = F.region(nd);
      d = nd;
      reach = 0;
      const int mask = ~((1 << di_cs(info)) - 1);
      p[0] &= mask;
      p[1] &= mask;
      p[2] &= mask;
      return;
    }
    const int r = 31 - __clz(F.stacked & ((2u << nd) - 1u));
    const uint2 sv = stk[slot_of(F.stacked, r) * BLOCK];
    base = sv.x;
    valid = sv.y;
    info = dtab[r];
    if (FAM & FAM_REGIONS) rb = F.region(r);
    for (int k = r; k < nd; ++k) {
      const uint32_t knk = di_nk(info), kl = cell_lin<FAM>(info);
      uint32_t child = 0u;
      uint2 cm = make_uint2(0u, 0u);
      if (((FAM & fam_nk(NK_RAW_PTR)) && knk == NK_RAW_PTR) || ((FAM & fam_nk(NK_DF_PTR)) && knk == NK_DF_PTR)) {
        child = F.template w1<FAM>(gx<FAM>(base + kl, rb));  // an ancestor cell: non-empty, so a plain pointer
        mem.note((uint32_t)gx<FAM>(base + kl, rb), 1);
      } else if ((FAM & fam_nk(NK_BLOCKS)) && knk == NK_BLOCKS) {
        cm = F.template w2<FAM>(gx<FAM>(base + 2u * kl, rb));
        mem.note((uint32_t)gx<FAM>(base + 2u * kl, rb), 2);
      } else if ((FAM & fam_nk(NK_DF_BLOCKS)) && knk == NK_DF_BLOCKS) {
        cm = F.template w2<FAM>(gx<FAM>(base + 4u * kl, rb));
        mem.note((uint32_t)gx<FAM>(base + 4u * kl, rb), 2);
      } else {
        octree_child<FAM>(F, knk, kl, base, valid, child, cm, rb, mem);
      }
      info = dtab[k + 1];
      if (FAM & FAM_REGIONS) rb = F.region(k + 1);
      const uint2 h = enter<FAM>(F, info, child, cm, rb, mem);
      base = h.x;
      valid = h.y;
    }
    d = nd;
    reach = 0;
    const int mask = ~((1 << di_cs(info)) - 1);
    p[0] &= mask;
    p[1] &= mask;
    p[2] &= mask;
  }
};

// Copy the first F.lds_words words of the buffer (a multiple of 4; the top depths) into
// LDS right after the node stack; returns that LDS copy, or null when nothing is staged.
// Must precede load_dtab, whose barrier publishes the copy.
__device__ __forceinline__ const uint32_t* stage_prefix(const DevFormat& F, uint2* stk_all) {
  if (F.lds_words == 0u) return nullptr;
  uint32_t* pre = reinterpret_cast<uint32_t*>(stk_all + (size_t)(F.nslots ? F.nslots : 1u) * BLOCK);
  const uint4* src = reinterpret_cast<const uint4*>(F.buf);
  uint4* dst = reinterpret_cast<uint4*>(pre);
  for (uint32_t i = threadIdx.x; i < F.lds_words / 4u; i += BLOCK) dst[i] = src[i];
  return pre;
}

__device__ __forceinline__ void load_dtab(const DevFormat& F, uint32_t* dtab) {
  if (threadIdx.x < HVF_MAX_DEPTH) {
    dtab[threadIdx.x] = F.dinfo[threadIdx.x];
    reinterpret_cast<uint64_t*>(dtab + HVF_MAX_DEPTH)[threadIdx.x] = F.rbase[threadIdx.x];
  }
  __syncthreads();
}

__device__ __forceinline__ int4 miss_hit() { return make_int4(-1, -1, -1, __float_as_int(INFINITY)); }

// A launch reads each ray once and writes each hit once: streaming (non-temporal) accesses
// keep these arrays from evicting the format's nodes from L2.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ray_half(const float4* rays, size_t k) {
  const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(rays) + k);
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void put_hit(int4* hits, size_t k, int4 h) {
  const i32x4 v = {h.x, h.y, h.z, h.w};
  __builtin_nontemporal_store(v, reinterpret_cast<i32x4*>(hits) + k);
}

// The whole walk of one ray: its result (a miss if it never hits).
template <uint32_t FAM>
__device__ __forceinline__ int4 trace_one(const Fmt& fm, uint2* stk, const float4 r0, const float4 r1) {
  int4 out = miss_hit();
  Walk w;
  Plain mem;
  if (setup(r0, r1, fm.ext, w.R) && w.template start<FAM>(fm, mem) == RUN)
    while (w.template step<FAM>(fm, stk, out, mem) == RUN) {
    }
  return out;
}

// The walk of one ray for at most `budget` steps (0: no limit). A walk still running after
// them stops with *rest = its t, the entry time of the cell it would test next; the rest
// of the ray, [t, t1), is then traced by the split pass. *rest < 0 otherwise.
template <uint32_t FAM>
__device__ __forceinline__ int4 trace_budget(const Fmt& fm, uint2* stk, const float4 r0, const float4 r1,
                                             uint32_t budget, float* rest) {
  int4 out = miss_hit();
  Walk w;
  Plain mem;
  *rest = -1.0f;
  if (setup(r0, r1, fm.ext, w.R) && w.template start<FAM>(fm, mem) == RUN)
    while (w.template step<FAM>(fm, stk, out, mem) == RUN)
      if (w.steps == budget) {
        *rest = w.t;
        break;
      }
  return out;
}

// Append the lanes with rest >= 0 to the survivor list (ray index, t): one atomic per wave.
__device__ __forceinline__ void push_survivor(bool cut, uint32_t i, float rest, uint2* __restrict__ surv,
                                              uint32_t* __restrict__ nsurv) {
  const uint64_t cm = __ballot(cut);
  if (!cut) return;
  const uint32_t lane = threadIdx.x & 63u;
  const int leader = __ffsll((unsigned long long)cm) - 1;
  uint32_t base = 0;
  if ((int)lane == leader) base = atomicAdd(nsurv, (uint32_t)__popcll(cm));
  base = __shfl(base, leader);
  surv[base + (uint32_t)__popcll(cm & ((1ull << lane) - 1ull))] = make_uint2(i, __float_as_uint(rest));
}

// The ray of the lane with global index g: g itself, or with interleaving (W > 0: the
// number of waves that hold rays) lane l < R of wave w takes ray l * W + w, so a wave's
// rays are spread over the whole batch. Lanes from R on and waves from W on take none
// (n stands for "no ray"; an index of n or more is no ray either).
__device__ __forceinline__ uint32_t ray_of(uint32_t g, uint32_t W, uint32_t n, uint32_t R = 64u) {
  if (W == 0u) return g;
  const uint32_t w = g >> 6, l = g & 63u;
  return (w < W && l < R) ? l * W + w : n;
}

template <uint32_t FAM>
__global__ __launch_bounds__(BLOCK) void trace_kernel(const DevFormat F, const float4* __restrict__ rays,
                                                      int4* __restrict__ hits, uint32_t n, uint32_t W) {
  __shared__ __align__(8) uint32_t dtab[DTAB_WORDS];
  extern __shared__ uint2 stk_all[];
  const uint32_t* pre = stage_prefix(F, stk_all);
  load_dtab(F, dtab);
  const Fmt fm = fmt_of(F, dtab, pre);
  const uint32_t i = ray_of(blockIdx.x * BLOCK + threadIdx.x, W, n);
  if (i >= n) return;
  const float4 r0 = ray_half(rays, 2 * (size_t)i), r1 = ray_half(rays, 2 * (size_t)i + 1);
  put_hit(hits, i, F.lds_words ? trace_one<FAM | FAM_PRE>(fm, stk_all + threadIdx.x, r0, r1)
                        : trace_one<FAM>(fm, stk_all + threadIdx.x, r0, r1));
}

// First pass of the split schedule: trace_kernel with a step budget. Rays that finish
// write their result; the others join the survivor list for trace_split_kernel.
template <uint32_t FAM>
__global__ __launch_bounds__(BLOCK) void trace_budget_kernel(const DevFormat F, const float4* __restrict__ rays,
                                                             int4* __restrict__ hits, uint32_t n, uint32_t budget,
                                                             uint2* __restrict__ surv, uint32_t* __restrict__ nsurv) {
  __shared__ __align__(8) uint32_t dtab[DTAB_WORDS];
  extern __shared__ uint2 stk_all[];
  const uint32_t* pre = stage_prefix(F, stk_all);
  load_dtab(F, dtab);
  const Fmt fm = fmt_of(F, dtab, pre);
  const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  const float4 r0 = ray_half(rays, 2 * (size_t)i), r1 = ray_half(rays, 2 * (size_t)i + 1);
  float rest;
  const int4 out = F.lds_words ? trace_budget<FAM | FAM_PRE>(fm, stk_all + threadIdx.x, r0, r1, budget, &rest)
                               : trace_budget<FAM>(fm, stk_all + threadIdx.x, r0, r1, budget, &rest);
  const bool cut = rest >= 0.0f;
  if (!cut) put_hit(hits, i, out);
  push_survivor(cut, i, rest, surv, nsurv);
}

// Boundary k of the split of the rest [tc, t1) of a ray into K segments: tc, t1 at the
// ends, in between tc + (t1 - tc) * k / K (k / K is exact for a power of two K).
// Non-decreasing in k and never above t1, so the segments [f(k), f(k + 1)) partition
// [tc, t1) whatever the rounding.
__device__ __forceinline__ float split_time(float tc, float t1, uint32_t k, uint32_t K) {
  if (k == 0u) return tc;
  if (k == K) return t1;
  return tc + (t1 - tc) * ((float)k / (float)K);
}

// Second pass of the split schedule: each survivor's rest [tc, t1) is cut into K segments
// traced side by side, one lane each, by K consecutive lanes of a wave; each segment is a
// fresh walk from the root over its own interval. A walk over [a, b) tests every cell
// entered before b, and plane times are monotone in the plane coordinate, so a walk
// started at a stands in the cell the whole walk occupies at time a. Hence the result of
// the ray is that of its first segment with a result, and a miss if none has one. Wave w
// of the grid takes the groups of 64 / K survivors w, w + (waves in the grid), ... (a
// fixed stride: a shared work counter would serialise every wave on one address).
template <uint32_t FAM>
__device__ __forceinline__ void split_loop(const DevFormat& F, const Fmt& fm, uint2* stk,
                                           const float4* __restrict__ rays, int4* __restrict__ hits,
                                           const uint2* __restrict__ surv, uint32_t ns, uint32_t klog2) {
  const uint32_t lane = threadIdx.x & 63u, K = 1u << klog2, per_wave = 64u >> klog2;
  const uint32_t k = lane & (K - 1u), g0 = lane & ~(K - 1u);
  const uint64_t gmask = (K == 64u) ? ~0ull : ((1ull << K) - 1ull);
  const uint32_t waves = gridDim.x * (BLOCK / 64u), wave = blockIdx.x * (BLOCK / 64u) + threadIdx.x / 64u;
  for (uint32_t grp = wave;; grp += waves) {
    const uint32_t base = grp * per_wave;
    if (base >= ns) break;  // uniform across the wave
    const uint32_t sidx = base + (lane >> klog2);
    int4 out = miss_hit();
    uint32_t ray = 0;
    if (sidx < ns) {
      const uint2 sv = surv[sidx];
      ray = sv.x;
      const float tc = __uint_as_float(sv.y);
      const float4 r0 = ray_half(rays, 2 * (size_t)ray), r1 = ray_half(rays, 2 * (size_t)ray + 1);
      Walk w;
      Plain mem;
      if (setup(r0, r1, fm.ext, w.R)) {
        const float t1 = w.R.t1;
        w.R.t0 = split_time(tc, t1, k, K);
        w.R.t1 = split_time(tc, t1, k + 1u, K);
        if (w.R.t0 < w.R.t1 && w.template start<FAM>(fm, mem) == RUN)
          while (w.template step<FAM>(fm, stk, out, mem) == RUN) {
          }
      }
    }
    const uint64_t gm = (__ballot(out.x != -1) >> g0) & gmask;  // segments with a result
    const uint32_t first = gm ? (uint32_t)(__ffsll((unsigned long long)gm) - 1) : 0u;
    if (sidx < ns && k == first) put_hit(hits, ray, out);
  }
}

template <uint32_t FAM>
__global__ __launch_bounds__(BLOCK) void trace_split_kernel(const DevFormat F, const float4* __restrict__ rays,
                                                            int4* __restrict__ hits, const uint2* __restrict__ surv,
                                                            const uint32_t* __restrict__ nsurv, uint32_t klog2) {
  __shared__ __align__(8) uint32_t dtab[DTAB_WORDS];
  extern __shared__ uint2 stk_all[];
  const uint32_t* pre = stage_prefix(F, stk_all);
  load_dtab(F, dtab);
  const Fmt fm = fmt_of(F, dtab, pre);
  const uint32_t ns = *nsurv;
  // K adapts to the survivors: at most the schedule's K, and no more segments than the
  // grid has lanes (K = 1 for a long list: each survivor's rest walked by one lane).
  const uint32_t lanes = gridDim.x * BLOCK;
  uint32_t kl = klog2;
  while (kl > 0u && (uint64_t)ns << kl > lanes) --kl;
  if (F.lds_words)
    split_loop<FAM | FAM_PRE>(F, fm, stk_all + threadIdx.x, rays, hits, surv, ns, kl);
  else
    split_loop<FAM>(F, fm, stk_all + threadIdx.x, rays, hits, surv, ns, kl);
}

// Restart rounds of the split schedule, between its first and its last launch. Each
// survivor (ray, t) of the previous launch walks again from the root over [t, t1), which
// visits the cells the interrupted walk had still to visit, in the same order (see
// split_loop), for at most `budget` steps; a walk still running then joins the next list.
// Survivors sit densely in the list, so the waves of a round start full instead of
// carrying the finished lanes of the previous launch. Lane l of the grid takes survivors
// l, l + (lanes in the grid), ...; the loop bound is uniform per wave, so push_survivor's
// ballot sees every lane of the wave.
template <uint32_t FAM>
__device__ __forceinline__ void resume_loop(const Fmt& fm, uint2* stk, const float4* __restrict__ rays,
                                            int4* __restrict__ hits, const uint2* __restrict__ in, uint32_t ns,
                                            uint32_t budget, uint2* __restrict__ out, uint32_t* __restrict__ nout) {
  const uint32_t lanes = gridDim.x * BLOCK;
  for (uint32_t base = blockIdx.x * BLOCK + (threadIdx.x & ~63u); base < ns; base += lanes) {
    const uint32_t sidx = base + (threadIdx.x & 63u);
    bool cut = false;
    uint32_t ray = 0;
    float rest = -1.0f;
    if (sidx < ns) {
      const uint2 sv = in[sidx];
      ray = sv.x;
      const float4 r0 = ray_half(rays, 2 * (size_t)ray), r1 = ray_half(rays, 2 * (size_t)ray + 1);
      int4 res = miss_hit();
      Walk w;
      Plain mem;
      if (setup(r0, r1, fm.ext, w.R)) {
        w.R.t0 = __uint_as_float(sv.y);
        if (w.R.t0 < w.R.t1 && w.template start<FAM>(fm, mem) == RUN)
          while (w.template step<FAM>(fm, stk, res, mem) == RUN)
            if (w.steps == budget) {
              rest = w.t;
              cut = true;
              break;
            }
      }
      if (!cut) put_hit(hits, ray, res);
    }
    push_survivor(cut, ray, rest, out, nout);
  }
}

template <uint32_t FAM>
__global__ __launch_bounds__(BLOCK) void trace_resume_kernel(const DevFormat F, const float4* __restrict__ rays,
                                                             int4* __restrict__ hits, const uint2* __restrict__ in,
                                                             const uint32_t* __restrict__ nin, uint32_t budget,
                                                             uint2* __restrict__ out, uint32_t* __restrict__ nout) {
  __shared__ __align__(8) uint32_t dtab[DTAB_WORDS];
  extern __shared__ uint2 stk_all[];
  const uint32_t* pre = stage_prefix(F, stk_all);
  load_dtab(F, dtab);
  const Fmt fm = fmt_of(F, dtab, pre);
  const uint32_t ns = *nin;
  if (F.lds_words)
    resume_loop<FAM | FAM_PRE>(fm, stk_all + threadIdx.x, rays, hits, in, ns, budget, out, nout);
  else
    resume_loop<FAM>(fm, stk_all + threadIdx.x, rays, hits, in, ns, budget, out, nout);
}

template <uint32_t FAM>
__device__ __forceinline__ void persistent_loop(const Fmt& fm, uint2* stk, const float4* __restrict__ rays,
                                                int4* __restrict__ hits, uint32_t n, uint32_t* __restrict__ counter,
                                                uint32_t refill, uint32_t inner) {
  const uint32_t lane = __lane_id();
  Walk w;
  Plain mem;
  bool active = false;
  uint32_t ray = 0;
  int4 out = miss_hit();
  bool drained = false;
  for (;;) {
    const uint64_t idle = __ballot(!active);
    const uint32_t nidle = (uint32_t)__popcll(idle);
    if (!drained && (nidle >= refill || nidle == 64u)) {
      uint32_t first = 0;
      if (lane == (uint32_t)(__ffsll((unsigned long long)idle) - 1)) first = atomicAdd(counter, nidle);
      first = __shfl(first, __ffsll((unsigned long long)idle) - 1);
      if (first >= n) drained = true;
      if (!active) {
        const uint32_t rank = (uint32_t)__popcll(idle & ((1ull << lane) - 1ull));
        const uint32_t id = first + rank;
        if (id < n) {
          ray = id;
          out = miss_hit();
          const float4 r0 = ray_half(rays, 2 * (size_t)id), r1 = ray_half(rays, 2 * (size_t)id + 1);
          active = setup(r0, r1, fm.ext, w.R) && w.template start<FAM>(fm, mem) == RUN;
          if (!active) put_hit(hits, id, out);
        }
      }
    }
    if (drained && __ballot(active) == 0ull) break;
    if (active) {
      for (uint32_t k = 0; k < inner; ++k) {
        if (w.template step<FAM>(fm, stk, out, mem) == DONE) {
          put_hit(hits, ray, out);
          active = false;
          break;
        }
      }
    }
  }
}

// Persistent variant: a grid sized to the device; each wave keeps its lanes busy by
// fetching a new ray for every idle lane from a global counter whenever at least
// `refill` lanes are idle (or the whole wave is). *counter must be 0 at launch.
template <uint32_t FAM>
__global__ __launch_bounds__(BLOCK) void trace_persistent_kernel(const DevFormat F, const float4* __restrict__ rays,
                                                                 int4* __restrict__ hits, uint32_t n,
                                                                 uint32_t* __restrict__ counter, uint32_t refill,
                                                                 uint32_t inner) {
  __shared__ __align__(8) uint32_t dtab[DTAB_WORDS];
  extern __shared__ uint2 stk_all[];
  const uint32_t* pre = stage_prefix(F, stk_all);
  load_dtab(F, dtab);
  const Fmt fm = fmt_of(F, dtab, pre);
  uint2* stk = stk_all + threadIdx.x;
  if (F.lds_words)
    persistent_loop<FAM | FAM_PRE>(fm, stk, rays, hits, n, counter, refill, inner);
  else
    persistent_loop<FAM>(fm, stk, rays, hits, n, counter, refill, inner);
}

// ---------------------------------------------------------------- work stealing in a wave
// One lane per ray, and the lanes whose walks have ended take over the rest of walks still
// running in their wave. Every `period` steps (a power of two) a wave with at least
// `min_idle` idle lanes looks at its running walks. A walk (its part [t, t1) of a ray) whose rest is longer than the time `tv` the ray
// needs to cross `minlen` voxels along its fastest axis forks at the exit time e of one of
// its ancestor nodes (the shallowest one it has not tried, that ends before t1): the walk
// keeps [t, e) and an idle lane continues the walk exactly as the walk itself would after
// leaving that node: at time e, in the cell beyond it, under the deepest node holding that
// cell, with the donor's node stack for the depths above (copied from the donor's LDS
// column). No step is walked twice. A ray's result is the hit of least t over its parts (the
// parts visit disjoint runs of the walk's cells, each reporting true entry times), so each
// ray keeps its least hit key in LDS (an atomic min over the parts' reports) and at the end
// its own lane writes it; the voxel of a hit another lane found is recovered by the
// mid-plane descent from the root at the hit time, which lands in the cell entered at that
// time. A part stops as soon as its ray holds a hit no later than its current t (it cannot
// report an earlier one). Walks of their own lane's ray are forked first. Lanes past the last
// ray of the grid help too.

// Orderable key of a time: key(a) < key(b) iff a < b (non-NaN a, b); 0 and all ones are the
// keys of two NaNs, used as markers: a tripped step guard and "no hit yet".
constexpr uint32_t KEY_GUARD = 0u;
constexpr uint32_t KEY_NOHIT = 0xFFFFFFFFu;
__device__ __forceinline__ uint32_t time_key(float t) {
  const uint32_t b = __float_as_uint(t);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key_time(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// The voxel holding the ray at time t: the mid-plane descent from the root at t.
__device__ __forceinline__ int4 voxel_at(const Ray& R, const int32_t ext[3], float t) {
  int p[3] = {0, 0, 0};
  for (int b = max(ext[0], max(ext[1], ext[2])) - 1; b >= 0; --b) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (b >= ext[a]) continue;
      const int mid = p[a] + (1 << b);
      const bool up = (R.T(a, mid) <= t) != R.is_neg(a);
      p[a] = up ? mid : p[a];
    }
  }
  return make_int4(p[0], p[1], p[2], __float_as_int(t));
}

// Time for the ray to cross `minlen` voxels along its fastest axis (parallel axes carry
// 1/d = +inf and drop out of the min).
__device__ __forceinline__ float cross_time(const Ray& R, float minlen) {
  return minlen * fmin_fx(fmin_fx(fabsf(R.inv[0]), fabsf(R.inv[1])), fabsf(R.inv[2]));
}

// best, tbl: this wave's 64-word LDS arrays (least hit key per ray of the wave; the donor
// lane of each helper).
template <uint32_t FAM>
__device__ __forceinline__ void steal_loop(const Fmt& fm, uint2* stk, const float4* __restrict__ rays,
                                           int4* __restrict__ hits, uint32_t i, uint32_t n, uint32_t period,
                                           float minlen, uint32_t min_idle, uint32_t* best, uint32_t* tbl) {
  const uint32_t lane = __lane_id();
  const uint64_t below = (1ull << lane) - 1ull;
  Walk w{};
  Plain mem;
  int4 out = miss_hit();
  uint32_t home = lane;   // the lane (of this wave) whose ray the current part belongs to
  int kf = 1;             // shallowest ancestor depth this part may still fork at
  float tv = 0.0f;
  best[lane] = KEY_NOHIT;
  bool run = false;
  if (i < n) {
    const float4 r0 = ray_half(rays, 2 * (size_t)i), r1 = ray_half(rays, 2 * (size_t)i + 1);
    run = setup(r0, r1, fm.ext, w.R) && w.template start<FAM>(fm, mem) == RUN;
    tv = cross_time(w.R, minlen);
  }
  for (uint32_t it = 1;; ++it) {
    // The step guard counts the wave's iterations (a part never takes more steps than the
    // iterations since the launch began).
    if (run && (it > MAX_STEPS || w.template step<FAM, false>(fm, stk, out, mem) == DONE)) {
      run = false;
      if (it > MAX_STEPS) out.x = -2;
      if (out.x != -1)  // a hit, or the step guard (-2)
        atomicMin(&best[home], out.x == -2 ? KEY_GUARD : time_key(__int_as_float(out.w)));
      out.x = -1;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    if ((it & (period - 1u)) != 0u) {
      if (__ballot(run) == 0ull) break;
      continue;
    }
    if (run && best[home] <= time_key(w.t)) run = false;  // an earlier part already hit
    const uint64_t rm = __ballot(run);
    if (rm == 0ull) break;
    const uint32_t nidle = 64u - (uint32_t)__popcll(rm);
    if (nidle < min_idle) continue;
    bool want = false;
    float e = 0.0f;
    int q[3] = {0, 0, 0}, nd = 0;
    const int k = min(kf, w.d);  // an ancestor: the nodes above it are on the donor's stack
    const bool cand = run && k >= 1 && (w.R.t1 - w.t) > tv;
    if (__ballot(cand) == 0ull) continue;  // no walk long enough to fork
    if (cand) {
      e = w.node_exit(fm, k, q, nd);
      want = e < w.R.t1;
      if (!want) kf = k + 1;  // that node reaches t1: try the next depth next time
    }
    const uint64_t wh = __ballot(want && home == lane), wo = __ballot(want && home != lane);
    const uint32_t nh = (uint32_t)__popcll(wh), nw = nh + (uint32_t)__popcll(wo);
    if (nw == 0u) continue;
    const uint32_t pairs = min(nw, nidle);
    const uint32_t drank = home == lane ? (uint32_t)__popcll(wh & below) : nh + (uint32_t)__popcll(wo & below);
    const uint32_t irank = (uint32_t)__popcll(~rm & below);
    const bool donor = want && drank < pairs, recv = !run && irank < pairs;
    if (donor) tbl[drank] = lane;
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int src = recv ? (int)tbl[irank] : (int)lane;
    // Every lane of the wave is active here, so each shuffle reads its source lane.
    float f[8];
    f[0] = __shfl(w.R.o[0], src);
    f[1] = __shfl(w.R.o[1], src);
    f[2] = __shfl(w.R.o[2], src);
    f[3] = __shfl(w.R.inv[0], src);
    f[4] = __shfl(w.R.inv[1], src);
    f[5] = __shfl(w.R.inv[2], src);
    f[6] = __shfl(w.R.t1, src);
    f[7] = __shfl(e, src);
    int g[6];
    g[0] = __shfl(q[0], src);
    g[1] = __shfl(q[1], src);
    g[2] = __shfl(q[2], src);
    g[3] = __shfl(nd, src);
    g[4] = __shfl(k, src);
    g[5] = __shfl((int)(w.R.neg | (w.R.par << 3) | (home << 6)), src);
    if (donor) {
      w.R.t1 = e;
      kf = k + 1;
    }
    if (recv) {
      w.R.o[0] = f[0];
      w.R.o[1] = f[1];
      w.R.o[2] = f[2];
      w.R.inv[0] = f[3];
      w.R.inv[1] = f[4];
      w.R.inv[2] = f[5];
      w.R.t0 = f[7];
      w.R.t1 = f[6];
      w.R.neg = (uint32_t)g[5] & 7u;
      w.R.par = ((uint32_t)g[5] >> 3) & 7u;
      home = (uint32_t)g[5] >> 6;
      kf = g[4];
      tv = cross_time(w.R, minlen);
      // The donor's node stack for every depth at or above nd, then the walk state just
      // after leaving the donor's node: pop_to restores the node at depth nd.
      const int nn = g[3];
      const uint32_t ns = fm.stacked == ALL_STACKED ? (uint32_t)nn + 1u : slot_of(fm.stacked, nn + 1);
      const uint2* dstk = stk - lane + (uint32_t)src;
      for (uint32_t j0 = 0; j0 < ns; j0 += 4) {  // four reads in flight, then four writes
        uint2 v[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u)
          if (j0 + u < ns) v[u] = dstk[(j0 + u) * BLOCK];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u)
          if (j0 + u < ns) stk[(j0 + u) * BLOCK] = v[u];
      }
      w.t = f[7];
      w.p[0] = g[0];
      w.p[1] = g[1];
      w.p[2] = g[2];
      w.d = nn + 1;
      w.template pop_to<FAM>(fm, stk, nn, mem);
      run = true;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  if (i >= n) return;
  const uint32_t k = best[lane];
  int4 res = miss_hit();
  if (k == KEY_GUARD) {
    res = make_int4(-2, -2, -2, 0);
  } else if (k != KEY_NOHIT) {  // the voxel entered at the hit time, whichever lane found it
    const float4 r0 = ray_half(rays, 2 * (size_t)i), r1 = ray_half(rays, 2 * (size_t)i + 1);
    Ray R;
    (void)setup(r0, r1, fm.ext, R);
    res = voxel_at(R, fm.ext, key_time(k));
  }
  put_hit(hits, i, res);
}

template <uint32_t FAM>
__global__ __launch_bounds__(BLOCK) void trace_steal_kernel(const DevFormat F, const float4* __restrict__ rays,
                                                            int4* __restrict__ hits, uint32_t n, uint32_t period,
                                                            float minlen, uint32_t min_idle, uint32_t W, uint32_t R) {
  __shared__ __align__(8) uint32_t dtab[DTAB_WORDS];
  __shared__ uint32_t best_all[BLOCK], tbl_all[BLOCK];
  extern __shared__ uint2 stk_all[];
  const uint32_t* pre = stage_prefix(F, stk_all);
  load_dtab(F, dtab);
  const Fmt fm = fmt_of(F, dtab, pre);
  const uint32_t i = ray_of(blockIdx.x * BLOCK + threadIdx.x, W, n, R), w0 = threadIdx.x & ~63u;
  if (F.lds_words)
    steal_loop<FAM | FAM_PRE>(fm, stk_all + threadIdx.x, rays, hits, i, n, period, minlen, min_idle, best_all + w0,
                              tbl_all + w0);
  else
    steal_loop<FAM>(fm, stk_all + threadIdx.x, rays, hits, i, n, period, minlen, min_idle, best_all + w0,
                    tbl_all + w0);
}

// One lane per ray, rays taken in the order perm[] gives (results at each ray's index).
template <uint32_t FAM>
__global__ __launch_bounds__(BLOCK) void trace_indexed_kernel(const DevFormat F, const float4* __restrict__ rays,
                                                              int4* __restrict__ hits, uint32_t n,
                                                              const uint32_t* __restrict__ perm,
                                                              const uint32_t* __restrict__ key) {
  __shared__ __align__(8) uint32_t dtab[DTAB_WORDS];
  extern __shared__ uint2 stk_all[];
  const uint32_t* pre = stage_prefix(F, stk_all);
  load_dtab(F, dtab);
  const Fmt fm = fmt_of(F, dtab, pre);
  const uint32_t k = blockIdx.x * BLOCK + threadIdx.x;
  if (k >= n || key[k] == 0xFFFFFFFFu) return;  // rays that miss the root box were answered
  const uint32_t i = perm[k];
  const float4 r0 = ray_half(rays, 2 * (size_t)i), r1 = ray_half(rays, 2 * (size_t)i + 1);
  put_hit(hits, i, F.lds_words ? trace_one<FAM | FAM_PRE>(fm, stk_all + threadIdx.x, r0, r1)
                        : trace_one<FAM>(fm, stk_all + threadIdx.x, r0, r1));
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Coherence key of each ray: direction octant (3 high bits), then the Morton code of
// the cell of side 2^cell_bits holding the ray's entry point into the volume (29 bits,
// coarsest first). Rays that miss the root box get the key 0xFFFFFFFF and their miss is
// written here.
__global__ __launch_bounds__(BLOCK) void ray_key_kernel(const DevFormat F, const float4* __restrict__ rays,
                                                        int4* __restrict__ hits, uint32_t n, int cell_bits,
                                                        uint32_t* __restrict__ key, uint32_t* __restrict__ idx) {
  const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  const float4 r0 = ray_half(rays, 2 * (size_t)i), r1 = ray_half(rays, 2 * (size_t)i + 1);
  Ray R;
  uint32_t k = 0xFFFFFFFFu;
  if (setup(r0, r1, F.ext, R)) {
    const float d[3] = {r1.x, r1.y, r1.z};
    uint32_t c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float q = R.o[a] + R.t0 * d[a];  // approximate entry point: only orders rays
      const int N = 1 << F.ext[a];
      const int v = (int)fminf(fmaxf(floorf(q), 0.0f), (float)(N - 1));
      c[a] = (uint32_t)v >> cell_bits;
    }
    const uint32_t m = spread10(c[0]) | (spread10(c[1]) << 1) | (spread10(c[2]) << 2);  // up to 30 bits
    k = (R.neg << 29) | (m >> 1);
    if (k == 0xFFFFFFFFu) k = 0xFFFFFFFEu;
  } else {
    put_hit(hits, i, miss_hit());
  }
  key[i] = k;
  idx[i] = i;
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, uint32_t v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Batched persistent kernel: many volumes (formats, sizes) and ray batches in one launch.
// A global counter hands out indices of the concatenated ray space; an idle lane finds
// its batch by binary search over the batch start table, and walks that batch's volume.
// Per-depth descriptor tables of every batch and the start table live in LDS.
// LDS layout: dtab[items * 16] | start[items + 1] | stack[max_depth * BLOCK] (uint2).
template <uint32_t FAM>
__global__ __launch_bounds__(BLOCK) void trace_batch_kernel(const BatchItem* __restrict__ items,
                                                            const uint32_t* __restrict__ dinfo_all, uint32_t nitems,
                                                            uint32_t total, uint32_t* __restrict__ counter,
                                                            uint32_t refill, uint32_t inner) {
  extern __shared__ uint32_t smem[];
  uint32_t* dt = smem;
  uint32_t* start = smem + nitems * HVF_MAX_DEPTH;
  const uint32_t stk_off = (nitems * HVF_MAX_DEPTH + nitems + 1 + 1) & ~1u;
  uint2* stk = reinterpret_cast<uint2*>(smem + stk_off) + threadIdx.x;
  for (uint32_t i = threadIdx.x; i < nitems * HVF_MAX_DEPTH; i += BLOCK) dt[i] = dinfo_all[i];
  for (uint32_t i = threadIdx.x; i < nitems; i += BLOCK) start[i] = items[i].first;
  if (threadIdx.x == 0) start[nitems] = total;
  __syncthreads();
  const uint32_t lane = __lane_id();
  Walk w;
  Plain mem;
  Fmt fm;
  fm.buf = nullptr;
  fm.pop_lut = 0;
  fm.dtab = dt;
  fm.rtab = nullptr;  // per item: its region starts (region-aware kernels only read them)
  fm.ext[0] = fm.ext[1] = fm.ext[2] = 0;
  fm.stacked = 1u;
  fm.pre = nullptr;
  fm.npre = 0u;
  int4* hits = nullptr;
  bool active = false;
  uint32_t ray = 0;
  int4 out = miss_hit();
  bool drained = false;
  for (;;) {
    const uint64_t idle = __ballot(!active);
    const uint32_t nidle = (uint32_t)__popcll(idle);
    if (!drained && (nidle >= refill || nidle == 64u)) {
      const int leader = __ffsll((unsigned long long)idle) - 1;
      uint32_t first = 0;
      if ((int)lane == leader) first = atomicAdd(counter, nidle);
      first = __shfl(first, leader);
      if (first >= total) drained = true;
      if (!active) {
        const uint32_t id = first + (uint32_t)__popcll(idle & ((1ull << lane) - 1ull));
        if (id < total) {
          // batch b: the last with start[b] <= id
          uint32_t lo = 0, hi = nitems;
          while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (start[mid] <= id) lo = mid;
            else hi = mid;
          }
          const BatchItem& it = items[lo];
          fm.buf = as_global(it.buf);
          fm.pop_lut = it.pop_lut;
          fm.dtab = dt + lo * HVF_MAX_DEPTH;
          fm.ext[0] = it.ext[0];
          fm.ext[1] = it.ext[1];
          fm.ext[2] = it.ext[2];
          fm.stacked = it.stacked;
          fm.rtab = it.rtab;
          hits = reinterpret_cast<int4*>(it.hits);
          ray = id - it.first;
          const float4* rays = reinterpret_cast<const float4*>(it.rays);
          const float4 r0 = ray_half(rays, 2 * (size_t)ray), r1 = ray_half(rays, 2 * (size_t)ray + 1);
          out = miss_hit();
          active = setup(r0, r1, fm.ext, w.R) && w.template start<FAM>(fm, mem) == RUN;
          if (!active) put_hit(hits, ray, out);
        }
      }
    }
    if (drained && __ballot(active) == 0ull) break;
    if (active) {
      for (uint32_t k = 0; k < inner; ++k) {
        if (w.template step<FAM>(fm, stk, out, mem) == DONE) {
          put_hit(hits, ray, out);
          active = false;
          break;
        }
      }
    }
  }
}

// Same traversal as trace_kernel, logging the word index of every format load:
// log[i * cap + k] for the first cap loads of ray i; count[i] = number of loads.
template <uint32_t FAM>
__global__ __launch_bounds__(BLOCK) void trace_count_kernel(const DevFormat F, const float4* __restrict__ rays,
                                                            int4* __restrict__ hits, uint32_t n,
                                                            uint32_t* __restrict__ log, uint32_t cap,
                                                            uint32_t* __restrict__ count,
                                                            uint32_t* __restrict__ nsteps) {
  __shared__ __align__(8) uint32_t dtab[DTAB_WORDS];
  extern __shared__ uint2 stk_all[];
  const uint32_t* pre = stage_prefix(F, stk_all);
  load_dtab(F, dtab);
  const Fmt fm = fmt_of(F, dtab, pre);
  const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  const float4 r0 = ray_half(rays, 2 * (size_t)i), r1 = ray_half(rays, 2 * (size_t)i + 1);
  int4 out = miss_hit();
  Walk w;
  Counting mem{log + (size_t)i * cap, cap, 0u};
  w.steps = 0;
  if (setup(r0, r1, F.ext, w.R) && w.template start<FAM>(fm, mem) == RUN)
    while (w.template step<FAM>(fm, stk_all + threadIdx.x, out, mem) == RUN) {
    }
  put_hit(hits, i, out);
  count[i] = mem.k;
  if (nsteps) nsteps[i] = w.steps;
}

hvf_status launch_check(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    hvf_set_error(std::string(what) + " launch failed: " + hipGetErrorString(e));
    return HVF_E_DEVICE;
  }
  return HVF_OK;
}

int g_cu_count = -1;

}  // namespace

// Dynamic LDS of a single-volume trace kernel: the node stack, then the staged prefix.
size_t stack_lds_bytes(const DevFormat& F) {
  return (size_t)(F.nslots ? F.nslots : 1) * BLOCK * sizeof(uint2) + (size_t)F.lds_words * 4u;
}

#define HVF_FAMILY_SWITCH(family, LAUNCH) \
  switch (family) {                          \
    case 0: LAUNCH(FAM_BRICK); break;        \
    case 1: LAUNCH(FAM_DAG_BRICK); break;    \
    case 2: LAUNCH(FAM_SVO_BRICK); break;    \
    case 3: LAUNCH(FAM_RAW_BRICK); break;    \
    case 4: LAUNCH(FAM_OCTREE); break;       \
    case 5: LAUNCH(FAM_RAW_OCTREE); break;   \
    case 6: LAUNCH(FAM_DF_BRICK); break;     \
    case 7: LAUNCH(FAM_DF_OCTREE); break;    \
    case 8: LAUNCH(FAM_OCT_BRICK); break;    \
    case 9: LAUNCH(FAM_NODF); break;         \
    case 10: LAUNCH(FAM_PAPER); break;       \
    case 12: LAUNCH(FAM_ALL | FAM_REGIONS); break; \
    default: LAUNCH(FAM_ALL); break;         \
  }

hvf_status launch_trace(const DevFormat& F, int family, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits,
                        bool interleave, hipStream_t s) {
  if (n == 0) return HVF_OK;
  if (n >= (1ull << 32) - (interleave ? 64u : 0u)) {
    hvf_set_error(interleave ? "at most 2^32 - 65 interleaved rays per call" : "at most 2^32 - 1 rays per call");
    return HVF_E_INPUT;
  }
  const unsigned grid = (unsigned)((n + BLOCK - 1) / BLOCK);
  const float4* r = reinterpret_cast<const float4*>(d_rays);
  int4* h = reinterpret_cast<int4*>(d_hits);
  const uint32_t W = interleave ? (uint32_t)((n + 63) / 64) : 0u;
#define HVF_LAUNCH_TRACE(FAMV) \
  hipLaunchKernelGGL(trace_kernel<FAMV>, dim3(grid), dim3(BLOCK), stack_lds_bytes(F), s, F, r, h, (uint32_t)n, W)
  HVF_FAMILY_SWITCH(family, HVF_LAUNCH_TRACE)
#undef HVF_LAUNCH_TRACE
  return launch_check("trace");
}

hvf_status launch_trace_steal(const DevFormat& F, int family, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits,
                              uint32_t period, float minlen, uint32_t min_idle, bool interleave, uint32_t rays_per_wave,
                              hipStream_t s) {
  if (n == 0) return HVF_OK;
  if (n >= (1ull << 32) - BLOCK) {
    hvf_set_error("at most 2^32 - 257 rays per stealing call");
    return HVF_E_INPUT;
  }
  // With interleaving, R rays per wave over W = ceil(n / R) waves; else one ray per lane.
  const uint32_t R = (interleave && rays_per_wave >= 1u && rays_per_wave < 64u) ? rays_per_wave : 64u;
  const uint64_t W = interleave ? ((uint64_t)n + R - 1) / R : 0u;
  const uint64_t lanes = interleave ? W * 64u : (uint64_t)n;
  if (lanes >= (1ull << 32) - BLOCK) {
    hvf_set_error("too many waves for one stealing call (rays / rays_per_wave * 64 reaches 2^32)");
    return HVF_E_INPUT;
  }
  const unsigned grid = (unsigned)((lanes + BLOCK - 1) / BLOCK);
  const float4* r = reinterpret_cast<const float4*>(d_rays);
  int4* h = reinterpret_cast<int4*>(d_hits);
#define HVF_LAUNCH_STEAL(FAMV)                                                                                  \
  hipLaunchKernelGGL(trace_steal_kernel<FAMV>, dim3(grid), dim3(BLOCK), stack_lds_bytes(F), s, F, r, h, (uint32_t)n, \
                     period, minlen, min_idle, (uint32_t)W, R)
  HVF_FAMILY_SWITCH(family, HVF_LAUNCH_STEAL)
#undef HVF_LAUNCH_STEAL
  return launch_check("stealing trace");
}

hvf_status launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t s);

// The split schedule: trace_budget_kernel over all rays (budget steps), then `rounds`
// restart rounds of trace_resume_kernel over the survivors (budgets budget, 2 budget,
// 4 budget, ...: the walks are capped at budget * 2^r steps in all after round r), then
// trace_split_kernel over the last survivors; the later launches run on device-filling
// grids. Scratch: HVF_SPLIT_HEAD_WORDS survivor counters (zeroed here; count r belongs to
// the list launch r fills), then one or, with rounds, two lists of room for n survivors
// (8 bytes each) used in turn; split_scratch_words gives the size. The caller's buffer of
// that size, else one allocated for this call on s and freed after it.
hipError_t scratch_alloc(void** p, size_t bytes, hipStream_t s);

hvf_status launch_trace_split(const DevFormat& F, int family, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits,
                              uint32_t budget, uint32_t klog2, uint32_t rounds, uint32_t* scratch, hipStream_t s) {
  if (n == 0) return HVF_OK;
  if (n >= (1ull << 31)) {
    hvf_set_error("at most 2^31 - 1 rays per split call");
    return HVF_E_INPUT;
  }
  if (g_cu_count < 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
      hvf_set_error("hipGetDeviceProperties failed");
      return HVF_E_DEVICE;
    }
    g_cu_count = prop.multiProcessorCount;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, trace_split_kernel<FAM_ALL>, BLOCK, stack_lds_bytes(F)) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const unsigned grid2 = (unsigned)(g_cu_count * per_cu);
  if (rounds > HVF_SPLIT_MAX_ROUNDS || ((uint64_t)budget << (rounds ? rounds - 1 : 0)) >= (1ull << 31)) {
    hvf_set_error("split schedule: too many restart rounds for the budget");
    return HVF_E_INPUT;
  }
  const bool own = scratch == nullptr;
  if (own) {
    const hipError_t e =
        scratch_alloc(reinterpret_cast<void**>(&scratch), split_scratch_words(n, rounds) * sizeof(uint32_t), s);
    if (e != hipSuccess) {
      hvf_set_error(std::string("allocation of the split schedule's survivor lists: ") + hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? HVF_E_NOMEM : HVF_E_DEVICE;
    }
  }
  uint32_t* cnt = scratch;
  uint2* lists[2] = {reinterpret_cast<uint2*>(scratch + HVF_SPLIT_HEAD_WORDS),
                     reinterpret_cast<uint2*>(scratch + HVF_SPLIT_HEAD_WORDS + 2 * n)};
  uint32_t* nsurv = cnt;
  uint2* surv = lists[0];
  hvf_status st = launch_fill_u32(scratch, 0u, HVF_SPLIT_HEAD_WORDS, s);
  if (st != HVF_OK) {
    if (own) (void)hipFreeAsync(scratch, s);
    return st;
  }
  const unsigned grid = (unsigned)((n + BLOCK - 1) / BLOCK);
  const float4* r = reinterpret_cast<const float4*>(d_rays);
  int4* h = reinterpret_cast<int4*>(d_hits);
#define HVF_LAUNCH_BUDGET(FAMV)                                                                                   \
  hipLaunchKernelGGL(trace_budget_kernel<FAMV>, dim3(grid), dim3(BLOCK), stack_lds_bytes(F), s, F, r, h, (uint32_t)n, \
                     budget, surv, nsurv)
  HVF_FAMILY_SWITCH(family, HVF_LAUNCH_BUDGET)
#undef HVF_LAUNCH_BUDGET
  st = launch_check("budgeted trace");
  for (uint32_t k = 1; k <= rounds && st == HVF_OK; ++k) {
    const uint32_t bk = budget << (k - 1);
    uint2* const in = lists[(k - 1) & 1u];
    uint2* const out = lists[k & 1u];
#define HVF_LAUNCH_RESUME(FAMV)                                                                                      \
  hipLaunchKernelGGL(trace_resume_kernel<FAMV>, dim3(grid2), dim3(BLOCK), stack_lds_bytes(F), s, F, r, h, in, cnt + k - 1, \
                     bk, out, cnt + k)
    HVF_FAMILY_SWITCH(family, HVF_LAUNCH_RESUME)
#undef HVF_LAUNCH_RESUME
    st = launch_check("restart round of the split schedule");
    surv = out;
    nsurv = cnt + k;
  }
  if (st == HVF_OK) {
#define HVF_LAUNCH_SPLIT(FAMV)                                                                                    \
  hipLaunchKernelGGL(trace_split_kernel<FAMV>, dim3(grid2), dim3(BLOCK), stack_lds_bytes(F), s, F, r, h, surv, nsurv, \
                     klog2)
    HVF_FAMILY_SWITCH(family, HVF_LAUNCH_SPLIT)
#undef HVF_LAUNCH_SPLIT
    st = launch_check("split trace");
  }
  if (own) (void)hipFreeAsync(scratch, s);
  return st;
}

// Blocks of the persistent kernel per CU (at most blocks_per_cu if > 0) times CUs.
hvf_status persistent_grid(const DevFormat& F, int blocks_per_cu, unsigned* grid) {
  if (g_cu_count < 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
      hvf_set_error("hipGetDeviceProperties failed");
      return HVF_E_DEVICE;
    }
    g_cu_count = prop.multiProcessorCount;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, trace_persistent_kernel<FAM_ALL>, BLOCK,
                                                   stack_lds_bytes(F)) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (blocks_per_cu > 0 && blocks_per_cu < per_cu) per_cu = blocks_per_cu;
  *grid = (unsigned)(g_cu_count * per_cu);
  return HVF_OK;
}

hvf_status launch_trace_persistent(const DevFormat& F, int family, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits,
                                   uint32_t* d_counter, uint32_t refill, uint32_t inner, unsigned grid, hipStream_t s) {
  if (n == 0) return HVF_OK;
  if (n >= (1ull << 31)) {
    hvf_set_error("at most 2^31 - 1 rays per persistent call");
    return HVF_E_INPUT;
  }
  const float4* r = reinterpret_cast<const float4*>(d_rays);
  int4* h = reinterpret_cast<int4*>(d_hits);
#define HVF_LAUNCH_PERSISTENT(FAMV)                                                                                  \
  hipLaunchKernelGGL(trace_persistent_kernel<FAMV>, dim3(grid), dim3(BLOCK), stack_lds_bytes(F), s, F, r, h, \
                     (uint32_t)n, d_counter, refill, inner)
  HVF_FAMILY_SWITCH(family, HVF_LAUNCH_PERSISTENT)
#undef HVF_LAUNCH_PERSISTENT
  return launch_check("persistent trace");
}

size_t batch_lds_bytes(uint32_t nitems, int max_depth) {
  const size_t words = ((size_t)nitems * HVF_MAX_DEPTH + nitems + 1 + 1) & ~(size_t)1;
  return words * 4 + (size_t)max_depth * BLOCK * sizeof(uint2);
}

// kinds (batch_kernel_code): 0 = the library's layout without distance-field levels, 1 =
// with them, 2 = some volume in the paper's word layout (the batched kernel is compiled for
// that kind set); 3..6 = every volume in one brick-final family (its own kernel); 7 = some
// volume with per-depth regions (every kind, 64-bit word indices).
#define HVF_BATCH_SWITCH(kinds, LAUNCH)  \
  switch (kinds) {                       \
    case 2: LAUNCH(FAM_ANY); break;      \
    case 1: LAUNCH(FAM_ALL); break;      \
    case 3: LAUNCH(FAM_DAG_BRICK); break; \
    case 4: LAUNCH(FAM_SVO_BRICK); break; \
    case 5: LAUNCH(FAM_OCT_BRICK); break; \
    case 6: LAUNCH(FAM_RAW_BRICK); break; \
    case 7: LAUNCH(FAM_ANY | FAM_REGIONS); break; \
    default: LAUNCH(FAM_NODF); break;    \
  }
hvf_status batch_grid(uint32_t nitems, int max_depth, int kinds, int blocks_per_cu, unsigned* grid) {
  if (g_cu_count < 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
      hvf_set_error("hipGetDeviceProperties failed");
      return HVF_E_DEVICE;
    }
    g_cu_count = prop.multiProcessorCount;
  }
  int per_cu = 0;
  const size_t lds = batch_lds_bytes(nitems, max_depth);
  hipError_t oe = hipSuccess;
#define HVF_BATCH_OCCUPANCY(FAMV) oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, trace_batch_kernel<FAMV>, BLOCK, lds)
  HVF_BATCH_SWITCH(kinds, HVF_BATCH_OCCUPANCY)
#undef HVF_BATCH_OCCUPANCY
  if (oe != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (blocks_per_cu > 0 && blocks_per_cu < per_cu) per_cu = blocks_per_cu;
  *grid = (unsigned)(g_cu_count * per_cu);
  return HVF_OK;
}

hvf_status launch_trace_batch(const BatchItem* d_items, const uint32_t* d_dinfo, uint32_t nitems, uint32_t total,
                              int max_depth, int kinds, uint32_t* d_counter, uint32_t refill, uint32_t inner,
                              unsigned grid, hipStream_t s) {
  hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, s, d_counter, 0u, (size_t)1);
  hvf_status st = launch_check("fill");
  if (st != HVF_OK) return st;
#define HVF_LAUNCH_BATCH(FAMV)                                                                                       \
  hipLaunchKernelGGL(trace_batch_kernel<FAMV>, dim3(grid), dim3(BLOCK), batch_lds_bytes(nitems, max_depth), s, d_items, \
                     d_dinfo, nitems, total, d_counter, refill, inner)
  HVF_BATCH_SWITCH(kinds, HVF_LAUNCH_BATCH)
#undef HVF_LAUNCH_BATCH
  return launch_check("batched trace");
}

hvf_status launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t s) {
  if (n == 0) return HVF_OK;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, value, n);
  return launch_check("fill");
}

// Scratch of one call from the stream-ordered allocator: freed on the call's stream after
// its kernels, so calls on other streams never share it and concurrent traces of one
// volume are safe. The device's default pool keeps freed blocks for the next call (its
// release threshold is raised once per device).
hipError_t scratch_alloc(void** p, size_t bytes, hipStream_t s) {
  static std::once_flag pool_once[64];
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64)
    std::call_once(pool_once[dev], [dev] {
      hipMemPool_t pool;
      if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
      }
    });
  return hipMallocAsync(p, bytes, s);
}

hvf_status trace_sorted(const DevFormat& F, int family, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits,
                        const hvf_schedule& sc, hipStream_t s) {
  if (n >= (1ull << 31)) {
    hvf_set_error("at most 2^31 - 1 rays per sorted call");
    return HVF_E_INPUT;
  }
  const size_t arr = ((n * sizeof(uint32_t) + 255) / 256) * 256;
  size_t temp = 0;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, temp, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                         (const uint32_t*)nullptr, (uint32_t*)nullptr, (int)n, 0, 32, s) !=
      hipSuccess) {
    hvf_set_error("radix sort size query failed");
    return HVF_E_DEVICE;
  }
  void* buf = nullptr;
  const hipError_t e = scratch_alloc(&buf, 4 * arr + temp, s);
  if (e != hipSuccess) {
    hvf_set_error(std::string("allocation of sort scratch: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? HVF_E_NOMEM : HVF_E_DEVICE;
  }
  char* base = (char*)buf;
  uint32_t* key_in = (uint32_t*)base;
  uint32_t* idx_in = (uint32_t*)(base + arr);
  uint32_t* key_out = (uint32_t*)(base + 2 * arr);
  uint32_t* idx_out = (uint32_t*)(base + 3 * arr);
  void* tmp = base + 4 * arr;
  const unsigned grid = (unsigned)((n + BLOCK - 1) / BLOCK);
  hipLaunchKernelGGL(ray_key_kernel, dim3(grid), dim3(BLOCK), 0, s, F, reinterpret_cast<const float4*>(d_rays),
                     reinterpret_cast<int4*>(d_hits), (uint32_t)n, sc.sort_bits, key_in, idx_in);
  hvf_status st = launch_check("ray key");
  if (st == HVF_OK &&
      hipcub::DeviceRadixSort::SortPairs(tmp, temp, key_in, key_out, idx_in, idx_out, (int)n, 0, 32, s) !=
          hipSuccess) {
    hvf_set_error("radix sort failed");
    st = HVF_E_DEVICE;
  }
  if (st == HVF_OK) {
    const float4* r = reinterpret_cast<const float4*>(d_rays);
    int4* h = reinterpret_cast<int4*>(d_hits);
#define HVF_LAUNCH_INDEXED(FAMV)                                                                                      \
  hipLaunchKernelGGL(trace_indexed_kernel<FAMV>, dim3(grid), dim3(BLOCK), stack_lds_bytes(F), s, F, r, h, (uint32_t)n, \
                     idx_out, key_out)
    HVF_FAMILY_SWITCH(family, HVF_LAUNCH_INDEXED)
#undef HVF_LAUNCH_INDEXED
    st = launch_check("sorted trace");
  }
  (void)hipFreeAsync(buf, s);
  return st;
}

// The generic family walks every layout of the library's own; the paper's layout has its own.
hvf_status launch_trace_count(const DevFormat& F, bool paper, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits,
                              uint32_t* d_log, uint32_t cap, uint32_t* d_count, uint32_t* d_steps, hipStream_t s) {
  if (n == 0) return HVF_OK;
  if (n >= (1ull << 32)) {
    hvf_set_error("at most 2^32 - 1 rays per call");
    return HVF_E_INPUT;
  }
  const unsigned grid = (unsigned)((n + BLOCK - 1) / BLOCK);
  if (paper)
    hipLaunchKernelGGL(trace_count_kernel<FAM_PAPER>, dim3(grid), dim3(BLOCK), stack_lds_bytes(F), s, F,
                       reinterpret_cast<const float4*>(d_rays), reinterpret_cast<int4*>(d_hits), (uint32_t)n, d_log,
                       cap, d_count, d_steps);
  else if (F.regions)
    hipLaunchKernelGGL(trace_count_kernel<FAM_ALL | FAM_REGIONS>, dim3(grid), dim3(BLOCK), stack_lds_bytes(F), s, F,
                       reinterpret_cast<const float4*>(d_rays), reinterpret_cast<int4*>(d_hits), (uint32_t)n, d_log,
                       cap, d_count, d_steps);
  else
    hipLaunchKernelGGL(trace_count_kernel<FAM_ALL>, dim3(grid), dim3(BLOCK), stack_lds_bytes(F), s, F,
                       reinterpret_cast<const float4*>(d_rays), reinterpret_cast<int4*>(d_hits), (uint32_t)n, d_log,
                       cap, d_count, d_steps);
  return launch_check("counting trace");
}

}  // namespace hvf
