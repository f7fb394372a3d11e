// Construction of a format on the device from a device array of sorted Morton codes
// (the bottom-up construction of Sec. 4.1, reorganised as data-parallel passes).
//
// The result is word for word the buffer the host builder produces (same layout rules):
//  * the nodes of a depth are the distinct values of code >> 3s (s = log2 of the node side;
//    the root depth has one node). Sorted codes give them in Morton order, which is the
//    order in which a depth-first construction in Morton order creates them;
//  * a node's children are a contiguous run of the next depth's nodes: those whose key,
//    shifted to the node's side, equals the node's key. One flag pass and one scan over the
//    child keys give every child its parent and every parent its run;
//  * word offsets are assigned bottom-up. An SVDAG node below its level's root takes the
//    offset of the first node in Morton order with the same content (mask word and child
//    offsets) inside the same sub-volume, or inside the whole level with whole-level
//    de-duplication (Sec. 4.3). Equal content is found by sorting 64-bit content hashes
//    and confirmed word by word, so a hash collision never merges different nodes;
//  * depths are placed in order at 64-byte aligned word offsets (SVO pointer arrays right
//    after their depth) and child references are written as absolute word offsets;
//  * a distance-field level stores, for every empty cell of a grid (or block of a brick),
//    the L1 distance to the nearest occupied one capped at M. L1 distance splits by axis,
//    so forward and backward relaxations along x, then y, then z, one thread per line and
//    in place in the output, give the same integers as the host's breadth-first search.
// The paper's own word layout (--paper-layout) is built from the same nodes by run_paper
// (its write order is described with its kernels below).
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>
#include <algorithm>
#include <climits>
#include <new>
#include <string>
#include <vector>

#include "hvf_internal.h"

namespace hvf {
namespace {

constexpr unsigned TB = 256;

inline unsigned grid_for(size_t n) { return (unsigned)((n + TB - 1) / TB); }

// One coordinate (bits 0, 3, 6, ...) of an interleaved Morton code.
__device__ __forceinline__ uint64_t coord_of(uint64_t v) {
  v &= 0x1249249249249249ull;
  v = (v ^ (v >> 2)) & 0x10C30C30C30C30C3ull;
  v = (v ^ (v >> 4)) & 0x100F00F00F00F00Full;
  v = (v ^ (v >> 8)) & 0x1F0000FF0000FFull;
  v = (v ^ (v >> 16)) & 0x1F00000000FFFFull;
  v = (v ^ (v >> 32)) & 0x1FFFFFull;
  return v;
}

// err bit 0: not strictly ascending; bit 1: outside the volume.
__global__ void k_validate(const uint64_t* __restrict__ c, size_t n, int ex, int ey, int ez,
                           uint32_t* __restrict__ err) {
  const size_t i = (size_t)blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  const uint64_t v = c[i];
  uint32_t e = 0;
  if (i > 0 && v <= c[i - 1]) e |= 1u;
  if ((coord_of(v) >> ex) || (coord_of(v >> 1) >> ey) || (coord_of(v >> 2) >> ez) || (v >> 63)) e |= 2u;
  if (e) atomicOr(err, e);
}

// flag[i] = 1 where x[i] >> sh starts a new run.
__global__ void k_run_flags(const uint64_t* __restrict__ x, size_t n, int sh, uint32_t* __restrict__ flag) {
  const size_t i = (size_t)blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  flag[i] = (i == 0 || (x[i] >> sh) != (x[i - 1] >> sh)) ? 1u : 0u;
}

// out[rank - 1] = x >> sh at every run start (rank: inclusive scan of the flags).
__global__ void k_run_keys(const uint64_t* __restrict__ x, size_t n, int sh, const uint32_t* __restrict__ flag,
                           const uint32_t* __restrict__ rank, uint64_t* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * TB + threadIdx.x;
  if (i >= n || !flag[i]) return;
  out[rank[i] - 1u] = x[i] >> sh;
}

__global__ void k_decrement(uint32_t* __restrict__ x, size_t n) {
  const size_t i = (size_t)blockIdx.x * TB + threadIdx.x;
  if (i < n) x[i] -= 1u;
}

__global__ void k_iota(uint32_t* __restrict__ x, size_t n) {
  const size_t i = (size_t)blockIdx.x * TB + threadIdx.x;
  if (i < n) x[i] = (uint32_t)i;
}

__global__ void k_stride_ids(uint32_t* __restrict__ x, size_t n, uint32_t f) {
  const size_t i = (size_t)blockIdx.x * TB + threadIdx.x;
  if (i < n) x[i] = (uint32_t)i * f;
}

__global__ void k_gather(const uint32_t* __restrict__ src, const uint32_t* __restrict__ idx, size_t n,
                         uint32_t* __restrict__ dst) {
  const size_t i = (size_t)blockIdx.x * TB + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}

// First child and child count of every parent (children of a parent are contiguous and
// every parent has at least one): starts first, ends in a second pass.
__global__ void k_child_first(const uint32_t* __restrict__ par, size_t nc, uint32_t* __restrict__ first) {
  const size_t j = (size_t)blockIdx.x * TB + threadIdx.x;
  if (j >= nc) return;
  const uint32_t p = par[j];
  if (j == 0 || par[j - 1] != p) first[p] = (uint32_t)j;
}

__global__ void k_child_count(const uint32_t* __restrict__ par, size_t nc, const uint32_t* __restrict__ first,
                              uint32_t* __restrict__ count) {
  const size_t j = (size_t)blockIdx.x * TB + threadIdx.x;
  if (j >= nc) return;
  const uint32_t p = par[j];
  if (j + 1 == nc || par[j + 1] != p) count[p] = (uint32_t)(j + 1) - first[p];
}

// Octree mask words (child mask, also the leaf mask at a level's deepest depth): bit
// (child key & 7) for every child in the node's run of children.
__global__ void k_masks_children(const uint64_t* __restrict__ ckey, const uint32_t* __restrict__ first,
                                 const uint32_t* __restrict__ count, size_t n, int deepest,
                                 uint32_t* __restrict__ masks) {
  const size_t x = (size_t)blockIdx.x * TB + threadIdx.x;
  if (x >= n) return;
  const uint32_t f = first[x], c = count[x];
  uint32_t v = 0;
  for (uint32_t t = 0; t < c; ++t) v |= 1u << (uint32_t)(ckey[f + t] & 7u);
  masks[x] = v | (deepest ? (v << 8) : 0u);
}

// The same at the last level's deepest depth, whose children are voxels: the first code of
// every node (node = rank - 1; the root when rank is null) ORs the node's run of codes.
__global__ void k_masks_voxels(const uint64_t* __restrict__ codes, const uint32_t* __restrict__ rank, size_t n,
                               uint32_t* __restrict__ masks) {
  const size_t i = (size_t)blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  const uint32_t r = rank ? rank[i] : 1u;
  if (i > 0 && (!rank || rank[i - 1] == r)) return;
  uint32_t v = 0;
  for (size_t j = i; j < n && j < i + 8 && (!rank || rank[j] == r); ++j) v |= 1u << (uint32_t)(codes[j] & 7u);
  masks[r - 1u] = v | (v << 8);
}

// ---------------------------------------------------------------- SVDAG de-duplication
struct DagView {
  const uint32_t* masks;
  const uint32_t* first;  // null: no children (the last level's deepest depth)
  const uint32_t* count;
  const uint32_t* cid;    // children's word offsets at the next depth
  const uint32_t* group;  // sub-volume of each node; null with whole-level de-duplication
};

__device__ __forceinline__ uint64_t mix64(uint64_t h, uint64_t v) {
  h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
  h *= 0xBF58476D1CE4E5B9ull;
  return h ^ (h >> 29);
}

__global__ void k_dag_hash(DagView V, size_t n, uint64_t* __restrict__ hash) {
  const size_t x = (size_t)blockIdx.x * TB + threadIdx.x;
  if (x >= n) return;
  uint64_t h = mix64(0x51ED27D3A9C1B4F5ull, V.group ? V.group[x] : 0u);
  h = mix64(h, V.masks[x]);
  if (V.first) {
    const uint32_t f = V.first[x], c = V.count[x];
    for (uint32_t t = 0; t < c; ++t) h = mix64(h, V.cid[f + t]);
  }
  hash[x] = h;
}

__device__ bool dag_equal(const DagView& V, uint32_t a, uint32_t b) {
  if (V.masks[a] != V.masks[b]) return false;
  if (V.group && V.group[a] != V.group[b]) return false;
  if (!V.first) return true;
  const uint32_t fa = V.first[a], fb = V.first[b], c = V.count[a];
  if (V.count[b] != c) return false;
  for (uint32_t t = 0; t < c; ++t)
    if (V.cid[fa + t] != V.cid[fb + t]) return false;
  return true;
}

// head[k] = k at the start of a run of equal sorted hashes, else 0 (max-scanned after).
__global__ void k_hash_heads(const uint64_t* __restrict__ sh, size_t n, uint32_t* __restrict__ head) {
  const size_t k = (size_t)blockIdx.x * TB + threadIdx.x;
  if (k >= n) return;
  head[k] = (k == 0 || sh[k] != sh[k - 1]) ? (uint32_t)k : 0u;
}

// canon[x]: the first node in Morton order with x's content. A run of equal hashes lists
// its nodes in ascending index (stable sort of an ascending index), so the first equal
// entry of x's run is that node; the run's head is it unless hashes collide.
__global__ void k_canon(DagView V, const uint32_t* __restrict__ sidx, const uint32_t* __restrict__ head, size_t n,
                        uint32_t* __restrict__ canon) {
  const size_t k = (size_t)blockIdx.x * TB + threadIdx.x;
  if (k >= n) return;
  const uint32_t x = sidx[k];
  const uint32_t h = head[k];
  uint32_t c = x;
  if (h != (uint32_t)k) {
    if (dag_equal(V, sidx[h], x)) {
      c = sidx[h];
    } else {
      for (uint32_t q = h + 1; q < (uint32_t)k; ++q)
        if (dag_equal(V, sidx[q], x)) {
          c = sidx[q];
          break;
        }
    }
  }
  canon[x] = c;
}

// Words of the nodes that are stored (their own canonical node), 0 for merged ones.
__global__ void k_dag_sizes(const uint32_t* __restrict__ canon, const uint32_t* __restrict__ count, size_t n,
                            int inner, uint64_t* __restrict__ usize, uint32_t* __restrict__ uflag) {
  const size_t x = (size_t)blockIdx.x * TB + threadIdx.x;
  if (x >= n) return;
  const bool u = canon[x] == (uint32_t)x;
  const uint64_t len = 1u + (count ? count[x] : 0u) * (inner ? 2u : 1u);
  usize[x] = u ? len : 0u;
  uflag[x] = u ? 1u : 0u;
}

__global__ void k_dag_ids(const uint32_t* __restrict__ canon, const uint64_t* __restrict__ off, size_t n,
                          uint32_t* __restrict__ id) {
  const size_t x = (size_t)blockIdx.x * TB + threadIdx.x;
  if (x < n) id[x] = (uint32_t)off[canon[x]];
}

// ---------------------------------------------------------------- writing the buffer
// Bricks of the last Raw level: one bit per voxel in the 64-bit mask of its block. A
// block is an aligned cube of side 2^b, so its voxels are one run of codes with equal
// code >> 3b; the run's first code builds both mask words and stores them.
__global__ void k_write_bricks(const uint64_t* __restrict__ codes, const uint32_t* __restrict__ rank, size_t n,
                               int ns, int b, int wx, int wy, uint64_t stride, uint32_t bwords,
                               uint32_t* __restrict__ dst) {
  const size_t i = (size_t)blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  const uint64_t c = codes[i];
  const uint64_t blk_key = c >> (3 * b);
  if (i > 0 && (codes[i - 1] >> (3 * b)) == blk_key) return;
  const uint64_t local = rank ? (c & ((1ull << (3 * ns)) - 1ull)) : c;
  const uint64_t lx = coord_of(local), ly = coord_of(local >> 1), lz = coord_of(local >> 2);
  const uint64_t blk = (lx >> b) | ((ly >> b) << wx) | ((lz >> b) << (wx + wy));
  const uint64_t m = (1ull << b) - 1ull;
  const uint64_t span = 1ull << (3 * b);
  uint32_t w[2] = {0u, 0u};
  for (size_t j = i; j < n && j < i + span && (codes[j] >> (3 * b)) == blk_key; ++j) {
    const uint64_t v = codes[j];
    const uint64_t bit = (coord_of(v) & m) | ((coord_of(v >> 1) & m) << b) | ((coord_of(v >> 2) & m) << (2 * b));
    w[bit >> 5] |= 1u << (uint32_t)(bit & 31u);
  }
  const uint64_t node = rank ? rank[i] - 1u : 0u;
  uint32_t* o = dst + node * stride + bwords * blk;
  o[0] = w[0];
  o[1] = w[1];
}

// ---------------------------------------------------------------- distance fields
constexpr uint32_t DF_FAR = 1u << 30;  // "no occupied cell yet" during the relaxations

// Every cell (or block) of a distance-field depth: 0 if occupied, DF_FAR if empty. A
// pointer-grid cell is occupied once a child is marked (k_df_mark); a DF brick block
// holds its masks in words 0 and 1 and its distance in word 2.
__global__ void k_df_init(uint32_t* __restrict__ dst, size_t cells, uint32_t words, uint32_t off, int from_masks) {
  const size_t c = (size_t)blockIdx.x * TB + threadIdx.x;
  if (c >= cells) return;
  uint32_t* o = dst + c * words;
  o[off] = (from_masks && (o[0] | o[1]) != 0u) ? 0u : DF_FAR;
}

__global__ void k_df_mark(const uint64_t* __restrict__ ckey, const uint32_t* __restrict__ par, size_t nc, int w0,
                          int w1, int root, uint64_t cells, uint32_t* __restrict__ dst) {
  const size_t j = (size_t)blockIdx.x * TB + threadIdx.x;
  if (j >= nc) return;
  const uint64_t k = ckey[j];
  const uint64_t local = root ? k : (k & ((1ull << (3 * w0)) - 1ull));
  const uint64_t cell = coord_of(local) | (coord_of(local >> 1) << w0) | (coord_of(local >> 2) << (w0 + w1));
  dst[(uint64_t)(par ? par[j] : 0u) * cells + cell] = 0u;
}

// One line per thread: the cells of a node with all coordinates fixed but axis a, at a
// step of `step` cells; d = min(d, neighbour + 1) forward, then backward.
__global__ void k_df_relax(uint32_t* __restrict__ dst, size_t lines, uint32_t len, uint64_t step, uint64_t lo_mask,
                           int lo_bits, uint32_t words, uint32_t off) {
  const size_t l = (size_t)blockIdx.x * TB + threadIdx.x;
  if (l >= lines) return;
  // line l: its cells differ only in the axis-a coordinate; the coordinates below axis a
  // are the low lo_bits bits of l, those above it the rest, shifted past axis a.
  const uint64_t first = (l & lo_mask) | ((l >> lo_bits) << (lo_bits + __builtin_ctzll((unsigned long long)len)));
  uint32_t* o = dst + first * words + off;
  const uint64_t st = step * words;
  uint32_t prev = o[0];
  for (uint32_t i = 1; i < len; ++i) {
    uint32_t v = o[i * st];
    if (prev + 1u < v) {
      v = prev + 1u;
      o[i * st] = v;
    }
    prev = v;
  }
  for (uint32_t i = len - 1; i-- > 0;) {
    uint32_t v = o[i * st];
    if (prev + 1u < v) {
      v = prev + 1u;
      o[i * st] = v;
    }
    prev = v;
  }
}

// Final words: a DF pointer-grid cell that is empty becomes DF_EMPTY | min(M, d) (occupied
// cells keep 0 until their pointer is written); a DF brick block's word 2 becomes min(M, d).
__global__ void k_df_finish(uint32_t* __restrict__ dst, size_t cells, uint32_t words, uint32_t off, uint32_t cap,
                            int grid) {
  const size_t c = (size_t)blockIdx.x * TB + threadIdx.x;
  if (c >= cells) return;
  uint32_t* o = dst + c * words + off;
  const uint32_t d = *o < cap ? *o : cap;
  *o = grid ? (d ? (DF_EMPTY | d) : 0u) : d;
}

// Raw pointer grids: the cell of each child holds its absolute word offset (0 = empty).
// The root grid may be non-cubic (w0, w1 = log2 cells along x, y); below it the child key's
// low 3*w0 bits locate the cell.
__global__ void k_write_raw(const uint64_t* __restrict__ ckey, const uint32_t* __restrict__ par,
                            const uint32_t* __restrict__ cid, size_t nc, int w0, int w1, int root, uint64_t cells,
                            uint32_t child_base, uint32_t* __restrict__ dst) {
  const size_t j = (size_t)blockIdx.x * TB + threadIdx.x;
  if (j >= nc) return;
  const uint64_t k = ckey[j];
  const uint64_t local = root ? k : (k & ((1ull << (3 * w0)) - 1ull));
  const uint64_t cell = coord_of(local) | (coord_of(local >> 1) << w0) | (coord_of(local >> 2) << (w0 + w1));
  dst[(uint64_t)(par ? par[j] : 0u) * cells + cell] = child_base + cid[j];
}

// SVO nodes {first word, masks}. mode 1: children are this level's nodes (the first
// child's absolute offset); mode 2: children are next-level roots (absolute offset of the
// node's first entry in the depth's pointer array); mode 0: no children.
__global__ void k_write_svo(const uint32_t* __restrict__ masks, const uint32_t* __restrict__ first,
                            const uint32_t* __restrict__ cid, size_t n, int mode, uint32_t target,
                            uint32_t* __restrict__ dst) {
  const size_t x = (size_t)blockIdx.x * TB + threadIdx.x;
  if (x >= n) return;
  uint32_t w0 = 0;
  if (mode == 1) w0 = target + cid[first[x]];
  if (mode == 2) w0 = target + first[x];
  dst[2 * x] = w0;
  dst[2 * x + 1] = masks[x];
}

__global__ void k_write_ptrs(const uint32_t* __restrict__ cid, size_t nc, uint32_t child_base,
                             uint32_t* __restrict__ dst) {
  const size_t j = (size_t)blockIdx.x * TB + threadIdx.x;
  if (j < nc) dst[j] = child_base + cid[j];
}

// Stored SVDAG nodes: mask word, then per child its absolute offset, followed by the
// child's mask word when the children belong to the same level.
__global__ void k_write_dag(DagView V, const uint32_t* __restrict__ canon, const uint32_t* __restrict__ id,
                            const uint32_t* __restrict__ cmask, size_t n, int inner, uint32_t child_base,
                            uint32_t* __restrict__ dst) {
  const size_t x = (size_t)blockIdx.x * TB + threadIdx.x;
  if (x >= n || canon[x] != (uint32_t)x) return;
  uint32_t* o = dst + id[x];
  o[0] = V.masks[x];
  if (!V.first) return;
  const uint32_t f = V.first[x], c = V.count[x];
  for (uint32_t t = 0; t < c; ++t) {
    if (inner) {
      o[1 + 2 * t] = child_base + V.cid[f + t];
      o[2 + 2 * t] = cmask[f + t];
    } else {
      o[1 + t] = child_base + V.cid[f + t];
    }
  }
}

// ---------------------------------------------------------------- the paper's word layout
// The paper's layout (--paper-layout) is written in the order of the construction pass
// (Sec. 4.1): every node first has its children's sub-trees written, in Morton order, and
// then its own words ("units"):
//   * a Raw or DF node (one sub-volume of the level): its cells, or (term, distance) pairs;
//   * an SVO node: the block of its children's entries, two words each; a sub-volume's
//     root SVO node then also its own entry (pointer to that block, masks);
//   * an SVDAG node: the words of each child it stores, in child order (a child below the
//     root is stored only if no equal node was stored before it in the same sub-volume, or
//     level with whole-level de-duplication), then, for a sub-volume root, its own words.
// Word 0 holds the pointer to the level-0 root's words. Within one depth, that order visits
// nodes in Morton (index) order, so "stored first" is "first in index order" as for the
// library's layout, and offsets follow from per-node subtree sizes: W(x) = its children's W
// plus its own units, summed bottom-up, then start(child) = start(x) + the W of the
// children before it, top-down.

constexpr uint32_t PAPER_VOXEL = 0xFFFFFFFFu;  // an occupied voxel's RGBA word

// Sum of v over every node's run of children [first, first + count): E is the exclusive
// scan of v.
__global__ void kp_run_sum(const uint64_t* __restrict__ v, const uint64_t* __restrict__ E,
                           const uint32_t* __restrict__ first, const uint32_t* __restrict__ count, size_t n,
                           uint64_t* __restrict__ out) {
  const size_t x = (size_t)blockIdx.x * TB + threadIdx.x;
  if (x >= n) return;
  const uint32_t f = first[x], c = count[x];
  out[x] = c ? E[f + c - 1u] + v[f + c - 1u] - E[f] : 0u;
}

// Unit sizes of SVDAG children (and leaves) that are stored: 1 + children, 0 if merged;
// cnt null: leaves (one word each).
__global__ void kp_unit_sizes(const uint32_t* __restrict__ canon, const uint32_t* __restrict__ cnt, size_t n,
                              uint64_t* __restrict__ usize, uint32_t* __restrict__ uflag) {
  const size_t y = (size_t)blockIdx.x * TB + threadIdx.x;
  if (y >= n) return;
  const bool st = canon ? canon[y] == (uint32_t)y : true;
  usize[y] = st ? 1u + (cnt ? cnt[y] : 0u) : 0u;
  uflag[y] = st ? 1u : 0u;
}

// Own words and subtree words of every node of a depth. kind 0: Raw (own = cells * per);
// 1: SVO (2 per child, + 2 for a sub-volume root); 2: SVDAG (the stored children's words,
// + 1 + children for a sub-volume root). kidw: the children's subtree words (null at the
// deepest depth); ksum: the stored children's unit words (SVDAG).
__global__ void kp_own(int kind, int root, uint64_t rawwords, const uint32_t* __restrict__ count,
                       const uint64_t* __restrict__ kidw, const uint64_t* __restrict__ ksum, size_t n,
                       uint64_t* __restrict__ own, uint64_t* __restrict__ W) {
  const size_t x = (size_t)blockIdx.x * TB + threadIdx.x;
  if (x >= n) return;
  uint64_t o;
  if (kind == 0)
    o = rawwords;
  else if (kind == 1)
    o = 2ull * count[x] + (root ? 2u : 0u);
  else
    o = ksum[x] + (root ? 1ull + count[x] : 0u);
  own[x] = o;
  W[x] = o + (kidw ? kidw[x] : 0u);
}

// start(y) = start(parent) + the subtree words of the siblings before y (E: exclusive scan of
// W over the depth); null parent: the single root, starting at word 1.
__global__ void kp_start(const uint32_t* __restrict__ par, const uint32_t* __restrict__ pfirst,
                         const uint64_t* __restrict__ pstart, const uint64_t* __restrict__ E, size_t n,
                         uint64_t* __restrict__ start) {
  const size_t y = (size_t)blockIdx.x * TB + threadIdx.x;
  if (y >= n) return;
  if (!par) {
    start[y] = 1u + E[y];
    return;
  }
  const uint32_t p = par[y];
  start[y] = pstart[p] + E[y] - E[pfirst[p]];
}

// base(x): the first word of x's own units (after its children's sub-trees).
__global__ void kp_base(const uint64_t* __restrict__ start, const uint64_t* __restrict__ W,
                        const uint64_t* __restrict__ own, size_t n, uint64_t* __restrict__ base) {
  const size_t x = (size_t)blockIdx.x * TB + threadIdx.x;
  if (x < n) base[x] = start[x] + W[x] - own[x];
}

// Offset of each child's (or leaf's) unit inside its parent's run of child units: the
// parent's base plus the unit words of the siblings before it (E: exclusive scan of usize).
__global__ void kp_unit_off(const uint32_t* __restrict__ par, const uint32_t* __restrict__ pfirst,
                            const uint64_t* __restrict__ pbase, const uint64_t* __restrict__ E, size_t n,
                            uint64_t* __restrict__ uoff) {
  const size_t y = (size_t)blockIdx.x * TB + threadIdx.x;
  if (y >= n) return;
  const uint32_t p = par ? par[y] : 0u;
  uoff[y] = pbase[p] + E[y] - E[pfirst[p]];
}

// Offset of a sub-volume root's own words (what a parent level's term points at): a Raw
// node's cells at base; an SVO root's entry after its block; an SVDAG root's words after
// its stored children's.
__global__ void kp_root_off(int kind, const uint64_t* __restrict__ base, const uint64_t* __restrict__ own,
                            const uint32_t* __restrict__ count, size_t n, uint64_t* __restrict__ roff) {
  const size_t x = (size_t)blockIdx.x * TB + threadIdx.x;
  if (x >= n) return;
  uint64_t o = base[x];
  if (kind == 1) o += 2ull * count[x];
  if (kind == 2) o += own[x] - 1u - count[x];
  roff[x] = o;
}

// Raw/DF cells: each child (a next-level root, or a voxel of the last level) writes its
// terminating integer into its parent's cells (per words per cell: 1, or 2 with a distance).
__global__ void kp_write_raw(const uint64_t* __restrict__ ckey, const uint32_t* __restrict__ par,
                             const uint64_t* __restrict__ croot, size_t nc, int w0, int w1, int root, uint32_t per,
                             const uint64_t* __restrict__ pbase, uint64_t lim, uint32_t* __restrict__ err,
                             uint32_t* __restrict__ dst) {
  const size_t j = (size_t)blockIdx.x * TB + threadIdx.x;
  if (j >= nc) return;
  const uint64_t k = ckey[j];
  const uint64_t local = root ? k : (k & ((1ull << (3 * w0)) - 1ull));
  const uint64_t cell = coord_of(local) | (coord_of(local >> 1) << w0) | (coord_of(local >> 2) << (w0 + w1));
  const uint64_t at = pbase[par ? par[j] : 0u] + per * cell;
  if (at >= lim) {
    atomicOr(err, 1u);
    return;
  }
  dst[at] = croot ? (uint32_t)croot[j] : PAPER_VOXEL;
}

// DF distances in place in the (term, distance) pairs of every node of a depth: 0 where the
// term is not 0, else far; relaxed per axis; capped.
__global__ void kp_df_init(uint32_t* __restrict__ dst, const uint64_t* __restrict__ nbase, size_t nodes,
                           int cbits, uint64_t lim, uint32_t* __restrict__ err) {
  const size_t g = (size_t)blockIdx.x * TB + threadIdx.x;
  if (g >= (nodes << cbits)) return;
  const size_t node = g >> cbits;
  if (nbase[node] + (2ull << cbits) > lim) {  // the node's pairs must fit (the relaxations rely on it)
    atomicOr(err, 1u);
    return;
  }
  uint32_t* o = dst + nbase[node] + 2u * (g & ((1ull << cbits) - 1u));
  o[1] = o[0] ? 0u : DF_FAR;
}

__global__ void kp_df_relax(uint32_t* __restrict__ dst, const uint64_t* __restrict__ nbase, size_t lines,
                            int lbits, int cbits, uint32_t len, uint64_t step, uint64_t lo_mask, int lo_bits,
                            uint64_t lim) {
  const size_t g = (size_t)blockIdx.x * TB + threadIdx.x;
  if (g >= lines) return;
  const size_t node = g >> lbits, l = g & ((1ull << lbits) - 1u);
  if (nbase[node] + (2ull << cbits) > lim) return;  // reported by kp_df_init
  const uint64_t first = (l & lo_mask) | ((l >> lo_bits) << (lo_bits + __builtin_ctzll((unsigned long long)len)));
  uint32_t* o = dst + nbase[node] + 2u * first + 1u;
  const uint64_t st = 2u * step;
  uint32_t prev = o[0];
  for (uint32_t i = 1; i < len; ++i) {
    uint32_t v = o[i * st];
    if (prev + 1u < v) {
      v = prev + 1u;
      o[i * st] = v;
    }
    prev = v;
  }
  for (uint32_t i = len - 1; i-- > 0;) {
    uint32_t v = o[i * st];
    if (prev + 1u < v) {
      v = prev + 1u;
      o[i * st] = v;
    }
    prev = v;
  }
}

__global__ void kp_df_cap(uint32_t* __restrict__ dst, const uint64_t* __restrict__ nbase, size_t nodes, int cbits,
                          uint32_t cap, uint64_t lim) {
  const size_t g = (size_t)blockIdx.x * TB + threadIdx.x;
  if (g >= (nodes << cbits) || nbase[g >> cbits] + (2ull << cbits) > lim) return;
  uint32_t* o = dst + nbase[g >> cbits] + 2u * (g & ((1ull << cbits) - 1u)) + 1u;
  if (*o > cap) *o = cap;
}

// SVO blocks: entry t of node x's block is its child's (pointer to the child's block,
// masks), or at a level's deepest depth (the next-level root's words, 0) / (voxel, 0).
// A sub-volume root also writes its own entry after the block.
__global__ void kp_write_svo(const uint32_t* __restrict__ first, const uint32_t* __restrict__ count,
                             const uint32_t* __restrict__ masks, const uint64_t* __restrict__ base, size_t n,
                             int mode, const uint64_t* __restrict__ kbase, const uint32_t* __restrict__ kmasks,
                             const uint64_t* __restrict__ kroot, int root, uint64_t lim, uint32_t* __restrict__ err,
                             uint32_t* __restrict__ dst) {
  const size_t x = (size_t)blockIdx.x * TB + threadIdx.x;
  if (x >= n) return;
  const uint32_t f = first[x], c = count[x];
  if (base[x] + 2ull * c + (root ? 2u : 0u) > lim) {
    atomicOr(err, 1u);
    return;
  }
  uint32_t* o = dst + base[x];
  for (uint32_t t = 0; t < c; ++t) {
    if (mode == 0) {  // children at the next depth of this level
      o[2 * t] = (uint32_t)kbase[f + t];
      o[2 * t + 1] = kmasks[f + t];
    } else {  // leaves: next-level roots (mode 1) or voxels (mode 2)
      o[2 * t] = mode == 1 ? (uint32_t)kroot[f + t] : PAPER_VOXEL;
      o[2 * t + 1] = 0u;
    }
  }
  if (root) {
    o[2 * c] = (uint32_t)base[x];
    o[2 * c + 1] = masks[x];
  }
}

// SVDAG words {masks, pointer per child} of every stored node at its unit offset (roots at
// their root offset). Children's pointers go to their canonical (stored) unit.
__global__ void kp_write_dag(const uint32_t* __restrict__ canon, const uint32_t* __restrict__ first,
                             const uint32_t* __restrict__ count, const uint32_t* __restrict__ masks,
                             const uint64_t* __restrict__ off, size_t n, const uint32_t* __restrict__ kcanon,
                             const uint64_t* __restrict__ koff, uint64_t lim, uint32_t* __restrict__ err,
                             uint32_t* __restrict__ dst) {
  const size_t y = (size_t)blockIdx.x * TB + threadIdx.x;
  if (y >= n || (canon && canon[y] != (uint32_t)y)) return;
  const uint32_t f = first[y], c = count[y];
  if (off[y] + 1ull + c > lim) {
    atomicOr(err, 1u);
    return;
  }
  uint32_t* o = dst + off[y];
  o[0] = masks[y];
  for (uint32_t t = 0; t < c; ++t) {
    const uint32_t k = kcanon ? kcanon[f + t] : f + t;
    o[1 + t] = (uint32_t)koff[k];
  }
}

// SVDAG leaf words {terminating integer} of the stored leaves: a voxel (last level) or the
// next-level root's words.
__global__ void kp_write_leaves(const uint32_t* __restrict__ canon, const uint64_t* __restrict__ off,
                                const uint64_t* __restrict__ kroot, size_t n, uint64_t lim,
                                uint32_t* __restrict__ err, uint32_t* __restrict__ dst) {
  const size_t l = (size_t)blockIdx.x * TB + threadIdx.x;
  if (l >= n || (canon && canon[l] != (uint32_t)l)) return;
  if (off[l] >= lim) {
    atomicOr(err, 1u);
    return;
  }
  dst[off[l]] = kroot ? (uint32_t)kroot[l] : PAPER_VOXEL;
}

// head[i] = i where g changes (the first element of a run), else 0 (max-scanned after).
__global__ void kp_run_heads(const uint32_t* __restrict__ g, size_t n, uint32_t* __restrict__ head) {
  const size_t i = (size_t)blockIdx.x * TB + threadIdx.x;
  if (i < n) head[i] = (i == 0 || g[i] != g[i - 1]) ? (uint32_t)i : 0u;
}

__global__ void kp_masks_count(const uint32_t* __restrict__ masks, size_t n, uint32_t* __restrict__ count) {
  const size_t x = (size_t)blockIdx.x * TB + threadIdx.x;
  if (x < n) count[x] = (uint32_t)__popc(masks[x] & 0xFFu);
}

// ---------------------------------------------------------------- host orchestration
struct DepthState {
  size_t n = 0;               // nodes (before de-duplication)
  uint64_t* keys = nullptr;   // node keys (code >> 3*ns), ascending
  uint32_t* parent = nullptr; // parent index of every node (depths >= 1)
  uint32_t* first = nullptr;  // first child at the next depth
  uint32_t* count = nullptr;
  uint32_t* group = nullptr;  // SVDAG levels: index of the node's sub-volume root
  uint32_t* masks = nullptr;  // octree nodes: mask word
  uint32_t* canon = nullptr;  // SVDAG nodes: canonical node
  uint32_t* id = nullptr;     // word offset inside the depth
  uint64_t stored = 0;        // nodes stored
  uint64_t words = 0;         // arena words
  uint64_t aux = 0;           // pointer-array words (SVO nodes above the next level)
  int ns = 0;                 // log2 node side (depths >= 1)
};

class DeviceBuilder {
 public:
  DeviceBuilder(const Spec& s, const Layout& l, const uint64_t* codes, size_t n, hipStream_t st)
      : S(s), L(l), codes_(codes), n_(n), s_(st) {}
  ~DeviceBuilder() {
    // After an error, kernels launched before it may still use the temporaries.
    (void)hipStreamSynchronize(s_);
    for (void* p : chunks_) (void)hipFree(p);
    if (buf_) (void)hipFree(buf_);
  }

  hvf_status run(Built& B, uint32_t** dbuf, size_t* nwords);
  hvf_status run_paper(Built& B, uint32_t** dbuf, size_t* nwords);  // the paper's layout
  const std::string& error() const { return err_; }

 private:
  const Spec& S;
  const Layout& L;
  const uint64_t* codes_;
  size_t n_;
  hipStream_t s_;
  // Temporaries come from a few large chunks (a bump allocator), all freed at the end:
  // one hipMalloc per array would cost more than the construction's kernels.
  std::vector<void*> chunks_;
  char* chunk_ = nullptr;
  size_t left_ = 0;
  void* tmp_ = nullptr;
  size_t tmp_bytes_ = 0;
  uint32_t* buf_ = nullptr;
  std::string err_;
  hvf_status st_ = HVF_OK;

  bool fail(hvf_status s, const std::string& m) {
    if (st_ == HVF_OK) {
      st_ = s;
      err_ = m;
    }
    return false;
  }
  // Record an error and return its status (for `return stop(...)` in run()).
  hvf_status stop(hvf_status s, const std::string& m) {
    fail(s, m);
    return st_;
  }
  bool hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return true;
    return fail(e == hipErrorOutOfMemory ? HVF_E_NOMEM : HVF_E_DEVICE,
                std::string("device construction, ") + what + ": " + hipGetErrorString(e));
  }
  bool launched(const char* what) { return hip(hipGetLastError(), what); }
  template <class T>
  T* alloc(size_t count) {
    const size_t bytes = ((count ? count : 1) * sizeof(T) + 255) & ~(size_t)255;
    if (bytes > left_) {
      // Chunks of about 40 bytes per code (enough for the deepest depths' arrays at once), at
      // most 1 GiB unless one array needs more.
      const size_t hint = std::min((size_t)40 * n_ + ((size_t)8 << 20), (size_t)1 << 30);
      const size_t size = std::max(bytes, hint);
      void* p = nullptr;
      if (!hip(hipMalloc(&p, size), "hipMalloc of construction temporaries")) return nullptr;
      chunks_.push_back(p);
      chunk_ = static_cast<char*>(p);
      left_ = size;
    }
    void* r = chunk_;
    chunk_ += bytes;
    left_ -= bytes;
    return static_cast<T*>(r);
  }
  bool scratch(size_t bytes) {
    if (bytes <= tmp_bytes_) return true;
    tmp_ = alloc<char>(bytes);
    tmp_bytes_ = tmp_ ? bytes : 0;
    return tmp_ != nullptr;
  }
  template <class T>
  bool fetch(const T* p, T& v) {
    return hip(hipMemcpyAsync(&v, p, sizeof(T), hipMemcpyDeviceToHost, s_), "hipMemcpyAsync") &&
           hip(hipStreamSynchronize(s_), "hipStreamSynchronize");
  }
  bool inclusive_sum(const uint32_t* in, uint32_t* out, size_t n) {
    size_t b = 0;
    if (!hip(hipcub::DeviceScan::InclusiveSum(nullptr, b, in, out, (int)n, s_), "scan") || !scratch(b)) return false;
    return hip(hipcub::DeviceScan::InclusiveSum(tmp_, b, in, out, (int)n, s_), "scan");
  }
  bool exclusive_sum(const uint64_t* in, uint64_t* out, size_t n) {
    size_t b = 0;
    if (!hip(hipcub::DeviceScan::ExclusiveSum(nullptr, b, in, out, (int)n, s_), "scan") || !scratch(b)) return false;
    return hip(hipcub::DeviceScan::ExclusiveSum(tmp_, b, in, out, (int)n, s_), "scan");
  }
  bool max_scan(const uint32_t* in, uint32_t* out, size_t n) {
    size_t b = 0;
    if (!hip(hipcub::DeviceScan::InclusiveScan(nullptr, b, in, out, hipcub::Max(), (int)n, s_), "scan") ||
        !scratch(b))
      return false;
    return hip(hipcub::DeviceScan::InclusiveScan(tmp_, b, in, out, hipcub::Max(), (int)n, s_), "scan");
  }
  bool sum(const uint32_t* in, uint32_t* out, size_t n) {
    size_t b = 0;
    if (!hip(hipcub::DeviceReduce::Sum(nullptr, b, in, out, (int)n, s_), "reduce") || !scratch(b)) return false;
    return hip(hipcub::DeviceReduce::Sum(tmp_, b, in, out, (int)n, s_), "reduce");
  }
  bool sort_pairs(const uint64_t* kin, uint64_t* kout, const uint32_t* vin, uint32_t* vout, size_t n) {
    size_t b = 0;
    if (!hip(hipcub::DeviceRadixSort::SortPairs(nullptr, b, kin, kout, vin, vout, (int)n, 0, 64, s_), "sort") ||
        !scratch(b))
      return false;
    return hip(hipcub::DeviceRadixSort::SortPairs(tmp_, b, kin, kout, vin, vout, (int)n, 0, 64, s_), "sort");
  }

  static bool is_brick(const DepthInfo& di) {
    return di.nk == NK_BLOCKS || di.nk == NK_DF_BLOCKS || (di.nk == NK_CELLS && di.hk == HK_MASKLOAD);
  }
  static bool is_grid(const DepthInfo& di) { return di.nk == NK_RAW_PTR || di.nk == NK_DF_PTR; }
  // Words per node: a brick's blocks (2 words each, 4 with a distance), a grid's cells.
  static uint64_t node_words(const DepthInfo& di) {
    const int sw = di.w[0] + di.w[1] + di.w[2];
    if (di.nk == NK_DF_BLOCKS) return 4ull << sw;
    if (di.nk == NK_BLOCKS) return 2ull << sw;
    if (is_brick(di)) return 2ull;
    return 1ull << sw;
  }
  void relax_df(uint32_t* dst, size_t nodes, const int w[3], uint32_t words, uint32_t off);
  static bool is_octree(const DepthInfo& di) {
    return di.nk == NK_SVO_INNER || di.nk == NK_DAG_INNER || di.nk == NK_OCT_PTR || di.nk == NK_OCT_FINAL;
  }
  bool dedup(int i, std::vector<DepthState>& D, bool has_children);
  bool validate_codes();
  bool structure(std::vector<DepthState>& D, int dl, uint32_t*& code_rank);
  bool groups(std::vector<DepthState>& D, int dl);
  bool canon_of(const DagView& V, size_t n, uint32_t* canon);
  bool scan64(const uint64_t* v, size_t n, uint64_t*& E);
};

// SVDAG depth i: canonical nodes, stored-node offsets, word count.
bool DeviceBuilder::dedup(int i, std::vector<DepthState>& D, bool has_children) {
  const DepthInfo& di = L.d[i];
  DepthState& q = D[i];
  const size_t n = q.n;
  DagView V{q.masks, has_children ? q.first : nullptr, has_children ? q.count : nullptr,
            has_children ? D[i + 1].id : nullptr, S.wld ? nullptr : q.group};
  q.canon = alloc<uint32_t>(n);
  if (!q.canon) return false;
  if (di.j == 0) {
    // A sub-volume root is stored as is (its parent level points at it).
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(TB), 0, s_, q.canon, n);
    if (!launched("iota")) return false;
  } else {
    uint64_t* hash = alloc<uint64_t>(n);
    uint64_t* shash = alloc<uint64_t>(n);
    uint32_t* idx = alloc<uint32_t>(n);
    uint32_t* sidx = alloc<uint32_t>(n);
    uint32_t* head = alloc<uint32_t>(n);
    uint32_t* runh = alloc<uint32_t>(n);
    if (!hash || !shash || !idx || !sidx || !head || !runh) return false;
    hipLaunchKernelGGL(k_dag_hash, dim3(grid_for(n)), dim3(TB), 0, s_, V, n, hash);
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(TB), 0, s_, idx, n);
    if (!launched("hash") || !sort_pairs(hash, shash, idx, sidx, n)) return false;
    hipLaunchKernelGGL(k_hash_heads, dim3(grid_for(n)), dim3(TB), 0, s_, shash, n, head);
    if (!launched("heads") || !max_scan(head, runh, n)) return false;
    hipLaunchKernelGGL(k_canon, dim3(grid_for(n)), dim3(TB), 0, s_, V, sidx, runh, n, q.canon);
    if (!launched("canon")) return false;
  }
  uint64_t* usize = alloc<uint64_t>(n);
  uint64_t* off = alloc<uint64_t>(n);
  uint32_t* uflag = alloc<uint32_t>(n);
  uint32_t* nstored = alloc<uint32_t>(1);
  q.id = alloc<uint32_t>(n);
  if (!usize || !off || !uflag || !nstored || !q.id) return false;
  const int inner = di.nk == NK_DAG_INNER;
  hipLaunchKernelGGL(k_dag_sizes, dim3(grid_for(n)), dim3(TB), 0, s_, q.canon, V.count, n, inner, usize, uflag);
  if (!launched("sizes") || !exclusive_sum(usize, off, n) || !sum(uflag, nstored, n)) return false;
  hipLaunchKernelGGL(k_dag_ids, dim3(grid_for(n)), dim3(TB), 0, s_, q.canon, off, n, q.id);
  if (!launched("ids")) return false;
  uint64_t last_off = 0, last_size = 0;
  uint32_t stored = 0;
  if (!fetch(off + n - 1, last_off) || !fetch(usize + n - 1, last_size) || !fetch(nstored, stored)) return false;
  q.words = last_off + last_size;
  q.stored = stored;
  return true;
}

// Forward and backward relaxations along x, then y, then z over every node's grid of
// 2^w[0] x 2^w[1] x 2^w[2] cells (x fastest), `words` words per cell, distance at `off`.
void DeviceBuilder::relax_df(uint32_t* dst, size_t nodes, const int w[3], uint32_t words, uint32_t off) {
  const size_t cells = nodes << (w[0] + w[1] + w[2]);
  int lo = 0;
  for (int a = 0; a < 3; ++a) {
    const uint32_t len = 1u << w[a];
    if (len > 1u) {
      const size_t lines = cells >> w[a];
      hipLaunchKernelGGL(k_df_relax, dim3(grid_for(lines)), dim3(TB), 0, s_, dst, lines, len, 1ull << lo,
                         (1ull << lo) - 1ull, lo, words, off);
    }
    lo += w[a];
  }
}

hvf_status DeviceBuilder::run(Built& B, uint32_t** dbuf, size_t* nwords) {
  const int nd = (int)L.d.size();
  std::vector<DepthState> D(nd);
  for (int i = 1; i < nd; ++i) D[i].ns = L.d[i].cs + L.d[i].w[0];
  // 1. the codes: strictly ascending and inside the volume
  if (!validate_codes()) return st_;
  // Nodes of more than 2^31 words are out of range of the traversal's 32-bit offsets.
  bool df_ptr = false;
  for (const DepthInfo& di : L.d) {
    if ((is_grid(di) || is_brick(di)) && node_words(di) >= (1ull << 31))
      return stop(HVF_E_OVERFLOW, "a single node of this format needs 2^31 words or more, beyond 32-bit word offsets");
    df_ptr = df_ptr || di.nk == NK_DF_PTR;
  }
  // 2. node keys, bottom-up. The deepest stored depth takes its nodes from the codes (and
  //    keeps every code's node rank: bricks and final octree masks are filled per voxel).
  const int dl = L.d[nd - 1].arena ? nd - 1 : nd - 2;
  uint32_t* code_rank = nullptr;
  if (!structure(D, dl, code_rank)) return st_;
  // 3. sub-volume of every SVDAG node (top-down)
  if (!groups(D, dl)) return st_;
  // 4. word offsets inside every depth, bottom-up
  for (int i = dl; i >= 0; --i) {
    const DepthInfo& di = L.d[i];
    DepthState& q = D[i];
    const bool kids = i < dl;  // children at depth i + 1 (else voxels)
    if (is_brick(di) || is_grid(di)) {
      const uint64_t per = node_words(di);
      q.words = q.n * per;
      q.stored = q.n;
      if (q.words >= (1ull << 32)) return stop(HVF_E_OVERFLOW, "format needs 2^32 words or more");
      if (!(q.id = alloc<uint32_t>(q.n))) return st_;
      hipLaunchKernelGGL(k_stride_ids, dim3(grid_for(q.n)), dim3(TB), 0, s_, q.id, q.n, (uint32_t)per);
      if (!launched("ids")) return st_;
      continue;
    }
    if (!is_octree(di)) return stop(HVF_E_UNSUPPORTED, "node kind not built on the device");
    if (!(q.masks = alloc<uint32_t>(q.n))) return st_;
    const int deepest = di.nk == NK_OCT_FINAL || di.nk == NK_OCT_PTR;
    if (kids)
      hipLaunchKernelGGL(k_masks_children, dim3(grid_for(q.n)), dim3(TB), 0, s_, D[i + 1].keys, q.first, q.count, q.n,
                         deepest, q.masks);
    else
      hipLaunchKernelGGL(k_masks_voxels, dim3(grid_for(n_)), dim3(TB), 0, s_, codes_, code_rank, n_, q.masks);
    if (!launched("masks")) return st_;
    if (di.hk == HK_SVO) {
      q.words = 2ull * q.n;
      q.stored = q.n;
      q.aux = (di.nk == NK_OCT_PTR) ? D[i + 1].n : 0;
      if (!(q.id = alloc<uint32_t>(q.n))) return st_;
      hipLaunchKernelGGL(k_stride_ids, dim3(grid_for(q.n)), dim3(TB), 0, s_, q.id, q.n, 2u);
      if (!launched("ids")) return st_;
    } else if (!dedup(i, D, kids)) {
      return st_;
    }
    if (q.words >= (1ull << 32)) return stop(HVF_E_OVERFLOW, "format needs 2^32 words or more");
  }
  // 5. placement: depths in order, each at a 64-byte boundary, pointer arrays after them
  std::vector<uint64_t> base(nd), auxb(nd);
  uint64_t cur = 1;
  for (int i = 0; i < nd; ++i) {
    cur = (cur + 15) & ~15ull;
    base[i] = cur;
    cur += D[i].words;
    auxb[i] = cur;
    cur += D[i].aux;
  }
  // One buffer of 32-bit pointers while it fits (31 bits below a DF pointer grid, whose
  // cells keep the top bit for empty ones); past that, or with --depth-buffers, per-depth
  // regions with pointers relative to the region they point into, each within that bound.
  bool regions = S.regions;
  if (!regions && cur >= (df_ptr ? (1ull << 31) : (1ull << 32))) regions = true;
  if (regions)
    for (int i = 0; i < nd; ++i) {
      const uint64_t size = ((i + 1 < nd) ? base[i + 1] : cur) - base[i] + REGION_BIAS;
      const bool below_df = i > 0 && L.d[i - 1].nk == NK_DF_PTR;
      if (size >= (below_df ? (1ull << 31) : (1ull << 32)))
        return stop(HVF_E_OVERFLOW, "format needs " + std::to_string(cur) + " words, and its depth " +
                                        std::to_string(i) + " alone " + std::to_string(size) + ", beyond " +
                                        (below_df ? "31" : "32") + "-bit region-relative pointers");
    }
  // Spare zero words after the buffer; with regions, the table of region starts after them.
  const size_t total = regions ? region_table_word((size_t)cur) + 2 * HVF_MAX_DEPTH : (size_t)cur + HVF_BUFFER_PAD_WORDS;
  if (!hip(hipMalloc(&buf_, total * sizeof(uint32_t)), "hipMalloc of the word buffer") ||
      !hip(hipMemsetAsync(buf_, 0, total * sizeof(uint32_t), s_), "hipMemsetAsync"))
    return st_;
  // 6. node words with absolute child offsets, or offsets relative to the region of the
  //    depth they point into (the next depth's; an SVO node's pointer array lies in its own)
  for (int i = 0; i <= dl; ++i) {
    const DepthInfo& di = L.d[i];
    const DepthState& q = D[i];
    uint32_t* dst = buf_ + base[i];
    const uint32_t nb = regions ? (uint32_t)REGION_BIAS : (i + 1 < nd) ? (uint32_t)base[i + 1] : 0u;
    if (is_brick(di)) {
      const bool blocks = di.nk == NK_BLOCKS || di.nk == NK_DF_BLOCKS;
      const int wx = blocks ? di.w[0] : 0, wy = blocks ? di.w[1] : 0;
      const uint32_t bwords = di.nk == NK_DF_BLOCKS ? 4u : 2u;
      hipLaunchKernelGGL(k_write_bricks, dim3(grid_for(n_)), dim3(TB), 0, s_, codes_, i == 0 ? nullptr : code_rank,
                         n_, q.ns, L.brick_b, wx, wy, node_words(di), bwords, dst);
      if (di.nk == NK_DF_BLOCKS) {
        const size_t cells = q.n << (di.w[0] + di.w[1] + di.w[2]);
        hipLaunchKernelGGL(k_df_init, dim3(grid_for(cells)), dim3(TB), 0, s_, dst, cells, 4u, 2u, 1);
        relax_df(dst, q.n, di.w, 4u, 2u);
        hipLaunchKernelGGL(k_df_finish, dim3(grid_for(cells)), dim3(TB), 0, s_, dst, cells, 4u, 2u,
                           (uint32_t)S.lv[di.level].maxd, 0);
      }
    } else if (is_grid(di)) {
      const DepthState& c = D[i + 1];
      const uint64_t cells = 1ull << (di.w[0] + di.w[1] + di.w[2]);
      if (di.nk == NK_DF_PTR) {
        const size_t all = q.n * cells;
        hipLaunchKernelGGL(k_df_init, dim3(grid_for(all)), dim3(TB), 0, s_, dst, all, 1u, 0u, 0);
        hipLaunchKernelGGL(k_df_mark, dim3(grid_for(c.n)), dim3(TB), 0, s_, c.keys, i == 0 ? nullptr : c.parent, c.n,
                           di.w[0], di.w[1], i == 0 ? 1 : 0, cells, dst);
        relax_df(dst, q.n, di.w, 1u, 0u);
        hipLaunchKernelGGL(k_df_finish, dim3(grid_for(all)), dim3(TB), 0, s_, dst, all, 1u, 0u,
                           (uint32_t)S.lv[di.level].maxd, 1);
      }
      hipLaunchKernelGGL(k_write_raw, dim3(grid_for(c.n)), dim3(TB), 0, s_, c.keys, i == 0 ? nullptr : c.parent, c.id,
                         c.n, di.w[0], di.w[1], i == 0 ? 1 : 0, cells, nb, dst);
    } else if (di.hk == HK_SVO) {
      const int mode = di.nk == NK_SVO_INNER ? 1 : (di.nk == NK_OCT_PTR ? 2 : 0);
      const uint32_t target = mode == 1 ? nb : (uint32_t)(regions ? auxb[i] - base[i] + REGION_BIAS : auxb[i]);
      hipLaunchKernelGGL(k_write_svo, dim3(grid_for(q.n)), dim3(TB), 0, s_, q.masks, q.first,
                         mode == 1 ? D[i + 1].id : nullptr, q.n, mode, target, dst);
      if (mode == 2)
        hipLaunchKernelGGL(k_write_ptrs, dim3(grid_for(D[i + 1].n)), dim3(TB), 0, s_, D[i + 1].id, D[i + 1].n, nb,
                           buf_ + auxb[i]);
    } else {
      const bool kids = i < dl && di.nk != NK_OCT_FINAL;
      DagView V{q.masks, kids ? q.first : nullptr, kids ? q.count : nullptr, kids ? D[i + 1].id : nullptr, nullptr};
      const int inner = di.nk == NK_DAG_INNER;
      hipLaunchKernelGGL(k_write_dag, dim3(grid_for(q.n)), dim3(TB), 0, s_, V, q.canon, q.id,
                         inner ? D[i + 1].masks : nullptr, q.n, inner, nb, dst);
    }
    if (!launched("write")) return st_;
  }
  // the root is the first node of depth 0
  const uint32_t root = regions ? (uint32_t)REGION_BIAS : (uint32_t)base[0];
  if (!hip(hipMemcpyAsync(buf_, &root, sizeof(uint32_t), hipMemcpyHostToDevice, s_), "hipMemcpyAsync")) return st_;
  uint64_t rtab[HVF_MAX_DEPTH] = {};
  for (int i = 0; i < nd && regions; ++i) rtab[i] = base[i] - REGION_BIAS;
  if (regions && !hip(hipMemcpyAsync(buf_ + region_table_word((size_t)cur), rtab, sizeof(rtab), hipMemcpyHostToDevice, s_),
                      "hipMemcpyAsync"))
    return st_;
  if (!hip(hipStreamSynchronize(s_), "hipStreamSynchronize")) return st_;
  // 7. statistics (the host copy of the words is downloaded when first read)
  B.regions = regions;
  B.nvox = n_;
  B.depth_nodes.assign(nd, 0);
  B.depth_offset.assign(nd, 0);
  B.depth_words.assign(nd, 0);
  B.level_nodes.assign(S.lv.size(), 0);
  for (int i = 0; i < nd; ++i) {
    B.depth_nodes[i] = D[i].stored;
    B.depth_offset[i] = base[i];
    B.depth_words[i] = D[i].words + D[i].aux;
    B.level_nodes[L.d[i].level] += D[i].stored;
  }
  *nwords = (size_t)cur;
  *dbuf = buf_;
  buf_ = nullptr;
  return HVF_OK;
}


// Strictly ascending codes inside the volume (else a recorded error).
bool DeviceBuilder::validate_codes() {
  uint32_t* err = alloc<uint32_t>(1);
  if (!err || !hip(hipMemsetAsync(err, 0, sizeof(uint32_t), s_), "hipMemsetAsync")) return false;
  hipLaunchKernelGGL(k_validate, dim3(grid_for(n_)), dim3(TB), 0, s_, codes_, n_, S.ext[0], S.ext[1], S.ext[2], err);
  uint32_t herr = 0;
  if (!launched("validate") || !fetch(err, herr)) return false;
  if (herr & 1u) return fail(HVF_E_INPUT, "Morton codes must be strictly ascending");
  if (herr & 2u) return fail(HVF_E_INPUT, "Morton code outside the volume");
  return true;
}

// Node keys of every depth down to dl (the deepest takes them from the codes and keeps
// every code's node rank in code_rank), every node's parent, and every parent's run of
// children.
bool DeviceBuilder::structure(std::vector<DepthState>& D, int dl, uint32_t*& code_rank) {
  uint32_t* flag = alloc<uint32_t>(n_);
  if (!flag) return false;
  code_rank = nullptr;
  if (dl == 0) {
    D[0].n = 1;
  } else {
    DepthState& q = D[dl];
    code_rank = alloc<uint32_t>(n_);
    if (!code_rank) return false;
    hipLaunchKernelGGL(k_run_flags, dim3(grid_for(n_)), dim3(TB), 0, s_, codes_, n_, 3 * q.ns, flag);
    uint32_t cnt = 0;
    if (!launched("flags") || !inclusive_sum(flag, code_rank, n_) || !fetch(code_rank + n_ - 1, cnt)) return false;
    q.n = cnt;
    if (!(q.keys = alloc<uint64_t>(q.n))) return false;
    hipLaunchKernelGGL(k_run_keys, dim3(grid_for(n_)), dim3(TB), 0, s_, codes_, n_, 3 * q.ns, flag, code_rank, q.keys);
    if (!launched("keys")) return false;
  }
  for (int i = dl - 1; i >= 0; --i) {
    DepthState& q = D[i];
    DepthState& c = D[i + 1];
    if (!(c.parent = alloc<uint32_t>(c.n))) return false;
    if (i == 0) {
      q.n = 1;
      if (!hip(hipMemsetAsync(c.parent, 0, c.n * sizeof(uint32_t), s_), "hipMemsetAsync")) return false;
    } else {
      const int sh = 3 * (q.ns - c.ns);
      hipLaunchKernelGGL(k_run_flags, dim3(grid_for(c.n)), dim3(TB), 0, s_, c.keys, c.n, sh, flag);
      uint32_t cnt = 0;
      if (!launched("flags") || !inclusive_sum(flag, c.parent, c.n) || !fetch(c.parent + c.n - 1, cnt)) return false;
      q.n = cnt;
      if (!(q.keys = alloc<uint64_t>(q.n))) return false;
      hipLaunchKernelGGL(k_run_keys, dim3(grid_for(c.n)), dim3(TB), 0, s_, c.keys, c.n, sh, flag, c.parent, q.keys);
      hipLaunchKernelGGL(k_decrement, dim3(grid_for(c.n)), dim3(TB), 0, s_, c.parent, c.n);
      if (!launched("parents")) return false;
    }
    q.first = alloc<uint32_t>(q.n);
    q.count = alloc<uint32_t>(q.n);
    if (!q.first || !q.count) return false;
    hipLaunchKernelGGL(k_child_first, dim3(grid_for(c.n)), dim3(TB), 0, s_, c.parent, c.n, q.first);
    hipLaunchKernelGGL(k_child_count, dim3(grid_for(c.n)), dim3(TB), 0, s_, c.parent, c.n, q.first, q.count);
    if (!launched("child runs")) return false;
  }
  return true;
}

// Sub-volume (the index of its level's root node) of every SVDAG node, top-down; none with
// whole-level de-duplication.
bool DeviceBuilder::groups(std::vector<DepthState>& D, int dl) {
  if (S.wld) return true;
  for (int i = 0; i <= dl; ++i) {
    const DepthInfo& di = L.d[i];
    if (S.lv[di.level].kind != LK_DAG) continue;
    DepthState& q = D[i];
    if (!(q.group = alloc<uint32_t>(q.n))) return false;
    if (di.j == 0)
      hipLaunchKernelGGL(k_iota, dim3(grid_for(q.n)), dim3(TB), 0, s_, q.group, q.n);
    else
      hipLaunchKernelGGL(k_gather, dim3(grid_for(q.n)), dim3(TB), 0, s_, D[i - 1].group, q.parent, q.n, q.group);
    if (!launched("groups")) return false;
  }
  return true;
}

// canon[x]: the first node in index order with x's content (V: masks, children's canonical
// ids, group), found through sorted content hashes and confirmed word by word.
bool DeviceBuilder::canon_of(const DagView& V, size_t n, uint32_t* canon) {
  uint64_t* hash = alloc<uint64_t>(n);
  uint64_t* shash = alloc<uint64_t>(n);
  uint32_t* idx = alloc<uint32_t>(n);
  uint32_t* sidx = alloc<uint32_t>(n);
  uint32_t* head = alloc<uint32_t>(n);
  uint32_t* runh = alloc<uint32_t>(n);
  if (!hash || !shash || !idx || !sidx || !head || !runh) return false;
  hipLaunchKernelGGL(k_dag_hash, dim3(grid_for(n)), dim3(TB), 0, s_, V, n, hash);
  hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(TB), 0, s_, idx, n);
  if (!launched("hash") || !sort_pairs(hash, shash, idx, sidx, n)) return false;
  hipLaunchKernelGGL(k_hash_heads, dim3(grid_for(n)), dim3(TB), 0, s_, shash, n, head);
  if (!launched("heads") || !max_scan(head, runh, n)) return false;
  hipLaunchKernelGGL(k_canon, dim3(grid_for(n)), dim3(TB), 0, s_, V, sidx, runh, n, canon);
  return launched("canon");
}

bool DeviceBuilder::scan64(const uint64_t* v, size_t n, uint64_t*& E) {
  E = alloc<uint64_t>(n);
  return E && exclusive_sum(v, E, n);
}

hvf_status DeviceBuilder::run_paper(Built& B, uint32_t** dbuf, size_t* nwords) {
  const int nd = (int)L.d.size();
  const int nlev = (int)S.lv.size();
  std::vector<DepthState> D(nd);
  for (int i = 1; i < nd; ++i) D[i].ns = L.d[i].cs + L.d[i].w[0];
  if (!validate_codes()) return st_;
  // 1. nodes of every depth (all are stored in this layout); the deepest depth's children
  //    are the codes.
  const int dl = nd - 1;
  uint32_t* code_rank = nullptr;
  if (!structure(D, dl, code_rank)) return st_;
  uint32_t* cpar = nullptr;  // every code's node at the deepest depth (null: the single root)
  {
    DepthState& q = D[dl];
    q.first = alloc<uint32_t>(q.n);
    q.count = alloc<uint32_t>(q.n);
    if (!q.first || !q.count) return st_;
    if (dl == 0) {
      const uint32_t z = 0, nn = (uint32_t)n_;
      if (!hip(hipMemcpyAsync(q.first, &z, sizeof(z), hipMemcpyHostToDevice, s_), "hipMemcpyAsync") ||
          !hip(hipMemcpyAsync(q.count, &nn, sizeof(nn), hipMemcpyHostToDevice, s_), "hipMemcpyAsync") ||
          !hip(hipStreamSynchronize(s_), "hipStreamSynchronize"))
        return st_;
    } else {
      if (!(cpar = alloc<uint32_t>(n_))) return st_;
      if (!hip(hipMemcpyAsync(cpar, code_rank, n_ * sizeof(uint32_t), hipMemcpyDeviceToDevice, s_), "hipMemcpyAsync"))
        return st_;
      hipLaunchKernelGGL(k_decrement, dim3(grid_for(n_)), dim3(TB), 0, s_, cpar, n_);
      hipLaunchKernelGGL(k_child_first, dim3(grid_for(n_)), dim3(TB), 0, s_, cpar, n_, q.first);
      hipLaunchKernelGGL(k_child_count, dim3(grid_for(n_)), dim3(TB), 0, s_, cpar, n_, q.first, q.count);
      if (!launched("code runs")) return st_;
    }
  }
  if (!groups(D, dl)) return st_;
  // 2. octree masks: valid children, and at a level's deepest depth also the leaf bits
  for (int i = dl; i >= 0; --i) {
    const DepthInfo& di = L.d[i];
    if (S.lv[di.level].kind == LK_RAW) continue;
    DepthState& q = D[i];
    if (!(q.masks = alloc<uint32_t>(q.n))) return st_;
    const int deepest = di.j == S.lv[di.level].e[0] - 1;
    if (i < dl)
      hipLaunchKernelGGL(k_masks_children, dim3(grid_for(q.n)), dim3(TB), 0, s_, D[i + 1].keys, q.first, q.count, q.n,
                         deepest, q.masks);
    else
      hipLaunchKernelGGL(k_masks_voxels, dim3(grid_for(n_)), dim3(TB), 0, s_, codes_, code_rank, n_, q.masks);
    if (!launched("masks")) return st_;
  }
  // 3. SVDAG de-duplication, bottom-up. Leaves of the last level are all the same voxel
  //    word: the first of each sub-volume (or of the level) is stored. A leaf above the next
  //    level holds that sub-volume's own pointer and is never merged. Nodes below a
  //    sub-volume root are merged with the first equal node (masks, children's canonical
  //    ids) of their group.
  const bool last_dag = S.lv[nlev - 1].kind == LK_DAG;
  uint32_t* canonL = nullptr;  // last level's leaves (one per code)
  if (last_dag) {
    uint32_t* g = alloc<uint32_t>(n_);
    uint32_t* head = alloc<uint32_t>(n_);
    canonL = alloc<uint32_t>(n_);
    if (!g || !head || !canonL) return st_;
    if (S.wld || dl == 0) {
      if (!hip(hipMemsetAsync(g, 0, n_ * sizeof(uint32_t), s_), "hipMemsetAsync")) return st_;
    } else {
      hipLaunchKernelGGL(k_gather, dim3(grid_for(n_)), dim3(TB), 0, s_, D[dl].group, cpar, n_, g);
    }
    hipLaunchKernelGGL(kp_run_heads, dim3(grid_for(n_)), dim3(TB), 0, s_, g, n_, head);
    if (!launched("leaf heads") || !max_scan(head, canonL, n_)) return st_;
  }
  std::vector<uint32_t*> ident(nd, nullptr);  // iota over a depth (leaves above the next level)
  for (int i = dl; i >= 0; --i) {
    const DepthInfo& di = L.d[i];
    if (S.lv[di.level].kind != LK_DAG) continue;
    DepthState& q = D[i];
    if (!(q.canon = alloc<uint32_t>(q.n))) return st_;
    if (di.j == 0) {
      hipLaunchKernelGGL(k_iota, dim3(grid_for(q.n)), dim3(TB), 0, s_, q.canon, q.n);
      if (!launched("iota")) return st_;
      continue;
    }
    const uint32_t* cid;
    if (i == dl) {
      cid = canonL;
    } else if (L.d[i + 1].level == di.level) {
      cid = D[i + 1].canon;
    } else {
      if (!(ident[i + 1] = alloc<uint32_t>(D[i + 1].n))) return st_;
      hipLaunchKernelGGL(k_iota, dim3(grid_for(D[i + 1].n)), dim3(TB), 0, s_, ident[i + 1], D[i + 1].n);
      if (!launched("iota")) return st_;
      cid = ident[i + 1];
    }
    const DagView V{q.masks, q.first, q.count, cid, S.wld ? nullptr : q.group};
    if (!canon_of(V, q.n, q.canon)) return st_;
  }
  // 4. words: each node's own units and its subtree (bottom-up); the unit words of SVDAG
  //    children and leaves (0 when merged) come first.
  std::vector<uint64_t*> W(nd), EW(nd), own(nd), usz(nd), EU(nd);
  std::vector<uint64_t> stored(nd, 0);
  uint64_t* uszL = nullptr;  // last level's leaf units
  uint64_t* EUL = nullptr;
  uint64_t storedL = 0;
  uint32_t* flag = alloc<uint32_t>(std::max(n_, (size_t)1));
  uint32_t* nst = alloc<uint32_t>(1);
  if (!flag || !nst) return st_;
  auto count_stored = [&](size_t n, uint64_t& out) {
    uint32_t c = 0;
    if (!sum(flag, nst, n) || !fetch(nst, c)) return false;
    out = c;
    return true;
  };
  if (last_dag) {
    if (!(uszL = alloc<uint64_t>(n_))) return st_;
    hipLaunchKernelGGL(kp_unit_sizes, dim3(grid_for(n_)), dim3(TB), 0, s_, canonL, nullptr, n_, uszL, flag);
    if (!launched("leaf sizes") || !count_stored(n_, storedL) || !scan64(uszL, n_, EUL)) return st_;
  }
  for (int i = dl; i >= 0; --i) {
    const DepthInfo& di = L.d[i];
    const int kind = S.lv[di.level].kind == LK_RAW ? 0 : (S.lv[di.level].kind == LK_SVO ? 1 : 2);
    DepthState& q = D[i];
    // this depth's units as children of the depth above: SVDAG nodes below a root, and
    // next-level roots under an SVDAG level's deepest depth (its leaves)
    if (i > 0 && S.lv[L.d[i - 1].level].kind == LK_DAG) {
      const bool leaf = L.d[i - 1].level != di.level;  // one-word leaves, never merged
      if (!(usz[i] = alloc<uint64_t>(q.n))) return st_;
      hipLaunchKernelGGL(kp_unit_sizes, dim3(grid_for(q.n)), dim3(TB), 0, s_, leaf ? nullptr : q.canon,
                         leaf ? nullptr : q.count, q.n, usz[i], flag);
      if (!launched("unit sizes") || !count_stored(q.n, stored[i]) || !scan64(usz[i], q.n, EU[i])) return st_;
    }
    uint64_t* kidw = nullptr;
    uint64_t* ksum = nullptr;
    if (i < dl) {
      if (!(kidw = alloc<uint64_t>(q.n))) return st_;
      hipLaunchKernelGGL(kp_run_sum, dim3(grid_for(q.n)), dim3(TB), 0, s_, W[i + 1], EW[i + 1], q.first, q.count, q.n,
                         kidw);
      if (!launched("subtree sums")) return st_;
    }
    if (kind == 2) {
      if (!(ksum = alloc<uint64_t>(q.n))) return st_;
      const uint64_t* ku = i < dl ? usz[i + 1] : uszL;
      const uint64_t* ke = i < dl ? EU[i + 1] : EUL;
      hipLaunchKernelGGL(kp_run_sum, dim3(grid_for(q.n)), dim3(TB), 0, s_, ku, ke, q.first, q.count, q.n, ksum);
      if (!launched("unit sums")) return st_;
    }
    const int cells = di.w[0] + di.w[1] + di.w[2];
    const uint64_t rawwords = kind == 0 ? (uint64_t)(S.lv[di.level].maxd ? 2 : 1) << cells : 0;
    if (!(own[i] = alloc<uint64_t>(q.n)) || !(W[i] = alloc<uint64_t>(q.n))) return st_;
    hipLaunchKernelGGL(kp_own, dim3(grid_for(q.n)), dim3(TB), 0, s_, kind, di.j == 0 ? 1 : 0, rawwords, q.count, kidw,
                       ksum, q.n, own[i], W[i]);
    if (!launched("own words") || !scan64(W[i], q.n, EW[i])) return st_;
  }
  uint64_t total = 0;
  if (!fetch(W[0], total)) return st_;
  total += 1;  // word 0: the root pointer
  if (total >= (1ull << 32)) return stop(HVF_E_OVERFLOW, "the format exceeds 2^32 words (16 GiB, the paper's limit)");
  // 5. offsets, top-down: subtree starts, own-unit bases, children's units, roots' words
  std::vector<uint64_t*> start(nd), base(nd), uoff(nd), roff(nd);
  uint64_t* loffL = nullptr;
  for (int i = 0; i <= dl; ++i) {
    DepthState& q = D[i];
    if (!(start[i] = alloc<uint64_t>(q.n)) || !(base[i] = alloc<uint64_t>(q.n))) return st_;
    hipLaunchKernelGGL(kp_start, dim3(grid_for(q.n)), dim3(TB), 0, s_, i ? q.parent : nullptr,
                       i ? D[i - 1].first : nullptr, i ? start[i - 1] : nullptr, EW[i], q.n, start[i]);
    hipLaunchKernelGGL(kp_base, dim3(grid_for(q.n)), dim3(TB), 0, s_, start[i], W[i], own[i], q.n, base[i]);
    if (!launched("starts")) return st_;
    if (usz[i]) {
      if (!(uoff[i] = alloc<uint64_t>(q.n))) return st_;
      hipLaunchKernelGGL(kp_unit_off, dim3(grid_for(q.n)), dim3(TB), 0, s_, q.parent, D[i - 1].first, base[i - 1],
                         EU[i], q.n, uoff[i]);
      if (!launched("unit offsets")) return st_;
    }
    const DepthInfo& di = L.d[i];
    if (di.j == 0) {
      const int kind = S.lv[di.level].kind == LK_RAW ? 0 : (S.lv[di.level].kind == LK_SVO ? 1 : 2);
      if (!(roff[i] = alloc<uint64_t>(q.n))) return st_;
      hipLaunchKernelGGL(kp_root_off, dim3(grid_for(q.n)), dim3(TB), 0, s_, kind, base[i], own[i], q.count, q.n,
                         roff[i]);
      if (!launched("root offsets")) return st_;
    }
  }
  if (last_dag) {
    if (!(loffL = alloc<uint64_t>(n_))) return st_;
    hipLaunchKernelGGL(kp_unit_off, dim3(grid_for(n_)), dim3(TB), 0, s_, cpar, D[dl].first, base[dl], EUL, n_, loffL);
    if (!launched("leaf offsets")) return st_;
  }
  // 6. the words. Every write is checked against the buffer's end (a violation would be a
  //    construction error, reported, never a write out of bounds).
  const size_t nw = (size_t)total + HVF_BUFFER_PAD_WORDS;
  uint32_t* werr = alloc<uint32_t>(1);
  if (!werr || !hip(hipMemsetAsync(werr, 0, sizeof(uint32_t), s_), "hipMemsetAsync")) return st_;
  if (!hip(hipMalloc(&buf_, nw * sizeof(uint32_t)), "hipMalloc of the word buffer") ||
      !hip(hipMemsetAsync(buf_, 0, nw * sizeof(uint32_t), s_), "hipMemsetAsync"))
    return st_;
  const uint64_t lim = total;
  for (int i = 0; i <= dl; ++i) {
    const DepthInfo& di = L.d[i];
    const LevelSpec& lv = S.lv[di.level];
    DepthState& q = D[i];
    const bool deepest = lv.kind == LK_RAW || di.j == lv.e[0] - 1;  // children in the next level (or voxels)
    if (lv.kind == LK_RAW) {
      const uint32_t per = lv.maxd ? 2u : 1u;
      if (i < dl) {
        const DepthState& c = D[i + 1];
        hipLaunchKernelGGL(kp_write_raw, dim3(grid_for(c.n)), dim3(TB), 0, s_, c.keys, i == 0 ? nullptr : c.parent,
                           roff[i + 1], c.n, di.w[0], di.w[1], i == 0 ? 1 : 0, per, base[i], lim, werr, buf_);
      } else {
        hipLaunchKernelGGL(kp_write_raw, dim3(grid_for(n_)), dim3(TB), 0, s_, codes_, cpar, nullptr, n_, di.w[0],
                           di.w[1], i == 0 ? 1 : 0, per, base[i], lim, werr, buf_);
      }
      if (!launched("raw cells")) return st_;
      if (lv.maxd) {
        const int cb = di.w[0] + di.w[1] + di.w[2];
        const size_t all = q.n << cb;
        hipLaunchKernelGGL(kp_df_init, dim3(grid_for(all)), dim3(TB), 0, s_, buf_, base[i], q.n, cb, lim, werr);
        int lo = 0;
        for (int a = 0; a < 3; ++a) {
          const uint32_t len = 1u << di.w[a];
          if (len > 1u) {
            const int lb = cb - di.w[a];
            const size_t lines = q.n << lb;
            hipLaunchKernelGGL(kp_df_relax, dim3(grid_for(lines)), dim3(TB), 0, s_, buf_, base[i], lines, lb, cb,
                               len, 1ull << lo, (1ull << lo) - 1ull, lo, lim);
          }
          lo += di.w[a];
        }
        hipLaunchKernelGGL(kp_df_cap, dim3(grid_for(all)), dim3(TB), 0, s_, buf_, base[i], q.n, cb, (uint32_t)lv.maxd,
                           lim);
        if (!launched("distances")) return st_;
      }
    } else if (lv.kind == LK_SVO) {
      const int mode = !deepest ? 0 : (i < dl ? 1 : 2);
      hipLaunchKernelGGL(kp_write_svo, dim3(grid_for(q.n)), dim3(TB), 0, s_, q.first, q.count, q.masks, base[i], q.n,
                         mode, mode == 0 ? base[i + 1] : nullptr, mode == 0 ? D[i + 1].masks : nullptr,
                         mode == 1 ? roff[i + 1] : nullptr, di.j == 0 ? 1 : 0, lim, werr, buf_);
      if (!launched("svo blocks")) return st_;
    } else {
      const uint32_t* kc;
      const uint64_t* ko;
      if (!deepest) {
        kc = D[i + 1].canon;
        ko = uoff[i + 1];
      } else if (i < dl) {
        kc = nullptr;
        ko = uoff[i + 1];
      } else {
        kc = canonL;
        ko = loffL;
      }
      hipLaunchKernelGGL(kp_write_dag, dim3(grid_for(q.n)), dim3(TB), 0, s_, di.j == 0 ? nullptr : q.canon, q.first,
                         q.count, q.masks, di.j == 0 ? roff[i] : uoff[i], q.n, kc, ko, lim, werr, buf_);
      if (deepest && i < dl)
        hipLaunchKernelGGL(kp_write_leaves, dim3(grid_for(D[i + 1].n)), dim3(TB), 0, s_, nullptr, uoff[i + 1],
                           roff[i + 1], D[i + 1].n, lim, werr, buf_);
      if (deepest && i == dl)
        hipLaunchKernelGGL(kp_write_leaves, dim3(grid_for(n_)), dim3(TB), 0, s_, canonL, loffL, nullptr, n_, lim, werr,
                           buf_);
      if (!launched("svdag words")) return st_;
    }
  }
  uint32_t herr = 0;
  uint64_t r0 = 0;
  if (!fetch(werr, herr) || !fetch(roff[0], r0)) return st_;
  if (herr || r0 >= total) return stop(HVF_E_DEVICE, "device construction of the paper's layout: a word fell outside the buffer");
  const uint32_t root = (uint32_t)r0;
  if (!hip(hipMemcpyAsync(buf_, &root, sizeof(uint32_t), hipMemcpyHostToDevice, s_), "hipMemcpyAsync") ||
      !hip(hipStreamSynchronize(s_), "hipStreamSynchronize"))
    return st_;
  // 7. statistics, as the host builder counts them: Raw levels their sub-volumes; SVO levels
  //    their roots and every child entry; SVDAG levels their roots and stored children.
  B.nvox = n_;
  B.level_nodes.assign(nlev, 0);
  for (int i = 0; i <= dl; ++i) {
    const DepthInfo& di = L.d[i];
    const LevelSpec& lv = S.lv[di.level];
    if (lv.kind == LK_RAW || di.j == 0) B.level_nodes[di.level] += D[i].n;
    if (lv.kind == LK_SVO && di.j > 0) B.level_nodes[di.level] += D[i].n;
    if (lv.kind == LK_DAG && di.j > 0) B.level_nodes[di.level] += stored[i];
    const bool deepest = lv.kind != LK_RAW && di.j == lv.e[0] - 1;
    if (deepest && lv.kind == LK_SVO) B.level_nodes[di.level] += i < dl ? D[i + 1].n : n_;
    if (deepest && lv.kind == LK_DAG) B.level_nodes[di.level] += i < dl ? D[i + 1].n : storedL;
  }
  B.depth_nodes.assign(nd, 0);
  B.depth_offset.assign(nd, 0);
  B.depth_words.assign(nd, 0);
  *nwords = (size_t)total;
  *dbuf = buf_;
  buf_ = nullptr;
  return HVF_OK;
}
}  // namespace
}  // namespace hvf

namespace {
hvf_status devbuild_fail(hvf_status s, const std::string& m) {
  hvf_set_error(m);
  return s;
}
}  // namespace

extern "C" hvf_status hvf_build_device(const char* format_spec, const uint64_t* d_morton, size_t n, void* stream,
                                       hvf_volume** out) {
  if (!out) return devbuild_fail(HVF_E_INPUT, "null output handle pointer");
  *out = nullptr;
  hvf::Spec spec;
  std::string err;
  hvf_status st = hvf::parse_spec(format_spec, spec, err);
  if (st != HVF_OK) return devbuild_fail(st, err);
  if (spec.regions && spec.paper)
    return devbuild_fail(HVF_E_UNSUPPORTED, "the paper's word layout is one buffer (no --depth-buffers)");
  if (n && !d_morton) return devbuild_fail(HVF_E_INPUT, "null Morton code array");
  if (n > (size_t)INT_MAX) return devbuild_fail(HVF_E_UNSUPPORTED, "a device construction takes fewer than 2^31 codes");
  hvf_volume* v = new (std::nothrow) hvf_volume();
  if (!v) return devbuild_fail(HVF_E_NOMEM, "host allocation failed");
  v->spec = spec;
  v->layout = spec.paper ? hvf::make_paper_layout(spec) : hvf::make_layout(spec);
  if (n == 0) {
    st = spec.paper ? hvf::build_paper_words(v->spec, v->layout, nullptr, 0, v->built, err)
                    : hvf::build_words(v->spec, v->layout, nullptr, 0, v->built, err);
    if (st == HVF_OK) st = hvf_upload(v, stream);
    if (st != HVF_OK) {
      hvf_free(v);
      return st;
    }
    *out = v;
    return HVF_OK;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    hvf_free(v);
    return devbuild_fail(HVF_E_DEVICE, "hipGetDevice failed");
  }
  uint32_t* dbuf = nullptr;
  size_t nwords = 0;
  {
    hvf::DeviceBuilder b(v->spec, v->layout, d_morton, n, (hipStream_t)stream);
    st = spec.paper ? b.run_paper(v->built, &dbuf, &nwords) : b.run(v->built, &dbuf, &nwords);
    if (st != HVF_OK) {
      const std::string m = b.error();
      hvf_free(v);
      return devbuild_fail(st, m);
    }
  }
  if (v->built.regions) v->spec.regions = true;  // chosen by the builder past 2^32 words
  v->dbuf = dbuf;
  v->device = dev;
  v->host_pending = true;
  v->pending_words = nwords;
  *out = v;
  return HVF_OK;
}
