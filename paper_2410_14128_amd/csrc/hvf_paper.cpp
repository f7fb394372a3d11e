// The paper's own memory layout (Sec. 3.3, Sec. 4.1), built on the host for a spec given
// with --paper-layout, and the traversal depths that walk it.
//
// Layout: every level writes its non-empty child sub-volumes first and then itself, in the
// order of the construction pass (Sec. 4.1): a level visits its child cells in Morton order
// of their cell coordinates (Sec. 5) and records for each a terminating integer, 0 when
// empty, else the pointer to the written child sub-volume or, in the last level, the
// voxel's RGBA word. The input is binary occupancy, so an occupied voxel is 0xFFFFFFFF.
//   * Raw level: the 2^(W+H+D) terminating integers, x fastest.
//   * DF level: the same cells, each followed by its L1 distance (in cells of the grid) to
//     the nearest non-empty cell, capped at M.
//   * SVO level: a node is two words, (pointer to its children, masks); the children are
//     written contiguously, two words each; a child at the level's last depth is
//     (terminating integer, 0).
//   * SVDAG level: a node is its masks word followed by one pointer per valid child; a
//     child at the level's last depth is the terminating integer itself (one word).
//     Identical children share one copy: within a sub-volume, or across the whole level
//     with whole-level de-duplication (Sec. 4.3); the first copy written is the one kept.
//   * masks = valid octants | (octants at the last depth) << 8; word 0 holds the pointer to
//     the root sub-volume (0: empty volume).
#include <algorithm>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "hvf_internal.h"

namespace hvf {

Layout make_paper_layout(const Spec& s) {
  Layout L;
  const int n = (int)s.lv.size();
  for (int k = 0; k < n; ++k) {
    const LevelSpec& lv = s.lv[k];
    const bool last = (k == n - 1);
    const int cs_level = s.sub[k + 1];
    if (lv.kind == LK_RAW) {
      DepthInfo d{};
      d.level = k;
      d.nk = lv.maxd ? (last ? NK_PDF_VOX : NK_PDF_PTR) : (last ? NK_PRAW_VOX : NK_RAW_PTR);
      d.hk = HK_RAW;
      d.cs = cs_level;
      for (int a = 0; a < 3; ++a) d.w[a] = lv.e[a];
      d.arena = true;
      L.d.push_back(d);
      continue;
    }
    const int D = lv.e[0];
    for (int j = 0; j < D; ++j) {
      DepthInfo d{};
      d.level = k;
      d.j = j;
      d.cs = cs_level + (D - 1 - j);
      d.w[0] = d.w[1] = d.w[2] = 1;
      d.hk = (lv.kind == LK_SVO) ? HK_SVO : HK_DAG;
      if (j < D - 1)
        d.nk = (lv.kind == LK_SVO) ? NK_SVO_INNER : NK_OCT_PTR;
      else
        d.nk = last ? NK_OCT_FINAL : (lv.kind == LK_SVO ? NK_PSVO_TERM : NK_PDAG_TERM);
      d.arena = true;
      L.d.push_back(d);
    }
  }
  return L;
}

namespace {

constexpr uint32_t RGBA_VOXEL = 0xFFFFFFFFu;

// Bits 0..20 of v moved to bits 0, 3, 6, ... (and back): the usual mask-and-shift
// interleave for 3-D Morton codes.
inline uint64_t spread(uint64_t v) {
  v &= 0x1FFFFFull;
  v = (v | (v << 32)) & 0x1F00000000FFFFull;
  v = (v | (v << 16)) & 0x1F0000FF0000FFull;
  v = (v | (v << 8)) & 0x100F00F00F00F00Full;
  v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}
inline uint64_t unspread(uint64_t v) {
  v &= 0x1249249249249249ull;
  v = (v ^ (v >> 2)) & 0x10C30C30C30C30C3ull;
  v = (v ^ (v >> 4)) & 0x100F00F00F00F00Full;
  v = (v ^ (v >> 8)) & 0x1F0000FF0000FFull;
  v = (v ^ (v >> 16)) & 0x1F00000000FFFFull;
  v = (v ^ (v >> 32)) & 0x1FFFFFull;
  return v;
}

struct WordsHash {
  size_t operator()(const std::vector<uint32_t>& w) const {
    uint64_t h = 0x9E3779B97F4A7C15ull ^ w.size();
    for (uint32_t x : w) h = (h ^ x) * 0xBF58476D1CE4E5B9ull + (h >> 29);
    return (size_t)h;
  }
};
using Shared = std::unordered_map<std::vector<uint32_t>, uint32_t, WordsHash>;

struct TooBig {};

class PaperBuilder {
 public:
  PaperBuilder(const Spec& s, const uint64_t* codes, size_t n, Built& out)
      : S(s), C(codes), N(n), B(out), level_shared(s.lv.size()) {}

  void run() {
    B.words.assign(1, 0u);
    B.level_nodes.assign(S.lv.size(), 0);
    bool empty = true;
    std::vector<uint32_t> root = level(0, 0, 0, 0, 0, N, empty);
    if (!empty) {
      if (S.lv[0].kind != LK_RAW) ++B.level_nodes[0];
      B.words[0] = put(root);
    }
  }

 private:
  const Spec& S;
  const uint64_t* C;
  size_t N;
  Built& B;
  std::vector<Shared> level_shared;  // whole-level de-duplication maps

  uint32_t put(const std::vector<uint32_t>& w) {
    const uint64_t at = B.words.size();
    if (at + w.size() >= (1ull << 32)) throw TooBig{};
    B.words.insert(B.words.end(), w.begin(), w.end());
    return (uint32_t)at;
  }

  // Codes of the aligned cube of side 2^s at (x, y, z), within [lo, hi).
  void cube(uint64_t x, uint64_t y, uint64_t z, int s, size_t lo, size_t hi, size_t& a, size_t& b) const {
    const uint64_t c0 = spread(x) | (spread(y) << 1) | (spread(z) << 2);
    const uint64_t c1 = c0 + (1ull << (3 * s));
    a = (size_t)(std::lower_bound(C + lo, C + hi, c0) - C);
    b = (size_t)(std::lower_bound(C + a, C + hi, c1) - C);
  }

  // Terminating integer of a child cell of level k (a cube of side 2^sub[k+1]).
  uint32_t term(int k, uint64_t x, uint64_t y, uint64_t z, size_t lo, size_t hi) {
    if (lo == hi) return 0u;
    if (k + 1 == (int)S.lv.size()) {
      ++B.nvox;
      return RGBA_VOXEL;
    }
    bool empty = true;
    std::vector<uint32_t> sub = level(k + 1, x, y, z, lo, hi, empty);
    if (empty) return 0u;
    if (S.lv[k + 1].kind != LK_RAW) ++B.level_nodes[k + 1];  // the sub-volume's root node
    return put(sub);
  }

  // Words of the level-k sub-volume at (x, y, z) (side 2^sub[k]); empty if it holds nothing.
  std::vector<uint32_t> level(int k, uint64_t x, uint64_t y, uint64_t z, size_t lo, size_t hi, bool& empty) {
    empty = true;
    if (lo == hi) return {};
    const LevelSpec& lv = S.lv[k];
    const int cs = S.sub[k + 1];
    if (lv.kind == LK_RAW) {
      const uint64_t nx = 1ull << lv.e[0], ny = 1ull << lv.e[1], nz = 1ull << lv.e[2];
      std::vector<uint32_t> cells(nx * ny * nz, 0u);
      const int m = std::max(lv.e[0], std::max(lv.e[1], lv.e[2]));
      // Child cells in Morton order. The sub-volume is aligned to its side, so cell c holds
      // the codes [c0 + c 8^cs, c0 + (c + 1) 8^cs): the cells' code ranges follow one another,
      // and a cursor over the sorted codes finds each in turn (an empty cell in O(1)).
      const uint64_t c0 = spread(x) | (spread(y) << 1) | (spread(z) << 2);
      size_t cur = lo;
      for (uint64_t c = 0; c < (1ull << (3 * m)) && cur < hi; ++c) {
        const uint64_t end = c0 + ((c + 1) << (3 * cs));
        if (C[cur] >= end) continue;  // no code in this cell
        const uint64_t cx = unspread(c), cy = unspread(c >> 1), cz = unspread(c >> 2);
        const size_t a = cur, b = (size_t)(std::lower_bound(C + cur, C + hi, end) - C);
        cur = b;
        if (cx >= nx || cy >= ny || cz >= nz) continue;  // outside a non-cubic grid: holds no code
        const uint32_t t = term(k, x + (cx << cs), y + (cy << cs), z + (cz << cs), a, b);
        cells[cx + nx * (cy + ny * cz)] = t;
        if (t) empty = false;
      }
      if (!empty) ++B.level_nodes[k];
      if (!lv.maxd || empty) return cells;
      return with_distance(cells, (int64_t)nx, (int64_t)ny, (int64_t)nz, (uint32_t)lv.maxd);
    }
    Shared own;
    Shared& shared = S.wld ? level_shared[k] : own;
    return node(k, 0, x, y, z, lo, hi, shared, empty);
  }

  // Interleave each cell with its capped L1 distance to the nearest non-empty cell. The
  // distance is the minimum over non-empty cells of |dx| + |dy| + |dz|; it separates into
  // three one-axis passes of d = min(d, neighbour + 1), each forwards then backwards.
  static std::vector<uint32_t> with_distance(const std::vector<uint32_t>& cells, int64_t nx, int64_t ny, int64_t nz,
                                             uint32_t cap) {
    const int32_t far = (int32_t)(nx + ny + nz);  // above any L1 distance in the grid (sides <= 2^15)
    std::vector<int32_t> d(cells.size());
    for (size_t i = 0; i < cells.size(); ++i) d[i] = cells[i] ? 0 : far;
    const int64_t stride[3] = {1, nx, nx * ny}, len[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
      const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
      for (int64_t u = 0; u < len[b1]; ++u)
        for (int64_t v = 0; v < len[b2]; ++v) {
          const int64_t base = u * stride[b1] + v * stride[b2];
          for (int64_t i = 1; i < len[a]; ++i) {
            int32_t& c = d[base + i * stride[a]];
            c = std::min(c, d[base + (i - 1) * stride[a]] + 1);
          }
          for (int64_t i = len[a] - 2; i >= 0; --i) {
            int32_t& c = d[base + i * stride[a]];
            c = std::min(c, d[base + (i + 1) * stride[a]] + 1);
          }
        }
    }
    std::vector<uint32_t> out(2 * cells.size());
    for (size_t i = 0; i < cells.size(); ++i) {
      out[2 * i] = cells[i];
      out[2 * i + 1] = std::min<uint32_t>((uint32_t)d[i], cap);
    }
    return out;
  }

  // Node at depth j of an SVO/SVDAG level k, a cube of side 2^(sub[k+1] + D - j).
  std::vector<uint32_t> node(int k, int j, uint64_t x, uint64_t y, uint64_t z, size_t lo, size_t hi, Shared& shared,
                             bool& empty) {
    const LevelSpec& lv = S.lv[k];
    const int D = lv.e[0];
    if (j == D) {
      const uint32_t t = term(k, x, y, z, lo, hi);
      empty = t == 0u;
      if (lv.kind == LK_SVO) return {t, 0u};
      return {t};
    }
    const int half = S.sub[k + 1] + (D - j - 1);
    uint32_t valid = 0;
    std::vector<std::vector<uint32_t>> kids;
    for (int o = 0; o < 8; ++o) {
      const uint64_t cx = x + ((uint64_t)(o & 1) << half), cy = y + ((uint64_t)((o >> 1) & 1) << half),
                     cz = z + ((uint64_t)((o >> 2) & 1) << half);
      size_t a, b;
      cube(cx, cy, cz, half, lo, hi, a, b);
      if (a == b) continue;
      bool ce = true;
      std::vector<uint32_t> kid = node(k, j + 1, cx, cy, cz, a, b, shared, ce);
      if (ce) continue;
      valid |= 1u << o;
      kids.push_back(std::move(kid));
    }
    empty = valid == 0u;
    if (empty) return {};
    const uint32_t masks = valid | ((j + 1 == D ? valid : 0u) << 8);
    if (lv.kind == LK_SVO) {
      std::vector<uint32_t> block;
      for (const auto& c : kids) block.insert(block.end(), c.begin(), c.end());
      B.level_nodes[k] += kids.size();
      return {put(block), masks};
    }
    std::vector<uint32_t> out{masks};
    for (const auto& c : kids) {
      auto it = shared.find(c);
      if (it == shared.end()) {
        it = shared.emplace(c, put(c)).first;
        ++B.level_nodes[k];
      }
      out.push_back(it->second);
    }
    return out;
  }
};

}  // namespace

hvf_status build_paper_words(const Spec& s, const Layout& L, const uint64_t* codes, size_t n, Built& out,
                             std::string& err) {
  if (n && !codes) {
    err = "null Morton code array";
    return HVF_E_INPUT;
  }
  for (size_t i = 0; i < n; ++i) {
    if (i && codes[i] <= codes[i - 1]) {
      err = "Morton codes must be strictly increasing";
      return HVF_E_INPUT;
    }
    const uint64_t x = unspread(codes[i]), y = unspread(codes[i] >> 1), z = unspread(codes[i] >> 2);
    if ((codes[i] >> 63) || (x >> s.ext[0]) || (y >> s.ext[1]) || (z >> s.ext[2])) {
      err = "Morton code outside the volume";
      return HVF_E_INPUT;
    }
  }
  out = Built{};
  try {
    PaperBuilder(s, codes, n, out).run();
  } catch (const TooBig&) {
    out = Built{};
    err = "the format exceeds 2^32 words (16 GiB, the paper's limit)";
    return HVF_E_OVERFLOW;
  } catch (const std::bad_alloc&) {
    out = Built{};
    err = "host allocation failed";
    return HVF_E_NOMEM;
  }
  // Nodes are not grouped by depth in this layout: no per-depth ranges.
  out.depth_nodes.assign(L.d.size(), 0);
  out.depth_offset.assign(L.d.size(), 0);
  out.depth_words.assign(L.d.size(), 0);
  return HVF_OK;
}

}  // namespace hvf
