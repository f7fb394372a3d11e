// Host side: spec parser, traversal layout and the builder of the GPU word buffer.
//
// Construction follows Sec. 4.1 (and Sec. 5 for Morton order): every level maps the lower
// corner of a sub-volume to its constructed content, recursing into the next level for
// each non-empty cell; empty sub-volumes are represented by 0. SVO children are laid out
// contiguously and found from the valid mask; SVDAG nodes carry one pointer per valid
// child and are de-duplicated per sub-volume or, with --whole-level-dedup, per level
// (Sec. 4.3). The memory layout follows Sec. 3.3 with these deviations, none of which
// changes which voxels are occupied:
//  * the input is binary occupancy, so the last level carries no RGBA words: a last Raw
//    level is a bit brick, stored as 4x4x4-voxel blocks of one 64-bit mask each (blocks
//    x-fastest, bits x-fastest inside a block), and the deepest octree depth of a last
//    SVO/SVDAG level is its valid mask;
//  * a terminating integer below an SVDAG node is stored in the parent's pointer slot
//    instead of a separate one-word leaf node; an SVO node just above the next level
//    points to a packed array of those pointers instead of two-word leaf nodes;
//  * an SVDAG node whose children are SVDAG nodes stores, per valid child, the child's
//    pointer and a copy of the child's mask word, so a descent reads one 8-byte slot;
//  * nodes are grouped by traversal depth (all depth-0 nodes, then depth 1, ...), so the
//    upper levels form one contiguous prefix of the buffer;
//  * a DF level (Sec. 3.3) keeps one word per cell instead of an interleaved pair: a
//    non-empty cell's word is its pointer, an empty cell's word is DF_EMPTY | distance
//    (a non-empty cell's distance is 0 by definition, so nothing is lost). A last DF
//    level is a brick like a last Raw level whose blocks take 4 words: the mask and the
//    capped L1 distance, in blocks, to the nearest non-empty block -- the walk reads one
//    block per step there, so its distances are counted in blocks.
#include <algorithm>
#include <cstring>
#include <unordered_map>
#include <unordered_set>

#include "hvf_internal.h"

namespace hvf {

// ------------------------------------------------------------------ parser
namespace {

bool read_num(const std::string& s, size_t& i, int& v) {
  while (i < s.size() && (s[i] == ' ' || s[i] == '\t')) ++i;
  size_t j = i;
  while (j < s.size() && std::isdigit((unsigned char)s[j])) ++j;
  if (j == i || j - i > 2) return false;
  v = std::atoi(s.substr(i, j - i).c_str());
  i = j;
  while (i < s.size() && (s[i] == ' ' || s[i] == '\t')) ++i;
  return true;
}

}  // namespace

hvf_status parse_spec(const char* text, Spec& out, std::string& err) {
  if (!text) {
    err = "null format spec";
    return HVF_E_INPUT;
  }
  Spec s;
  s.text = text;
  const std::string str(text);
  size_t i = 0;
  while (i < str.size()) {
    char c = str[i];
    if (c == ' ' || c == '\t') {
      ++i;
      continue;
    }
    if (c == '-') {
      size_t j = i;
      while (j < str.size() && str[j] != ' ' && str[j] != '\t') ++j;
      std::string flag = str.substr(i, j - i);
      if (flag == "--whole-level-dedup" || flag == "-whole-level-dedup" || flag == "--wld") {
        s.wld = true;
      } else if (flag == "--restart-sv" || flag == "-restart-sv") {
        s.restart_sv = true;
      } else if (flag == "--paper-layout") {
        s.paper = true;
      } else if (flag == "--depth-buffers") {
        s.regions = true;
      } else {
        err = "unknown flag '" + flag + "'";
        return HVF_E_SPEC;
      }
      i = j;
      continue;
    }
    if (c != 'R' && c != 'S' && c != 'G' && c != 'D') {
      err = std::string("unknown level kind '") + c + "'";
      return HVF_E_SPEC;
    }
    ++i;
    while (i < str.size() && str[i] == ' ') ++i;
    if (i >= str.size() || str[i] != '(') {
      err = "expected '(' after level kind";
      return HVF_E_SPEC;
    }
    ++i;
    std::vector<int> a;
    int v;
    if (!read_num(str, i, v)) {
      err = "expected a number";
      return HVF_E_SPEC;
    }
    a.push_back(v);
    if (i < str.size() && str[i] == '^') {
      ++i;
      int p;
      if (!read_num(str, i, p) || p != 3) {
        err = "only the k^3 shorthand is accepted";
        return HVF_E_SPEC;
      }
      a = {v, v, v};
    }
    while (i < str.size() && str[i] == ',') {
      ++i;
      if (!read_num(str, i, v)) {
        err = "expected a number";
        return HVF_E_SPEC;
      }
      a.push_back(v);
    }
    if (i >= str.size() || str[i] != ')') {
      err = "expected ')'";
      return HVF_E_SPEC;
    }
    ++i;
    LevelSpec L{};
    if (c == 'R') {
      if (a.size() != 3) {
        err = "R(W,H,D) takes three exponents";
        return HVF_E_SPEC;
      }
      L.kind = LK_RAW;
      for (int k = 0; k < 3; ++k) L.e[k] = a[k];
    } else if (c == 'D') {
      if (a.size() != 4 || a[3] < 1) {
        err = "D(W,H,D,M) takes three exponents and a maximum distance M >= 1";
        return HVF_E_SPEC;
      }
      L.kind = LK_RAW;
      for (int k = 0; k < 3; ++k) L.e[k] = a[k];
      L.maxd = a[3];
    } else {
      if (a.size() != 1 || a[0] < 1) {
        err = std::string(1, c) + "(L) takes one depth >= 1";
        return HVF_E_SPEC;
      }
      L.kind = (c == 'S') ? LK_SVO : LK_DAG;
      L.e[0] = L.e[1] = L.e[2] = a[0];
    }
    s.lv.push_back(L);
  }
  if (s.lv.empty()) {
    err = "no levels";
    return HVF_E_SPEC;
  }
  if (s.lv.size() > HVF_MAX_LEVELS) {
    err = "too many levels";
    return HVF_E_SPEC;
  }
  const int n = (int)s.lv.size();
  for (int k = 1; k < n; ++k)
    if (s.lv[k].e[0] != s.lv[k].e[1] || s.lv[k].e[0] != s.lv[k].e[2]) {
      err = "every level below the first must be cubic";
      return HVF_E_SPEC;
    }
  s.sub.assign(n + 1, 0);
  for (int k = n - 1; k >= 1; --k) s.sub[k] = s.sub[k + 1] + s.lv[k].e[0];
  int depths = 0;
  for (int k = 0; k < n; ++k) depths += (s.lv[k].kind == LK_RAW) ? 1 : s.lv[k].e[0];
  if (s.lv[n - 1].kind == LK_RAW) depths += 1;  // a last Raw level is walked as blocks + voxels
  for (int a = 0; a < 3; ++a) {
    s.ext[a] = s.sub[1] + s.lv[0].e[a];
    if (s.ext[a] > 16) {
      err = "volume side above 2^16 voxels";
      return HVF_E_SPEC;
    }
  }
  if (depths > HVF_MAX_DEPTH) {
    err = "more than 16 node depths";
    return HVF_E_SPEC;
  }
  if (s.paper) {
    if (s.restart_sv) {
      err = "--restart-sv is not supported with --paper-layout";
      return HVF_E_UNSUPPORTED;
    }
    if (s.regions) {
      err = "--depth-buffers is not supported with --paper-layout";
      return HVF_E_UNSUPPORTED;
    }
    for (const LevelSpec& L : s.lv)
      if (L.kind == LK_RAW && std::max(L.e[0], std::max(L.e[1], L.e[2])) > 15) {
        err = "--paper-layout walks a Raw level as one depth: at most 2^15 cells per axis";
        return HVF_E_SPEC;
      }
  }
  out = s;
  return HVF_OK;
}

Layout make_layout(const Spec& s) {
  Layout L;
  const int n = (int)s.lv.size();
  for (int k = 0; k < n; ++k) {
    const LevelSpec& lv = s.lv[k];
    const bool last = (k == n - 1);
    const int cs_level = s.sub[k + 1];
    if (lv.kind == LK_RAW && !last) {
      DepthInfo d{};
      d.level = k;
      d.nk = lv.maxd ? NK_DF_PTR : NK_RAW_PTR;
      d.hk = HK_RAW;
      d.cs = cs_level;
      for (int a = 0; a < 3; ++a) d.w[a] = lv.e[a];
      d.arena = true;
      L.d.push_back(d);
    } else if (lv.kind == LK_RAW) {
      // Brick of blocks of side 2^b (b = 2 unless an exponent is smaller).
      const int b = std::min(2, std::min(lv.e[0], std::min(lv.e[1], lv.e[2])));
      L.brick_b = b;
      const int blk[3] = {lv.e[0] - b, lv.e[1] - b, lv.e[2] - b};
      if (blk[0] + blk[1] + blk[2] > 0) {
        DepthInfo d{};
        d.level = k;
        d.nk = lv.maxd ? NK_DF_BLOCKS : NK_BLOCKS;
        d.hk = HK_RAW;
        d.cs = b;
        for (int a = 0; a < 3; ++a) d.w[a] = blk[a];
        d.arena = true;
        L.d.push_back(d);
        DepthInfo c{};
        c.level = k;
        c.j = 1;
        c.nk = NK_CELLS;
        c.hk = HK_MASK;
        c.cs = 0;
        c.w[0] = c.w[1] = c.w[2] = b;
        c.arena = false;
        L.d.push_back(c);
      } else {
        DepthInfo c{};
        c.level = k;
        c.nk = NK_CELLS;
        c.hk = HK_MASKLOAD;
        c.cs = 0;
        c.w[0] = c.w[1] = c.w[2] = b;
        c.arena = true;
        L.d.push_back(c);
      }
    } else {
      const int D = lv.e[0];
      for (int j = 0; j < D; ++j) {
        DepthInfo d{};
        d.level = k;
        d.j = j;
        d.cs = cs_level + (D - 1 - j);
        d.w[0] = d.w[1] = d.w[2] = 1;
        // An SVDAG node below the level's root is entered through its parent's descriptor.
        d.hk = (lv.kind == LK_SVO) ? HK_SVO : (j == 0 ? HK_DAG : HK_MASK);
        if (j < D - 1)
          d.nk = (lv.kind == LK_SVO) ? NK_SVO_INNER : NK_DAG_INNER;
        else
          d.nk = last ? NK_OCT_FINAL : NK_OCT_PTR;
        d.arena = true;
        L.d.push_back(d);
      }
    }
  }
  return L;
}

uint32_t stacked_mask(const Layout& L, bool restart_sv, int stack_depth) {
  uint32_t m = 0;
  for (size_t d = 0; d < L.d.size(); ++d) {
    bool keep = true;
    if (restart_sv && (L.d[d].nk == NK_SVO_INNER || L.d[d].nk == NK_DAG_INNER || L.d[d].nk == NK_OCT_PTR ||
                       L.d[d].nk == NK_OCT_FINAL))
      keep = (L.d[d].j == 0);  // only the root node of an SVO/SVDAG level keeps a slot
    if (stack_depth > 0 && (int)d >= stack_depth) keep = false;
    if (d == 0) keep = true;
    if (keep) m |= 1u << d;
  }
  return m;
}

bool lds_prefix_words(const Layout& L, const Built& B, int lds_depths, uint32_t* words) {
  uint64_t w = 0;
  if (lds_depths > 0 && B.words.size() > 1) {
    if (lds_depths < (int)L.d.size() && lds_depths < (int)B.depth_offset.size())
      w = B.depth_offset[lds_depths];
    else
      w = B.words.size() & ~3ull;
  }
  if (w > HVF_LDS_PREFIX_MAX_WORDS) return false;
  *words = (uint32_t)w;
  return true;
}

namespace {
// Depth-first pass over every node a walk can reach, checking each word index it reads.
struct Validator {
  const Layout& L;
  const std::vector<uint32_t>& w;
  std::vector<uint64_t> rb;  // per-depth region starts (zero: absolute pointers)
  std::unordered_set<uint64_t> seen;
  std::string err;
  uint64_t up(size_t d) const { return d + 1 < rb.size() ? rb[d + 1] : 0; }  // region of depth d + 1
  uint64_t here(size_t d) const { return d < rb.size() ? rb[d] : 0; }        // region of depth d
  bool in(uint64_t ix) {
    if (ix < w.size()) return true;
    err = "word index " + std::to_string(ix) + " past the buffer (" + std::to_string(w.size()) + " words)";
    return false;
  }
  // The node at depth d that the walk enters at pointer ptr; (hb, hv): the header its parent
  // read (HK_MASK depths).
  bool node(size_t d, uint64_t ptr, uint64_t hb, uint32_t hv) {
    if (d >= L.d.size()) {
      err = "a pointer below the last depth";
      return false;
    }
    const DepthInfo& D = L.d[d];
    if (!seen.insert(((uint64_t)d << 40) | ptr).second) return true;
    uint64_t base = ptr;
    uint32_t valid = 0;
    switch (D.hk) {
      case HK_SVO:
        if (!in(ptr + 1)) return false;
        base = w[ptr] + (D.nk == NK_SVO_INNER ? up(d) : here(d));
        valid = w[ptr + 1] & 0xFFu;
        break;
      case HK_DAG:
        if (!in(ptr)) return false;
        base = ptr + 1;
        valid = w[ptr] & 0xFFu;
        break;
      case HK_MASK:
        base = hb;
        valid = hv;
        break;
      case HK_MASKLOAD:
        return in(ptr + 1);
      default:
        break;
    }
    const uint64_t cells = 1ull << (D.w[0] + D.w[1] + D.w[2]);
    uint32_t rank = 0;
    for (uint64_t lin = 0; lin < cells; ++lin) {
      const bool oct = D.nk >= NK_SVO_INNER && D.nk != NK_PRAW_VOX && D.nk != NK_PDF_PTR && D.nk != NK_PDF_VOX;
      if (oct && !((valid >> lin) & 1u)) continue;
      switch (D.nk) {
        case NK_RAW_PTR:
          if (!in(base + lin)) return false;
          if (w[base + lin] && !node(d + 1, up(d) + w[base + lin], 0, 0)) return false;
          break;
        case NK_DF_PTR:
          if (!in(base + lin)) return false;
          if (!(w[base + lin] & DF_EMPTY) && !node(d + 1, up(d) + w[base + lin], 0, 0)) return false;
          break;
        case NK_BLOCKS:
        case NK_PRAW_VOX:
          if (!in(base + (D.nk == NK_BLOCKS ? 2 : 1) * lin + (D.nk == NK_BLOCKS ? 1 : 0))) return false;
          break;
        case NK_DF_BLOCKS:
          if (!in(base + 4 * lin + 3)) return false;
          break;
        case NK_PDF_VOX:
          if (!in(base + 2 * lin + 1)) return false;
          break;
        case NK_PDF_PTR:
          if (!in(base + 2 * lin + 1)) return false;
          if (w[base + 2 * lin] && !node(d + 1, w[base + 2 * lin], 0, 0)) return false;
          break;
        case NK_SVO_INNER:
          if (!node(d + 1, base + 2 * rank, 0, 0)) return false;
          break;
        case NK_OCT_PTR:
          if (!in(base + rank) || !node(d + 1, up(d) + w[base + rank], 0, 0)) return false;
          break;
        case NK_DAG_INNER: {
          if (!in(base + 2 * rank + 1)) return false;
          const uint64_t c = up(d) + w[base + 2 * rank];
          if (!in(c) || !node(d + 1, c, c + 1u, w[base + 2 * rank + 1] & 0xFFu)) return false;
          break;
        }
        case NK_PSVO_TERM:
          if (!in(base + 2 * rank) || !node(d + 1, w[base + 2 * rank], 0, 0)) return false;
          break;
        case NK_PDAG_TERM:
          if (!in(base + rank) || !in(w[base + rank]) || !node(d + 1, w[w[base + rank]], 0, 0)) return false;
          break;
        default:  // NK_CELLS, NK_OCT_FINAL: register tests only
          return true;
      }
      ++rank;
    }
    return true;
  }
};
}  // namespace

bool validate_words(const Layout& L, const Built& B, std::string& err) {
  const uint64_t nw = B.words.size();
  for (uint64_t off : B.depth_offset)
    if (off > nw || (off & 15u)) {
      err = "depth offset " + std::to_string(off) + " is past the buffer or not 16-word aligned";
      return false;
    }
  if (nw == 0) {
    err = "empty word buffer";
    return false;
  }
  Validator v{L, B.words, {}, {}, {}};
  if (B.regions)
    for (uint64_t off : B.depth_offset) v.rb.push_back(off - REGION_BIAS);
  if (B.words[0] != 0 && !v.node(0, (B.regions ? v.rb[0] : 0) + B.words[0], 0, 0)) {
    err = v.err;
    return false;
  }
  return true;
}

void set_stacked(DevFormat& F, uint32_t mask) {
  // Every depth stacked is stored as all ones, which the kernels test for a uniform fast
  // path (slot = depth).
  const uint32_t all = (F.ndepth >= 32) ? 0xFFFFFFFFu : ((1u << F.ndepth) - 1u);
  F.stacked = (mask == all) ? 0xFFFFFFFFu : mask;
  F.nslots = (uint32_t)__builtin_popcount(mask);
}

int volume_family(const Spec& s, const Layout& L) { return s.regions ? FAMILY_REGIONS : family_of(L); }

uint32_t family_value(int family) { return family == FAMILY_REGIONS ? (FAM_ALL | FAM_REGIONS) : FAMILIES[family]; }

void set_regions(DevFormat& F, const Built& B) {
  F.regions = B.regions ? 1u : 0u;
  for (size_t d = 0; d < HVF_MAX_DEPTH; ++d)
    F.rbase[d] = (B.regions && d < B.depth_offset.size()) ? B.depth_offset[d] - REGION_BIAS : 0;
}

int family_of(const Layout& L) {
  uint32_t need = 0;
  bool cubic = true, w1 = true;
  for (const DepthInfo& d : L.d) {
    need |= fam_nk(d.nk) | fam_hk(d.hk);
    cubic = cubic && d.w[0] == d.w[1] && d.w[1] == d.w[2];
    w1 = w1 && d.w[0] == 1 && d.w[1] == 1 && d.w[2] == 1;
  }
  for (int i = 0; i < NUM_FAMILIES; ++i)
    if ((FAMILIES[i] & need) == need && (cubic || !fam_cubic(FAMILIES[i])) && (w1 || !fam_w1(FAMILIES[i]))) return i;
  return NUM_FAMILIES - 1;
}

bool has_df(const Layout& L) {
  for (const DepthInfo& d : L.d)
    if (d.nk == NK_DF_PTR || d.nk == NK_DF_BLOCKS) return true;
  return false;
}

DevFormat make_devformat(const Layout& L, const Spec& s, const uint32_t* dbuf) {
  DevFormat f{};
  f.buf = dbuf;
  for (int a = 0; a < 3; ++a) f.ext[a] = s.ext[a];
  f.ndepth = (int)L.d.size();
  for (size_t i = 0; i < L.d.size() && i < HVF_MAX_DEPTH; ++i) {
    const DepthInfo& d = L.d[i];
    f.dinfo[i] = (uint32_t)(d.nk & 15) | ((uint32_t)(d.hk & 15) << 4) | ((uint32_t)(d.cs & 15) << 8) |
                 ((uint32_t)(d.w[0] & 15) << 12) | ((uint32_t)(d.w[1] & 15) << 16) | ((uint32_t)(d.w[2] & 15) << 20);
  }
  set_stacked(f, stacked_mask(L, s.restart_sv, 0));
  // Depth to return to when the cell position changes in bit h: the deepest depth >= 1
  // whose node side 2^(cs + w) exceeds 2^h, else the root (depth 0).
  for (int h = 0; h < 16; ++h) {
    uint64_t nd = 0;
    for (size_t i = 1; i < L.d.size(); ++i)
      if (L.d[i].cs + L.d[i].w[0] > h) nd = i;
    f.pop_lut |= (nd & 15) << (4 * h);
  }
  return f;
}

// ------------------------------------------------------------------ builder
namespace {

inline uint64_t spread3(uint64_t v) {
  v &= 0x1FFFFFull;
  v = (v | (v << 32)) & 0x1F00000000FFFFull;
  v = (v | (v << 16)) & 0x1F0000FF0000FFull;
  v = (v | (v << 8)) & 0x100F00F00F00F00Full;
  v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}
inline uint64_t compact3(uint64_t v) {
  v &= 0x1249249249249249ull;
  v = (v ^ (v >> 2)) & 0x10C30C30C30C30C3ull;
  v = (v ^ (v >> 4)) & 0x100F00F00F00F00Full;
  v = (v ^ (v >> 8)) & 0x1F0000FF0000FFull;
  v = (v ^ (v >> 16)) & 0x1F00000000FFFFull;
  v = (v ^ (v >> 32)) & 0x1FFFFFull;
  return v;
}
inline uint64_t morton(uint64_t x, uint64_t y, uint64_t z) { return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2); }

struct Overflow {};

// Content-addressed node map for SVDAG de-duplication: key = (depth, node words), where
// child references are already canonical ids; value = node id in that depth's arena.
struct NodeMap {
  std::unordered_map<uint64_t, std::vector<uint32_t>> buckets;
  static uint64_t hash(int depth, const uint32_t* w, size_t n) {
    uint64_t h = 0x9E3779B97F4A7C15ull ^ ((uint64_t)depth << 40) ^ n;
    for (size_t i = 0; i < n; ++i) {
      h ^= w[i] + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
      h *= 0xBF58476D1CE4E5B9ull;
    }
    return h ^ (h >> 31);
  }
};

// Capped L1 distance transform of a 2^wx x 2^wy x 2^wz grid (x fastest): dist[i] =
// min(cap, L1 distance from cell i to the nearest cell with occ set). L1 distance on the
// grid is the length of a shortest path of face-neighbour moves, so a breadth-first search
// from every occupied cell at once, stopped at depth cap, computes it.
void capped_l1(const std::vector<uint8_t>& occ, int wx, int wy, int wz, uint32_t cap, std::vector<uint32_t>& dist) {
  const uint64_t nx = 1ull << wx, ny = 1ull << wy, nz = 1ull << wz, n = nx * ny * nz;
  dist.assign(n, cap);
  std::vector<uint64_t> frontier, next;
  for (uint64_t i = 0; i < n; ++i)
    if (occ[i]) {
      dist[i] = 0;
      frontier.push_back(i);
    }
  for (uint32_t r = 1; r < cap && !frontier.empty(); ++r) {
    next.clear();
    for (uint64_t i : frontier) {
      const uint64_t x = i & (nx - 1), y = (i >> wx) & (ny - 1), z = i >> (wx + wy);
      auto visit = [&](uint64_t j) {
        if (dist[j] > r) {
          dist[j] = r;
          next.push_back(j);
        }
      };
      if (x > 0) visit(i - 1);
      if (x + 1 < nx) visit(i + 1);
      if (y > 0) visit(i - nx);
      if (y + 1 < ny) visit(i + nx);
      if (z > 0) visit(i - nx * ny);
      if (z + 1 < nz) visit(i + nx * ny);
    }
    frontier.swap(next);
  }
}

struct Builder {
  const Spec& S;
  const Layout& L;
  const uint64_t* codes;
  std::vector<std::vector<uint32_t>> arena;  // per depth: node words (child refs as ids)
  std::vector<std::vector<uint32_t>> aux;    // per depth: pointer arrays of SVO nodes
  std::vector<uint64_t> nodes;               // per depth
  std::vector<NodeMap> level_map;            // whole-level maps, per level
  std::vector<int> level_first_depth;
  std::string err;

  Builder(const Spec& s, const Layout& l, const uint64_t* c) : S(s), L(l), codes(c) {
    arena.resize(L.d.size());
    aux.resize(L.d.size());
    nodes.assign(L.d.size(), 0);
    level_map.resize(S.lv.size());
    level_first_depth.assign(S.lv.size(), 0);
    for (int d = (int)L.d.size() - 1; d >= 0; --d) level_first_depth[L.d[d].level] = d;
  }

  // End of the run of codes starting at i that share code >> shift (one aligned cube).
  size_t group_end(size_t i, size_t hi, int shift) const {
    const uint64_t g = codes[i] >> shift;
    if (shift >= 63) return hi;
    return (size_t)(std::lower_bound(codes + i, codes + hi, (g + 1) << shift) - codes);
  }

  // Build the node at depth d whose region has lower corner (x,y,z); codes[lo,hi) lie in
  // it (non-empty). Returns its id (word offset) in arena[d]. map: the SVDAG dedup map
  // in force (per sub-volume or per level), null outside SVDAG levels.
  uint32_t build(int d, uint64_t x, uint64_t y, uint64_t z, size_t lo, size_t hi, NodeMap* map) {
    const DepthInfo& di = L.d[d];
    const LevelSpec& lv = S.lv[di.level];
    const int cs = di.cs;
    std::vector<uint32_t>& A = arena[d];
    if (di.nk == NK_BLOCKS || di.nk == NK_DF_BLOCKS || (di.nk == NK_CELLS && di.hk == HK_MASKLOAD)) {
      // A brick of the last Raw/DF level: blocks of side 2^b, one 64-bit mask each; a DF
      // brick adds per block the capped L1 distance to the nearest non-empty block.
      const int b = L.brick_b;
      const int wx = lv.e[0] - b, wy = lv.e[1] - b;
      const int wz = lv.e[2] - b;
      const uint64_t nblocks = 1ull << (wx + wy + wz);
      const uint64_t stride = (di.nk == NK_DF_BLOCKS) ? 4 : 2;
      if (nblocks * stride >= (1ull << 31)) throw Overflow();
      const uint32_t id = (uint32_t)A.size();
      A.resize(A.size() + stride * nblocks, 0u);
      const uint64_t m = (1ull << b) - 1;
      for (size_t i = lo; i < hi; ++i) {
        const uint64_t vx = compact3(codes[i]) - x, vy = compact3(codes[i] >> 1) - y, vz = compact3(codes[i] >> 2) - z;
        const uint64_t blk = (vx >> b) | ((vy >> b) << wx) | ((vz >> b) << (wx + wy));
        const uint64_t bit = (vx & m) | ((vy & m) << b) | ((vz & m) << (2 * b));
        A[id + stride * blk + (bit >> 5)] |= 1u << (bit & 31);
      }
      if (di.nk == NK_DF_BLOCKS) {
        std::vector<uint8_t> occ(nblocks);
        for (uint64_t k = 0; k < nblocks; ++k) occ[k] = (A[id + 4 * k] | A[id + 4 * k + 1]) != 0u;
        std::vector<uint32_t> dist;
        capped_l1(occ, wx, wy, wz, (uint32_t)lv.maxd, dist);
        for (uint64_t k = 0; k < nblocks; ++k) A[id + 4 * k + 2] = dist[k];
      }
      ++nodes[d];
      return id;
    }
    if (di.nk == NK_RAW_PTR || di.nk == NK_DF_PTR) {
      const int wx = di.w[0], wy = di.w[1], wz = di.w[2];
      const uint64_t cells = 1ull << (wx + wy + wz);
      if (cells >= (1ull << 31)) throw Overflow();
      std::vector<uint32_t> arr(cells, 0u);
      // Non-empty children in Morton order (Sec. 5): each is one run of codes.
      for (size_t a = lo; a < hi;) {
        const size_t b = group_end(a, hi, 3 * cs);
        const uint64_t g = codes[a] >> (3 * cs);
        const uint64_t cx = compact3(g) - (x >> cs), cy = compact3(g >> 1) - (y >> cs), cz = compact3(g >> 2) - (z >> cs);
        uint32_t child = build_root_of_next(d + 1, x + (cx << cs), y + (cy << cs), z + (cz << cs), a, b);
        arr[cx | (cy << wx) | (cz << (wx + wy))] = child + 1;  // id + 1; 0 = empty
        a = b;
      }
      if (di.nk == NK_DF_PTR) {
        std::vector<uint8_t> occ(cells);
        for (uint64_t k = 0; k < cells; ++k) occ[k] = arr[k] != 0u;
        std::vector<uint32_t> dist;
        capped_l1(occ, wx, wy, wz, (uint32_t)lv.maxd, dist);
        for (uint64_t k = 0; k < cells; ++k)
          if (!occ[k]) arr[k] = DF_EMPTY | dist[k];
      }
      const uint32_t id = (uint32_t)A.size();
      A.insert(A.end(), arr.begin(), arr.end());
      ++nodes[d];
      return id;
    }
    // Octree node (SVO or SVDAG) at depth j of its level.
    const bool svo = (lv.kind == LK_SVO);
    uint32_t valid = 0;
    uint32_t kids[8];
    int nk = 0;
    for (size_t a = lo; a < hi;) {
      const size_t b = group_end(a, hi, 3 * cs);
      const int o = (int)((codes[a] >> (3 * cs)) & 7);
      const uint64_t X = x + ((uint64_t)(o & 1) << cs), Y = y + ((uint64_t)((o >> 1) & 1) << cs),
                     Z = z + ((uint64_t)((o >> 2) & 1) << cs);
      valid |= 1u << o;
      if (di.nk != NK_OCT_FINAL) {
        if (di.nk == NK_SVO_INNER || di.nk == NK_DAG_INNER)
          kids[nk++] = build(d + 1, X, Y, Z, a, b, map);
        else
          kids[nk++] = build_root_of_next(d + 1, X, Y, Z, a, b);
      }
      a = b;
    }
    const bool deepest = (di.nk == NK_OCT_FINAL) || !(d + 1 < (int)L.d.size() && L.d[d + 1].level == di.level);
    const uint32_t leafmask = deepest ? valid : 0u;
    const uint32_t masks = valid | (leafmask << 8);
    if (svo) {
      uint32_t w0 = 0;
      if (di.nk == NK_SVO_INNER) {
        w0 = kids[0];  // children are consecutive 2-word nodes in arena[d+1]
      } else if (di.nk == NK_OCT_PTR) {
        w0 = (uint32_t)aux[d].size();
        aux[d].insert(aux[d].end(), kids, kids + nk);
      }
      const uint32_t id = (uint32_t)A.size();
      A.push_back(w0);
      A.push_back(masks);
      ++nodes[d];
      return id;
    }
    // SVDAG: mask word, then per valid child either a (pointer, child masks) descriptor
    // (children in this level) or a pointer (children are next-level roots).
    // De-duplicate, except the root of a sub-volume, which its parent level writes as is.
    uint32_t w[17];
    w[0] = masks;
    size_t len = 1;
    for (int i = 0; i < nk; ++i) {
      w[len++] = kids[i];
      if (di.nk == NK_DAG_INNER) w[len++] = arena[d + 1][kids[i]];  // the child's mask word
    }
    const bool root = (di.j == 0);
    uint64_t h = 0;
    if (!root && map) {
      h = NodeMap::hash(d, w, len);
      auto it = map->buckets.find(h);
      if (it != map->buckets.end())
        for (uint32_t cand : it->second)
          if (cand + len <= A.size() && std::memcmp(&A[cand], w, len * 4) == 0) return cand;
    }
    const uint32_t id = (uint32_t)A.size();
    A.insert(A.end(), w, w + len);
    ++nodes[d];
    if (!root && map) map->buckets[h].push_back(id);
    return id;
  }

  // Build the root node of the level starting at depth d (a sub-volume of that level).
  uint32_t build_root_of_next(int d, uint64_t x, uint64_t y, uint64_t z, size_t lo, size_t hi) {
    const DepthInfo& di = L.d[d];
    if (S.lv[di.level].kind == LK_DAG) {
      if (S.wld) return build(d, x, y, z, lo, hi, &level_map[di.level]);
      NodeMap local;
      return build(d, x, y, z, lo, hi, &local);
    }
    return build(d, x, y, z, lo, hi, nullptr);
  }
};

}  // namespace

hvf_status build_words(const Spec& s, const Layout& L, const uint64_t* codes, size_t n, Built& out,
                       std::string& err) {
  if (n && !codes) {
    err = "null Morton code array";
    return HVF_E_INPUT;
  }
  for (size_t i = 0; i < n; ++i) {
    if (i && codes[i] <= codes[i - 1]) {
      err = "Morton codes must be strictly ascending (index " + std::to_string(i) + ")";
      return HVF_E_INPUT;
    }
    uint64_t x = compact3(codes[i]), y = compact3(codes[i] >> 1), z = compact3(codes[i] >> 2);
    if ((x >> s.ext[0]) || (y >> s.ext[1]) || (z >> s.ext[2]) || (codes[i] >> 63)) {
      err = "Morton code outside the volume (index " + std::to_string(i) + ")";
      return HVF_E_INPUT;
    }
  }
  Built B;
  B.nvox = n;
  const size_t D = L.d.size();
  B.depth_nodes.assign(D, 0);
  B.depth_offset.assign(D, 0);
  B.depth_words.assign(D, 0);
  B.level_nodes.assign(s.lv.size(), 0);
  if (n == 0) {
    B.words.assign(1, 0u);
    out = std::move(B);
    return HVF_OK;
  }
  Builder b(s, L, codes);
  uint32_t root_id;
  try {
    root_id = b.build_root_of_next(0, 0, 0, 0, 0, n);
  } catch (const std::bad_alloc&) {
    err = "host allocation failed while building";
    return HVF_E_NOMEM;
  } catch (const Overflow&) {
    err = "a single node of this format needs 2^31 words or more, beyond 32-bit word offsets";
    return HVF_E_OVERFLOW;
  }
  // Lay the depths out in order, each arena aligned to 64 bytes, SVO pointer arrays
  // right after their depth. Compute sizes before allocating.
  std::vector<uint64_t> base(D), auxb(D);
  uint64_t cur = 1;
  for (size_t d = 0; d < D; ++d) {
    cur = (cur + 15) & ~15ull;
    base[d] = cur;
    cur += b.arena[d].size();
    auxb[d] = cur;
    cur += b.aux[d].size();
  }
  bool df_ptr = false;
  for (const DepthInfo& di : L.d) df_ptr = df_ptr || di.nk == NK_DF_PTR;
  // One buffer addressed by 32-bit pointers while it fits (31 bits below a DF pointer grid,
  // whose cells keep the top bit for empty ones); past that, per-depth regions with
  // region-relative pointers, each region within the same bound.
  bool regions = s.regions;
  if (!regions && cur >= (df_ptr ? (1ull << 31) : (1ull << 32))) regions = true;
  if (regions) {
    for (size_t d = 0; d < D; ++d) {
      const uint64_t size = ((d + 1 < D) ? base[d + 1] : cur) - base[d] + REGION_BIAS;
      const bool below_df = d > 0 && L.d[d - 1].nk == NK_DF_PTR;
      if (size >= (below_df ? (1ull << 31) : (1ull << 32))) {
        err = "format needs " + std::to_string(cur) + " words, and its depth " + std::to_string(d) + " alone " +
              std::to_string(size) + ", beyond " + (below_df ? "31" : "32") + "-bit region-relative pointers";
        return HVF_E_OVERFLOW;
      }
    }
  }
  B.regions = regions;
  try {
    B.words.assign(cur, 0u);
  } catch (const std::bad_alloc&) {
    err = "host allocation failed";
    return HVF_E_NOMEM;
  }
  // Pointers: absolute word indices, or with per-depth regions indices relative to the
  // region of the depth they point into (the next depth's; an SVO node's pointer array
  // lies in its own depth's region).
  B.words[0] = (uint32_t)((regions ? REGION_BIAS : base[0]) + root_id);
  for (size_t d = 0; d < D; ++d) {
    const DepthInfo& di = L.d[d];
    std::vector<uint32_t>& A = b.arena[d];
    uint32_t* dst = B.words.data() + base[d];
    std::memcpy(dst, A.data(), A.size() * 4);
    const uint64_t nb = regions ? REGION_BIAS : ((d + 1 < D) ? base[d + 1] : 0);
    const uint64_t ab = regions ? auxb[d] - base[d] + REGION_BIAS : auxb[d];
    switch (di.nk) {
      case NK_RAW_PTR:
        for (size_t i = 0; i < A.size(); ++i) dst[i] = A[i] ? (uint32_t)(nb + A[i] - 1) : 0u;
        break;
      case NK_DF_PTR:
        for (size_t i = 0; i < A.size(); ++i) dst[i] = (A[i] & DF_EMPTY) ? A[i] : (uint32_t)(nb + A[i] - 1);
        break;
      case NK_SVO_INNER:
        for (size_t i = 0; i < A.size(); i += 2) dst[i] = (uint32_t)(nb + A[i]);
        break;
      case NK_DAG_INNER:
        for (size_t i = 0; i < A.size();) {
          const uint32_t cnt = (uint32_t)__builtin_popcount(A[i] & 0xFFu);
          for (uint32_t k = 0; k < cnt; ++k) dst[i + 1 + 2 * k] = (uint32_t)(nb + A[i + 1 + 2 * k]);
          i += 1 + 2 * cnt;
        }
        break;
      case NK_OCT_PTR:
        if (di.hk == HK_SVO) {
          for (size_t i = 0; i < A.size(); i += 2) dst[i] = (uint32_t)(ab + A[i]);
          uint32_t* ad = B.words.data() + auxb[d];
          for (size_t i = 0; i < b.aux[d].size(); ++i) ad[i] = (uint32_t)(nb + b.aux[d][i]);
        } else {
          for (size_t i = 0; i < A.size();) {
            uint32_t cnt = (uint32_t)__builtin_popcount(A[i] & 0xFFu);
            for (uint32_t k = 1; k <= cnt; ++k) dst[i + k] = (uint32_t)(nb + A[i + k]);
            i += 1 + cnt;
          }
        }
        break;
      default:
        break;  // bit bricks and final octree masks hold no pointers
    }
    B.depth_nodes[d] = b.nodes[d];
    B.depth_offset[d] = base[d];
    B.depth_words[d] = A.size() + b.aux[d].size();
    B.level_nodes[di.level] += b.nodes[d];
  }
  out = std::move(B);
  return HVF_OK;
}

}  // namespace hvf
