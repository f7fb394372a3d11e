// CPU ORACLE for ray intersection through hybrid voxel formats.
//
// TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the benchmark's CPU
// baseline may load this library. It shares no source with the GPU library: its own spec
// parser, its own builder (in the paper's memory layout) and its own tracer.
//
// What it computes (Hybrid Voxel Formats, Sec. 3 and Sec. 4):
//   * build: a hybrid format is a list of levels, each a base format -- Raw R(W,H,D),
//     distance field D(W,H,D,M), SVO S(L) or SVDAG G(L) (Table "Description of
//     Implemented Formats"). A DF level is built like a Raw level, then each cell gets the
//     L1 distance to the nearest non-empty cell of its grid, capped at M, interleaved with
//     the cell's terminating integer (Sec. 3.3, Sec. 4.1). Construction
//     follows Sec. 4.1 and the construct() pseudo-code: each level visits its child
//     sub-volumes in Morton order (Sec. 5), writes every non-empty child sub-volume to the
//     word buffer ("disk") and records its pointer; empty children are 0. SVO nodes are two
//     words (child pointer or terminating integer, then valid|leaf masks); SVDAG nodes are
//     a mask word plus one pointer per valid child, or a single terminating-integer word
//     for a leaf, de-duplicated per sub-volume or, with whole-level de-duplication, per
//     level (Sec. 4.3). Single voxels store RGBA; the input is binary occupancy, so an
//     occupied voxel is 0xFFFFFFFF. The root pointer is written to word 0 (Sec. 4.1).
//     Memory layout: Sec. 3.3 and the layout figure.
//   * trace: root intersection reads word 0 and clips the ray against the root volume;
//     each level visits its non-empty hit children in order of hit time and calls the
//     next level on them, returning at the first single voxel hit (Sec. 4.2 and the
//     intersect() pseudo-code). Raw levels walk their grid with a DDA (Amanatides & Woo);
//     DF levels walk the same DDA but do not check occupancy while the walk stays within
//     the stored distance of the last empty cell they read (Sec. 4.2); SVO/SVDAG levels
//     recurse over octants in entry-time order.
//   * buffers: the paper caps a format at 2^32 words and notes that several buffers with
//     indirection would lift the cap (Sec. 3.3). Past 2^32 words (or with --depth-buffers)
//     each level gets a buffer of its own: a level's node words and in-level pointers live
//     in its buffer, and the terminating integers of its cells and leaves point into the
//     next level's buffer (word 0 of every buffer is reserved, so no pointer is 0, the
//     empty marker). Word 0 of the format, the root pointer, points into level 0's buffer.
//   * flat_dda: the same first-hit query on a dense occupancy bitset (a single Raw level).
//   * brute: the plain definition -- among all occupied voxels, the visited one with the
//     smallest entry time.
//
// Numerics (the paper fixes none; this is the reading both implementations share):
//   inv_a = 1/d_a correctly rounded fp32; an axis is parallel iff inv_a is not finite.
//   Plane time T_a(p) = (float(p) - o_a) * inv_a, two rounded fp32 ops, no contraction.
//   max(a,b) = a<b ? b : a, min(a,b) = b<a ? b : a.
//   Voxel v is visited iff e(v) < x(v) with e = max(t0, max_a T_a(near_a)),
//   x = min(t1, min_a T_a(far_a)) over non-parallel axes; a parallel axis requires
//   v_a == floor(o_a). Result: the visited occupied voxel with least e, t = e.
//   Built with -O2 -ffp-contract=off and without -ffast-math.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

// ------------------------------------------------------------------ format description
struct Level {
  char kind;  // 'R', 'D', 'S', 'G'
  int e[3];   // log2 of the number of cells per axis (S/G: depth L on every axis)
  int M = 0;  // DF: maximum stored L1 distance
};

struct Format {
  std::vector<Level> lv;
  bool wld = false;
  bool split = false;  // one buffer per level (--depth-buffers; also chosen past 2^32 words)
  std::vector<int> sub;  // sub[k]: log2 side of a level-k sub-volume per axis (k >= 1 cubic)
  int ext[3] = {0, 0, 0};
};

std::string g_err;

bool parse_int(const std::string& s, size_t& i, int& v) {
  size_t j = i;
  while (j < s.size() && s[j] == ' ') ++j;
  size_t k = j;
  while (k < s.size() && s[k] >= '0' && s[k] <= '9') ++k;
  if (k == j || k - j > 3) return false;
  v = std::stoi(s.substr(j, k - j));
  while (k < s.size() && s[k] == ' ') ++k;
  i = k;
  return true;
}

bool parse_spec(const char* spec, Format& f) {
  std::string s(spec ? spec : "");
  size_t i = 0;
  f = Format();
  while (i < s.size()) {
    char c = s[i];
    if (c == ' ' || c == '\t') {
      ++i;
      continue;
    }
    if (c == '-') {
      size_t j = i;
      while (j < s.size() && s[j] != ' ') ++j;
      std::string flag = s.substr(i, j - i);
      if (flag == "--whole-level-dedup" || flag == "-whole-level-dedup" || flag == "--wld")
        f.wld = true;
      else if (flag == "--restart-sv" || flag == "-restart-sv")
        ;  // restarting intersection (Sec. 4.3) changes how a tracer revisits nodes, not the result
      else if (flag == "--depth-buffers")
        f.split = true;
      else {
        g_err = "unknown flag " + flag;
        return false;
      }
      i = j;
      continue;
    }
    if (c != 'R' && c != 'D' && c != 'S' && c != 'G') {
      g_err = std::string("unknown level kind '") + c + "'";
      return false;
    }
    ++i;
    while (i < s.size() && s[i] == ' ') ++i;
    if (i >= s.size() || s[i] != '(') {
      g_err = "expected '('";
      return false;
    }
    ++i;
    std::vector<int> args;
    int v;
    if (!parse_int(s, i, v)) {
      g_err = "bad number";
      return false;
    }
    args.push_back(v);
    if (i < s.size() && s[i] == '^') {  // k^3 shorthand
      ++i;
      int p;
      if (!parse_int(s, i, p) || p != 3) {
        g_err = "only ^3 shorthand";
        return false;
      }
      args = {v, v, v};
    }
    while (i < s.size() && s[i] == ',') {
      ++i;
      if (!parse_int(s, i, v)) {
        g_err = "bad number";
        return false;
      }
      args.push_back(v);
    }
    if (i >= s.size() || s[i] != ')') {
      g_err = "expected ')'";
      return false;
    }
    ++i;
    Level L;
    L.kind = c;
    if (c == 'R') {
      if (args.size() != 3) {
        g_err = "R needs 3 exponents";
        return false;
      }
      for (int a = 0; a < 3; ++a) L.e[a] = args[a];
    } else if (c == 'D') {
      if (args.size() != 4 || args[3] < 1) {
        g_err = "D needs 3 exponents and a maximum distance >= 1";
        return false;
      }
      for (int a = 0; a < 3; ++a) L.e[a] = args[a];
      L.M = args[3];
    } else {
      if (args.size() != 1 || args[0] < 1) {
        g_err = "S/G need one depth >= 1";
        return false;
      }
      L.e[0] = L.e[1] = L.e[2] = args[0];
    }
    f.lv.push_back(L);
  }
  if (f.lv.empty()) {
    g_err = "no levels";
    return false;
  }
  int n = (int)f.lv.size();
  // Every level but the highest must be a cube (Sec. 5).
  for (int k = 1; k < n; ++k)
    if (f.lv[k].e[0] != f.lv[k].e[1] || f.lv[k].e[1] != f.lv[k].e[2]) {
      g_err = "lower levels must be cubic";
      return false;
    }
  f.sub.assign(n + 1, 0);
  for (int k = n - 1; k >= 1; --k) f.sub[k] = f.sub[k + 1] + f.lv[k].e[0];
  for (int a = 0; a < 3; ++a) {
    f.ext[a] = f.sub[1] + f.lv[0].e[a];
    if (f.ext[a] > 20) {
      g_err = "extent too large";
      return false;
    }
  }
  return true;
}

// ------------------------------------------------------------------ Morton codes
uint64_t spread3(uint64_t v) {
  uint64_t r = 0;
  for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (3 * b);
  return r;
}
uint64_t compact3(uint64_t v) {
  uint64_t r = 0;
  for (int b = 0; b < 21; ++b) r |= ((v >> (3 * b)) & 1ull) << b;
  return r;
}
uint64_t morton(uint64_t x, uint64_t y, uint64_t z) { return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2); }

// ------------------------------------------------------------------ builder (paper layout)
const uint32_t VOXEL = 0xFFFFFFFFu;  // RGBA of an occupied single voxel

struct VecHash {
  size_t operator()(const std::vector<uint32_t>& v) const {
    uint64_t h = 1469598103934665603ull;
    for (uint32_t w : v) h = (h ^ w) * 1099511628211ull;
    return (size_t)h;
  }
};
using DedupMap = std::unordered_map<std::vector<uint32_t>, uint32_t, VecHash>;

struct Volume {
  Format f;
  std::vector<uint32_t> words;               // one buffer; with split buffers only word 0
  std::vector<std::vector<uint32_t>> level;  // split buffers: level k's buffer
  std::vector<int64_t> node_count;  // per level: nodes / arrays written
  bool overflow = false;
  // The buffer that pointers into level k index.
  const std::vector<uint32_t>& buf(int k) const { return f.split ? level[(size_t)k] : words; }
};

struct Builder {
  Volume& V;
  const uint64_t* codes;
  size_t n;
  std::vector<DedupMap> level_maps;  // whole-level maps (used with --whole-level-dedup)

  Builder(Volume& v, const uint64_t* c, size_t nn) : V(v), codes(c), n(nn) { level_maps.resize(v.f.lv.size()); }

  // Append words of level k; returns their index in the buffer pointers into level k use.
  uint32_t write(int k, const std::vector<uint32_t>& data) {
    std::vector<uint32_t>& B = V.f.split ? V.level[(size_t)k] : V.words;
    uint64_t p = B.size();
    if (p + data.size() >= (1ull << 32)) {
      V.overflow = true;
      return 0;
    }
    B.insert(B.end(), data.begin(), data.end());
    return (uint32_t)p;
  }

  // Code range of the cube of side 2^s at lower corner (x,y,z) (aligned to 2^s).
  void range(uint64_t x, uint64_t y, uint64_t z, int s, size_t lo, size_t hi, size_t& a, size_t& b) const {
    uint64_t c0 = morton(x, y, z), c1 = c0 + (1ull << (3 * s));
    a = std::lower_bound(codes + lo, codes + hi, c0) - codes;
    b = std::lower_bound(codes + a, codes + hi, c1) - codes;
  }

  // The single-voxel construction (the voxelizer's answer for one voxel).
  uint32_t unit(size_t lo, size_t hi) const { return lo < hi ? VOXEL : 0u; }

  // Terminating integer for a cell of level k: a voxel (final level) or a pointer to the
  // written next-level sub-volume; 0 when empty.
  uint32_t cell_term(int k, uint64_t x, uint64_t y, uint64_t z, size_t lo, size_t hi) {
    int nlv = (int)V.f.lv.size();
    if (k == nlv - 1) return unit(lo, hi);
    bool empty;
    std::vector<uint32_t> sub = construct(k + 1, x, y, z, lo, hi, empty);
    if (empty) return 0u;
    if (V.f.lv[k + 1].kind != 'R') V.node_count[k + 1] += 1;  // the sub-volume's root node
    return write(k + 1, sub);
  }

  std::vector<uint32_t> construct(int k, uint64_t x, uint64_t y, uint64_t z, size_t lo, size_t hi, bool& empty) {
    const Level& L = V.f.lv[k];
    int cs = V.f.sub[k + 1];  // log2 cell side of this level
    if (lo == hi) {           // every child sub-volume would be empty
      empty = true;
      return {};
    }
    if (L.kind == 'R' || L.kind == 'D') {
      int64_t nx = 1 << L.e[0], ny = 1 << L.e[1], nz = 1 << L.e[2];
      std::vector<uint32_t> arr((size_t)(nx * ny * nz), 0u);
      empty = true;
      // Children in Morton order of their cell coordinates (Sec. 5).
      int m = std::max(L.e[0], std::max(L.e[1], L.e[2]));
      for (uint64_t c = 0; c < (1ull << (3 * m)); ++c) {
        uint64_t cx = compact3(c), cy = compact3(c >> 1), cz = compact3(c >> 2);
        if ((int64_t)cx >= nx || (int64_t)cy >= ny || (int64_t)cz >= nz) continue;
        uint64_t X = x + (cx << cs), Y = y + (cy << cs), Z = z + (cz << cs);
        size_t a, b;
        range(X, Y, Z, cs, lo, hi, a, b);
        uint32_t t = cell_term(k, X, Y, Z, a, b);
        arr[(size_t)(cx + nx * (cy + ny * cz))] = t;  // flat array, x fastest
        if (t) empty = false;
      }
      V.node_count[k] += empty ? 0 : 1;
      if (L.kind == 'D') return with_distances(arr, nx, ny, nz, L.M);
      return arr;
    }
    DedupMap local;
    DedupMap& map = V.f.wld ? level_maps[k] : local;
    return node(k, 0, x, y, z, lo, hi, map, empty);
  }

  // DF sub-volume: per cell the L1 distance to the nearest non-empty cell of this grid,
  // capped at M, interleaved with the cell's terminating integer. The L1 distance
  // transform is separable: relax d[i] = min(d[i], d[i-1] + 1) forwards then backwards
  // along x, then along y, then along z.
  static std::vector<uint32_t> with_distances(const std::vector<uint32_t>& t, int64_t nx, int64_t ny, int64_t nz,
                                              int M) {
    const int64_t big = nx + ny + nz + 1;
    std::vector<int64_t> d(t.size());
    for (size_t i = 0; i < t.size(); ++i) d[i] = t[i] ? 0 : big;
    auto idx = [&](int64_t x, int64_t y, int64_t z) { return (size_t)(x + nx * (y + ny * z)); };
    for (int64_t z = 0; z < nz; ++z)
      for (int64_t y = 0; y < ny; ++y) {
        for (int64_t x = 1; x < nx; ++x) d[idx(x, y, z)] = std::min(d[idx(x, y, z)], d[idx(x - 1, y, z)] + 1);
        for (int64_t x = nx - 2; x >= 0; --x) d[idx(x, y, z)] = std::min(d[idx(x, y, z)], d[idx(x + 1, y, z)] + 1);
      }
    for (int64_t z = 0; z < nz; ++z)
      for (int64_t x = 0; x < nx; ++x) {
        for (int64_t y = 1; y < ny; ++y) d[idx(x, y, z)] = std::min(d[idx(x, y, z)], d[idx(x, y - 1, z)] + 1);
        for (int64_t y = ny - 2; y >= 0; --y) d[idx(x, y, z)] = std::min(d[idx(x, y, z)], d[idx(x, y + 1, z)] + 1);
      }
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        for (int64_t z = 1; z < nz; ++z) d[idx(x, y, z)] = std::min(d[idx(x, y, z)], d[idx(x, y, z - 1)] + 1);
        for (int64_t z = nz - 2; z >= 0; --z) d[idx(x, y, z)] = std::min(d[idx(x, y, z)], d[idx(x, y, z + 1)] + 1);
      }
    std::vector<uint32_t> out(2 * t.size());
    for (size_t i = 0; i < t.size(); ++i) {
      out[2 * i] = t[i];
      out[2 * i + 1] = (uint32_t)std::min<int64_t>(d[i], M);
    }
    return out;
  }

  // SVO / SVDAG node at depth j (0 = root) of level k covering a cube of side 2^(L-j) cells.
  std::vector<uint32_t> node(int k, int j, uint64_t x, uint64_t y, uint64_t z, size_t lo, size_t hi, DedupMap& map,
                             bool& empty) {
    const Level& L = V.f.lv[k];
    int cs = V.f.sub[k + 1];
    int D = L.e[0];
    if (j == D) {  // leaf: a terminating integer
      uint32_t t = cell_term(k, x, y, z, lo, hi);
      empty = (t == 0);
      if (L.kind == 'S') return {t, 0u};
      return {t};
    }
    int half = cs + (D - j - 1);  // log2 side of a child cube, in voxels
    uint32_t valid = 0, leaf = 0;
    std::vector<std::vector<uint32_t>> kids;
    for (int o = 0; o < 8; ++o) {
      uint64_t X = x + ((uint64_t)(o & 1) << half), Y = y + ((uint64_t)((o >> 1) & 1) << half),
               Z = z + ((uint64_t)((o >> 2) & 1) << half);
      size_t a, b;
      range(X, Y, Z, half, lo, hi, a, b);
      bool ce = true;
      std::vector<uint32_t> child = a < b ? node(k, j + 1, X, Y, Z, a, b, map, ce) : std::vector<uint32_t>();
      if (a == b) ce = true;
      if (ce) continue;
      valid |= 1u << o;
      if (j + 1 == D) leaf |= 1u << o;
      kids.push_back(std::move(child));
    }
    empty = (valid == 0);
    if (empty) return {};
    uint32_t masks = valid | (leaf << 8);
    if (L.kind == 'S') {
      // Children are laid out contiguously, two words each.
      std::vector<uint32_t> block;
      for (auto& c : kids) block.insert(block.end(), c.begin(), c.end());
      uint32_t first = write(k, block);
      V.node_count[k] += (int64_t)kids.size();
      return {first, masks};
    }
    std::vector<uint32_t> nd{masks};
    for (auto& c : kids) {
      auto it = map.find(c);
      uint32_t p;
      if (it != map.end()) {
        p = it->second;
      } else {
        p = write(k, c);
        map.emplace(c, p);
        V.node_count[k] += 1;
      }
      nd.push_back(p);
    }
    return nd;
  }

  void build_root() {
    V.words.assign(1, 0u);  // word 0: root pointer
    V.level.assign(V.f.split ? V.f.lv.size() : 0, std::vector<uint32_t>(1, 0u));  // word 0 of each: reserved
    V.node_count.assign(V.f.lv.size(), 0);
    bool empty;
    std::vector<uint32_t> root = construct(0, 0, 0, 0, 0, n, empty);
    if (!empty) {
      uint32_t p = write(0, root);
      V.words[0] = p;
      if (V.f.lv[0].kind != 'R') V.node_count[0] += 1;
    }
  }
};

// ------------------------------------------------------------------ ray numerics
struct Ray {
  float ox, oy, oz, tmin, dx, dy, dz, tmax;
};
struct Hit {
  int32_t x, y, z;
  float t;
};

inline float fmax_fixed(float a, float b) { return a < b ? b : a; }
inline float fmin_fixed(float a, float b) { return b < a ? b : a; }

struct RayCtx {
  float o[3], inv[3];
  bool par[3], neg[3];
  int vo[3];      // floor(o) on parallel axes
  float t0, t1;   // clipped parameter interval
  int N[3];
  // Plane time of integer plane p on axis a.
  float T(int a, int64_t p) const {
    float fp = (float)p;  // exact for |p| < 2^24
    float diff = fp - o[a];
    return diff * inv[a];
  }
};

// Clip against the whole grid [0,N). Returns false on a miss.
bool setup(const Ray& r, const int ext[3], RayCtx& c) {
  float o[3] = {r.ox, r.oy, r.oz}, d[3] = {r.dx, r.dy, r.dz};
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(o[a]) || !std::isfinite(d[a])) return false;
  bool anyn = false;
  for (int a = 0; a < 3; ++a) {
    c.N[a] = 1 << ext[a];
    c.o[a] = o[a];
    c.inv[a] = 1.0f / d[a];
    c.par[a] = !std::isfinite(c.inv[a]);
    c.neg[a] = d[a] < 0.0f;
    if (c.par[a]) {
      if (!(o[a] >= 0.0f && o[a] < (float)c.N[a])) return false;
      c.vo[a] = (int)std::floor(o[a]);
    } else {
      anyn = true;
    }
  }
  if (!anyn) return false;
  bool first = true;
  float tn = 0, tf = 0;
  for (int a = 0; a < 3; ++a) {
    if (c.par[a]) continue;
    float ne = c.T(a, c.neg[a] ? c.N[a] : 0);
    float fa = c.T(a, c.neg[a] ? 0 : c.N[a]);
    if (first) {
      tn = ne;
      tf = fa;
      first = false;
    } else {
      tn = fmax_fixed(tn, ne);
      tf = fmin_fixed(tf, fa);
    }
  }
  c.t0 = fmax_fixed(r.tmin, tn);
  c.t1 = fmin_fixed(r.tmax, tf);
  return c.t0 < c.t1;
}

// Visit interval of the axis-aligned box [lo, lo + 2^s) (per axis), clipped to [te, tx).
// Returns false if a parallel axis misses it.
bool interval(const RayCtx& c, const int64_t lo[3], int s, float te, float tx, float& e, float& x) {
  e = te;
  x = tx;
  int64_t w = (int64_t)1 << s;
  for (int a = 0; a < 3; ++a) {
    if (c.par[a]) {
      if (c.vo[a] < lo[a] || c.vo[a] >= lo[a] + w) return false;
      continue;
    }
    int64_t nearp = c.neg[a] ? lo[a] + w : lo[a];
    int64_t farp = c.neg[a] ? lo[a] : lo[a] + w;
    e = fmax_fixed(e, c.T(a, nearp));
    x = fmin_fixed(x, c.T(a, farp));
  }
  return true;
}

// ------------------------------------------------------------------ hybrid tracer
struct Tracer {
  const Volume& V;
  const RayCtx& c;

  Hit miss() const { return Hit{-1, -1, -1, INFINITY}; }

  // Level k, sub-volume at pointer p with lower corner lo, entered on [te, tx).
  bool intersect(int k, uint32_t p, const int64_t lo[3], float te, float tx, Hit& h) const {
    const Level& L = V.f.lv[k];
    if (L.kind == 'R' || L.kind == 'D') return raw(k, p, lo, te, tx, h);
    return octree(k, 0, p, lo, te, tx, h);
  }

  bool visit_child(int k, uint32_t term, const int64_t clo[3], float e, float x, Hit& h) const {
    if (term == 0) return false;
    int nlv = (int)V.f.lv.size();
    if (k == nlv - 1) {  // a single voxel
      h = Hit{(int32_t)clo[0], (int32_t)clo[1], (int32_t)clo[2], e};
      return true;
    }
    return intersect(k + 1, term, clo, e, x, h);
  }

  // Raw level: Amanatides & Woo DDA over the cell grid, closed-form plane times,
  // stepping every axis whose next plane is crossed at the same time.
  bool raw(int k, uint32_t p, const int64_t lo[3], float te, float tx, Hit& h) const {
    const Level& L = V.f.lv[k];
    int cs = V.f.sub[k + 1];
    int64_t n[3] = {1 << L.e[0], 1 << L.e[1], 1 << L.e[2]};
    int64_t cell[3];
    for (int a = 0; a < 3; ++a) {
      if (c.par[a]) {
        cell[a] = (c.vo[a] - lo[a]) >> cs;
        continue;
      }
      // The cell containing the ray at time te: the unique i whose slab [near, far) holds te.
      cell[a] = -1;
      for (int64_t i = 0; i < n[a]; ++i) {
        float tl = c.T(a, lo[a] + (i << cs)), th = c.T(a, lo[a] + ((i + 1) << cs));
        bool in = c.neg[a] ? (th <= te && te < tl) : (tl <= te && te < th);
        if (in) {
          cell[a] = i;
          break;
        }
      }
      if (cell[a] < 0) return false;  // te outside this sub-volume along a (empty interval)
    }
    const bool df = (L.kind == 'D');
    const size_t stride = df ? 2 : 1;
    int64_t anchor[3] = {0, 0, 0}, reach = 0;  // DF: cells at L1 distance < reach from anchor are empty
    for (;;) {
      int64_t clo[3] = {lo[0] + (cell[0] << cs), lo[1] + (cell[1] << cs), lo[2] + (cell[2] << cs)};
      const int64_t l1 = std::abs(cell[0] - anchor[0]) + std::abs(cell[1] - anchor[1]) + std::abs(cell[2] - anchor[2]);
      const bool known_empty = df && l1 < reach;
      float e, x;
      if (!known_empty && interval(c, clo, cs, te, tx, e, x) && e < x) {
        const size_t at = (size_t)p + stride * (size_t)(cell[0] + n[0] * (cell[1] + n[1] * cell[2]));
        uint32_t term = V.buf(k)[at];
        if (df && term == 0) {  // march up to this many cells before checking again
          reach = V.buf(k)[at + 1];
          for (int a = 0; a < 3; ++a) anchor[a] = cell[a];
        }
        if (visit_child(k, term, clo, e, x, h)) return true;
      }
      // Next cell: the least far-plane time among non-parallel axes.
      bool first = true;
      float m = 0;
      for (int a = 0; a < 3; ++a) {
        if (c.par[a]) continue;
        float fa = c.T(a, c.neg[a] ? clo[a] : clo[a] + ((int64_t)1 << cs));
        m = first ? fa : fmin_fixed(m, fa);
        first = false;
      }
      if (!(m < tx)) return false;
      for (int a = 0; a < 3; ++a) {
        if (c.par[a]) continue;
        float fa = c.T(a, c.neg[a] ? clo[a] : clo[a] + ((int64_t)1 << cs));
        if (fa == m) {
          cell[a] += c.neg[a] ? -1 : 1;
          if (cell[a] < 0 || cell[a] >= n[a]) return false;
        }
      }
    }
  }

  // SVO/SVDAG node at depth j covering side 2^(D-j) cells at lower corner lo.
  bool octree(int k, int j, uint32_t p, const int64_t lo[3], float te, float tx, Hit& h) const {
    const Level& L = V.f.lv[k];
    int cs = V.f.sub[k + 1];
    int D = L.e[0];
    int half = cs + (D - j - 1);
    const std::vector<uint32_t>& W = V.buf(k);
    uint32_t masks = (L.kind == 'S') ? W[p + 1] : W[p];
    uint32_t valid = masks & 0xFF;
    struct Cand {
      float e, x;
      int o;
    };
    std::vector<Cand> cand;
    for (int o = 0; o < 8; ++o) {
      if (!((valid >> o) & 1)) continue;
      int64_t clo[3] = {lo[0] + ((int64_t)(o & 1) << half), lo[1] + ((int64_t)((o >> 1) & 1) << half),
                        lo[2] + ((int64_t)((o >> 2) & 1) << half)};
      float e, x;
      if (interval(c, clo, half, te, tx, e, x) && e < x) cand.push_back({e, x, o});
    }
    // Ordered hit children: increasing entry time.
    std::stable_sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) { return a.e < b.e; });
    for (const Cand& cd : cand) {
      int o = cd.o;
      int64_t clo[3] = {lo[0] + ((int64_t)(o & 1) << half), lo[1] + ((int64_t)((o >> 1) & 1) << half),
                        lo[2] + ((int64_t)((o >> 2) & 1) << half)};
      uint32_t rank = (uint32_t)__builtin_popcount(valid & ((1u << o) - 1u));
      uint32_t childp;  // address of the child node
      if (L.kind == 'S')
        childp = W[p] + 2 * rank;
      else
        childp = W[p + 1 + rank];
      if (j + 1 == D) {
        uint32_t term = W[childp];  // leaf node: its first word is the terminating integer
        if (visit_child(k, term, clo, cd.e, cd.x, h)) return true;
      } else {
        if (octree(k, j + 1, childp, clo, cd.e, cd.x, h)) return true;
      }
    }
    return false;
  }
};

Hit trace_one(const Volume& V, const Ray& r) {
  Hit miss{-1, -1, -1, INFINITY};
  RayCtx c;
  if (!setup(r, V.f.ext, c)) return miss;
  uint32_t p = V.words[0];
  if (p == 0) return miss;
  Tracer tr{V, c};
  int64_t lo[3] = {0, 0, 0};
  Hit h;
  if (tr.intersect(0, p, lo, c.t0, c.t1, h)) return h;
  return miss;
}

// ------------------------------------------------------------------ decode (losslessness)
struct Decoder {
  const Volume& V;
  std::vector<uint64_t>& out;
  void level(int k, uint32_t p, const int64_t lo[3]) {
    const Level& L = V.f.lv[k];
    int cs = V.f.sub[k + 1];
    if (L.kind == 'R' || L.kind == 'D') {
      int64_t n[3] = {1 << L.e[0], 1 << L.e[1], 1 << L.e[2]};
      const size_t stride = (L.kind == 'D') ? 2 : 1;
      for (int64_t z = 0; z < n[2]; ++z)
        for (int64_t y = 0; y < n[1]; ++y)
          for (int64_t x = 0; x < n[0]; ++x) {
            uint32_t t = V.buf(k)[(size_t)p + stride * (size_t)(x + n[0] * (y + n[1] * z))];
            int64_t clo[3] = {lo[0] + (x << cs), lo[1] + (y << cs), lo[2] + (z << cs)};
            term(k, t, clo);
          }
      return;
    }
    node(k, 0, p, lo);
  }
  void term(int k, uint32_t t, const int64_t clo[3]) {
    if (!t) return;
    if (k == (int)V.f.lv.size() - 1)
      out.push_back(morton(clo[0], clo[1], clo[2]));
    else
      level(k + 1, t, clo);
  }
  void node(int k, int j, uint32_t p, const int64_t lo[3]) {
    const Level& L = V.f.lv[k];
    int cs = V.f.sub[k + 1];
    int D = L.e[0];
    int half = cs + (D - j - 1);
    const std::vector<uint32_t>& W = V.buf(k);
    uint32_t valid = ((L.kind == 'S') ? W[p + 1] : W[p]) & 0xFF;
    for (int o = 0; o < 8; ++o) {
      if (!((valid >> o) & 1)) continue;
      int64_t clo[3] = {lo[0] + ((int64_t)(o & 1) << half), lo[1] + ((int64_t)((o >> 1) & 1) << half),
                        lo[2] + ((int64_t)((o >> 2) & 1) << half)};
      uint32_t rank = (uint32_t)__builtin_popcount(valid & ((1u << o) - 1u));
      uint32_t childp = (L.kind == 'S') ? W[p] + 2 * rank : W[p + 1 + rank];
      if (j + 1 == D)
        term(k, W[childp], clo);
      else
        node(k, j + 1, childp, clo);
    }
  }
};

// ------------------------------------------------------------------ flat DDA and brute force
struct Dense {
  int ext[3];
  std::vector<uint8_t> occ;  // x fastest
};

Hit flat_dda_one(const Dense& G, const Ray& r) {
  Hit miss{-1, -1, -1, INFINITY};
  RayCtx c;
  if (!setup(r, G.ext, c)) return miss;
  int64_t cell[3];
  for (int a = 0; a < 3; ++a) {
    if (c.par[a]) {
      cell[a] = c.vo[a];
      continue;
    }
    cell[a] = -1;
    for (int64_t i = 0; i < c.N[a]; ++i) {
      float tl = c.T(a, i), th = c.T(a, i + 1);
      bool in = c.neg[a] ? (th <= c.t0 && c.t0 < tl) : (tl <= c.t0 && c.t0 < th);
      if (in) {
        cell[a] = i;
        break;
      }
    }
    if (cell[a] < 0) return miss;
  }
  for (;;) {
    float e, x;
    if (interval(c, cell, 0, c.t0, c.t1, e, x) && e < x) {
      if (G.occ[(size_t)(cell[0] + (int64_t)c.N[0] * (cell[1] + (int64_t)c.N[1] * cell[2]))])
        return Hit{(int32_t)cell[0], (int32_t)cell[1], (int32_t)cell[2], e};
    }
    bool first = true;
    float m = 0;
    for (int a = 0; a < 3; ++a) {
      if (c.par[a]) continue;
      float fa = c.T(a, c.neg[a] ? cell[a] : cell[a] + 1);
      m = first ? fa : fmin_fixed(m, fa);
      first = false;
    }
    if (!(m < c.t1)) return miss;
    for (int a = 0; a < 3; ++a) {
      if (c.par[a]) continue;
      float fa = c.T(a, c.neg[a] ? cell[a] : cell[a] + 1);
      if (fa == m) {
        cell[a] += c.neg[a] ? -1 : 1;
        if (cell[a] < 0 || cell[a] >= c.N[a]) return miss;
      }
    }
  }
}

}  // namespace

// ====================================================================== C interface
extern "C" {

const char* orc_last_error() { return g_err.c_str(); }

// Parse a spec; on success writes the per-axis log2 extents and returns the level count,
// else returns -1 (see orc_last_error).
int orc_parse(const char* spec, int* ext3) {
  Format f;
  if (!parse_spec(spec, f)) return -1;
  for (int a = 0; a < 3; ++a) ext3[a] = f.ext[a];
  return (int)f.lv.size();
}

// Build a volume in the paper's layout from strictly ascending Morton codes.
void* orc_build(const char* spec, const uint64_t* codes, int64_t n) {
  Format f;
  if (!parse_spec(spec, f)) return nullptr;
  for (int64_t i = 0; i < n; ++i) {
    if (i && codes[i] <= codes[i - 1]) {
      g_err = "codes not strictly ascending";
      return nullptr;
    }
    uint64_t x = compact3(codes[i]), y = compact3(codes[i] >> 1), z = compact3(codes[i] >> 2);
    if (x >> f.ext[0] || y >> f.ext[1] || z >> f.ext[2] || (codes[i] >> 63)) {
      g_err = "code outside the volume";
      return nullptr;
    }
  }
  auto* V = new Volume();
  V->f = f;
  {
    Builder b(*V, codes, (size_t)n);
    b.build_root();
  }
  if (V->overflow && !V->f.split) {  // past 2^32 words: one buffer per level (Sec. 3.3)
    delete V;
    V = new Volume();
    V->f = f;
    V->f.split = true;
    Builder b(*V, codes, (size_t)n);
    b.build_root();
  }
  if (V->overflow) {
    g_err = "a level of this format exceeds 2^32 words";
    delete V;
    return nullptr;
  }
  return V;
}

void orc_free(void* h) { delete (Volume*)h; }
// Words of the format: word 0, then (split buffers) each level's buffer in level order.
int64_t orc_num_words(void* h) {
  const Volume& V = *(Volume*)h;
  int64_t n = (int64_t)V.words.size();
  for (auto& b : V.level) n += (int64_t)b.size();
  return n;
}
void orc_copy_words(void* h, uint32_t* out) {
  const Volume& V = *(Volume*)h;
  std::memcpy(out, V.words.data(), V.words.size() * 4);
  out += V.words.size();
  for (auto& b : V.level) {
    std::memcpy(out, b.data(), b.size() * 4);
    out += b.size();
  }
}
int orc_split_buffers(void* h) { return ((Volume*)h)->f.split ? 1 : 0; }
int orc_num_levels(void* h) { return (int)((Volume*)h)->f.lv.size(); }
void orc_node_counts(void* h, int64_t* out) {
  auto& v = ((Volume*)h)->node_count;
  for (size_t i = 0; i < v.size(); ++i) out[i] = v[i];
}

// Trace n rays; nthreads >= 1 splits the ray array statically across std::threads.
void orc_trace(void* h, const Ray* rays, int64_t n, Hit* hits, int nthreads) {
  const Volume& V = *(Volume*)h;
  int nt = std::max(1, nthreads);
  if (nt == 1 || n < 1024) {
    for (int64_t i = 0; i < n; ++i) hits[i] = trace_one(V, rays[i]);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t]() {
      int64_t a = n * t / nt, b = n * (t + 1) / nt;
      for (int64_t i = a; i < b; ++i) hits[i] = trace_one(V, rays[i]);
    });
  for (auto& x : th) x.join();
}

// Recover the occupancy set (ascending Morton codes) from the built buffer.
int64_t orc_decode(void* h, uint64_t* out, int64_t cap) {
  const Volume& V = *(Volume*)h;
  std::vector<uint64_t> codes;
  if (V.words[0]) {
    Decoder d{V, codes};
    int64_t lo[3] = {0, 0, 0};
    d.level(0, V.words[0], lo);
  }
  std::sort(codes.begin(), codes.end());
  int64_t m = std::min<int64_t>(cap, (int64_t)codes.size());
  if (out) std::memcpy(out, codes.data(), (size_t)m * 8);
  return (int64_t)codes.size();
}

// First hit on a dense occupancy grid (x fastest, 1 byte per voxel) of extents 2^ext.
void orc_flat_dda(const uint8_t* occ, const int* ext3, const Ray* rays, int64_t n, Hit* hits) {
  Dense G;
  for (int a = 0; a < 3; ++a) G.ext[a] = ext3[a];
  size_t tot = (size_t)1 << (ext3[0] + ext3[1] + ext3[2]);
  G.occ.assign(occ, occ + tot);
  for (int64_t i = 0; i < n; ++i) hits[i] = flat_dda_one(G, rays[i]);
}

// The plain definition: every occupied voxel's visit interval, least entry time wins.
// ties[i] counts voxels that share the winning entry time (0 when the hit is unique).
void orc_brute(const uint64_t* codes, int64_t nc, const int* ext3, const Ray* rays, int64_t n, Hit* hits,
               int32_t* ties) {
  for (int64_t i = 0; i < n; ++i) {
    Hit best{-1, -1, -1, INFINITY};
    int32_t tie = 0;
    RayCtx c;
    if (setup(rays[i], ext3, c)) {
      bool found = false;
      for (int64_t j = 0; j < nc; ++j) {
        int64_t v[3] = {(int64_t)compact3(codes[j]), (int64_t)compact3(codes[j] >> 1),
                        (int64_t)compact3(codes[j] >> 2)};
        float e, x;
        if (!interval(c, v, 0, c.t0, c.t1, e, x) || !(e < x)) continue;
        if (!found || e < best.t) {
          best = Hit{(int32_t)v[0], (int32_t)v[1], (int32_t)v[2], e};
          found = true;
          tie = 0;
        } else if (e == best.t) {
          ++tie;
        }
      }
    }
    hits[i] = best;
    if (ties) ties[i] = tie;
  }
}

}  // extern "C"
