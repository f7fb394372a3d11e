// Internal declarations shared by the host builder, the C-ABI glue and the HIP kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "hvf.h"

namespace hvf {

// ------------------------------------------------------------------ format spec
enum LevelKind : int { LK_RAW = 0, LK_SVO = 1, LK_DAG = 2 };

struct LevelSpec {
  int kind;
  int e[3];  // log2 cells per axis (SVO/SVDAG: depth L on all three)
};

struct Spec {
  std::vector<LevelSpec> lv;
  bool wld = false;  // whole-level de-duplication of SVDAG nodes (Sec. 4.3)
  int ext[3] = {0, 0, 0};
  std::vector<int> sub;  // sub[k]: log2 side (voxels) of a level-k sub-volume, k >= 1; sub[n] = 0
  std::string text;
};

// Parse "R(4,4,4) G(8) --whole-level-dedup" (table of implemented formats, Sec. 3.2).
hvf_status parse_spec(const char* s, Spec& out, std::string& err);

// ------------------------------------------------------------------ traversal layout
// The traversal walks "node depths": a Raw level is one depth, an SVO/SVDAG level of
// depth L is L depths. Each depth has one node kind (how a child cell is tested and its
// pointer found) and one header kind (how a node at that depth is entered).
enum NodeKind : int {
  NK_RAW_PTR = 0,    // Raw level above the last: one pointer word per cell, 0 = empty
  NK_RAW_BITS = 1,   // last Raw level: one occupancy bit per voxel
  NK_SVO_INNER = 2,  // SVO node whose children are SVO nodes: child = first + 2 * rank
  NK_OCT_PTR = 3,    // child pointer word at base + rank (SVDAG nodes; SVO nodes of the
                     // deepest octree depth above the last level)
  NK_OCT_FINAL = 4   // deepest octree depth of the last level: valid mask = occupancy
};
enum HeaderKind : int {
  HK_RAW = 0,  // base = pointer
  HK_SVO = 1,  // {first child / pointer array, masks}
  HK_DAG = 2   // {masks, child pointers...}: base = pointer + 1
};

struct DepthInfo {
  int level;  // level index
  int j;      // depth inside the level (0 for Raw)
  int nk, hk;
  int cs;     // log2 side (voxels) of this depth's child cells
  int w;      // log2 children per axis (1 for octree nodes; Raw: the level exponent)
};

struct Layout {
  std::vector<DepthInfo> d;
  int top_w[3] = {0, 0, 0};  // per-axis log2 children of the depth-0 node
  bool bits_linear = false;  // final Raw level stored x-fastest (only a non-cubic single level)
};

Layout make_layout(const Spec& s);

// ------------------------------------------------------------------ built word buffer
struct Built {
  std::vector<uint32_t> words;
  std::vector<uint64_t> depth_nodes, depth_offset, depth_words, level_nodes;
  uint64_t nvox = 0;
};

hvf_status build_words(const Spec& s, const Layout& L, const uint64_t* codes, size_t n, Built& out,
                       std::string& err);

// ------------------------------------------------------------------ device descriptor
// Per-depth tables packed 4 bits per depth so that a lane reads its entry with one shift.
struct DevFormat {
  const uint32_t* buf;
  int32_t ext[3];
  int32_t top_w[3];
  int32_t ndepth;
  int32_t bits_linear;
  uint64_t cs_tab, w_tab, nk_tab, hk_tab;
};

DevFormat make_devformat(const Layout& L, const Spec& s, const uint32_t* dbuf);

}  // namespace hvf

// The opaque handle.
struct hvf_volume {
  hvf::Spec spec;
  hvf::Layout layout;
  hvf::Built built;
  uint32_t* dbuf = nullptr;  // device copy of built.words
  int device = -1;
};

// Thread-local error text.
void hvf_set_error(const std::string& s);
