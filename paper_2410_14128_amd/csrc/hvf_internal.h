// Internal declarations shared by the host builder, the C-ABI glue and the HIP kernels.
#pragma once

#include <atomic>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "hvf.h"

namespace hvf {

// ------------------------------------------------------------------ format spec
enum LevelKind : int { LK_RAW = 0, LK_SVO = 1, LK_DAG = 2 };

struct LevelSpec {
  int kind;
  int e[3];      // log2 cells per axis (SVO/SVDAG: depth L on all three)
  int maxd = 0;  // distance-field level D(W,H,D,M): M (>= 1); 0 for a plain Raw level.
                 // A DF level is a Raw level (kind LK_RAW) whose empty cells also carry
                 // their L1 distance to the nearest non-empty cell, capped at M (Sec. 3.3).
};

struct Spec {
  std::vector<LevelSpec> lv;
  bool wld = false;         // whole-level de-duplication of SVDAG nodes (Sec. 4.3)
  bool restart_sv = false;  // restarting sparse-voxel intersection (Sec. 4.3)
  bool paper = false;       // --paper-layout: the paper's word layout with RGBA voxels
  bool regions = false;     // per-depth word regions with region-relative pointers (--depth-buffers,
                            // or chosen by the builder when the format needs 2^32 words or more)
  int ext[3] = {0, 0, 0};
  std::vector<int> sub;  // sub[k]: log2 side (voxels) of a level-k sub-volume, k >= 1; sub[n] = 0
  std::string text;
};

// Parse "R(4,4,4) G(8) --whole-level-dedup" (table of implemented formats, Sec. 3.2).
hvf_status parse_spec(const char* s, Spec& out, std::string& err);

// ------------------------------------------------------------------ traversal layout
// The traversal walks "node depths": a Raw or DF level above the last is one depth, an
// SVO/SVDAG level of depth L is L depths, and the last level, if Raw or DF, is a brick of
// 4x4x4-voxel blocks (one 64-bit occupancy mask each) walked as two depths: the blocks,
// then the voxels of one block (whose mask is held in registers). Each depth has one
// node kind (how a child cell is tested and its pointer found) and one header kind (how
// a node at that depth is entered). Octree kinds are numbered last (>= NK_SVO_INNER).
enum NodeKind : int {
  NK_RAW_PTR = 0,    // Raw level above the last: one pointer word per cell, 0 = empty
  NK_BLOCKS = 1,     // last Raw level, block depth: one 64-bit mask per block, 0 = empty
  NK_CELLS = 2,      // last Raw/DF level, voxel depth: a bit of the block mask (registers)
  NK_DF_PTR = 3,     // DF level above the last: one word per cell, a pointer (< 2^31) if
                     // the cell is non-empty, else DF_EMPTY | capped L1 distance in cells
  NK_DF_BLOCKS = 4,  // last DF level, block depth: 4 words per block (mask lo, mask hi,
                     // capped L1 distance in blocks to the nearest non-empty block, 0)
  NK_SVO_INNER = 5,  // SVO node whose children are SVO nodes: child = first + 2 * rank
  NK_OCT_PTR = 6,    // child pointer word at base + rank (SVDAG nodes; SVO nodes of the
                     // deepest octree depth above the last level)
  NK_OCT_FINAL = 7,  // deepest octree depth of the last level: valid mask = occupancy
  NK_DAG_INNER = 8,  // SVDAG node whose children are SVDAG nodes: a 2-word descriptor
                     // (child pointer, child masks) per valid child at base + 2 * rank
  // Kinds of the paper's own layout (--paper-layout; see make_paper_layout):
  NK_PRAW_VOX = 9,    // last Raw level: one RGBA word per voxel, 0 = empty
  NK_PSVO_TERM = 10,  // last SVO depth above the last level: the child's first word (at
                      // base + 2 * rank) points to the next level's sub-volume
  NK_PDAG_TERM = 11,  // last SVDAG depth above the last level: the child pointer (at
                      // base + rank) points to a word that points to the next sub-volume
  NK_PDF_PTR = 12,    // DF level above the last: (pointer or 0, capped L1 distance) per cell
  NK_PDF_VOX = 13     // last DF level: (RGBA word or 0, capped L1 distance) per voxel
};
constexpr uint32_t DF_EMPTY = 0x80000000u;  // marks an empty cell word of a DF pointer grid
enum HeaderKind : int {
  HK_RAW = 0,       // base = pointer
  HK_SVO = 1,       // {first child / pointer array, masks}
  HK_DAG = 2,       // {masks, child pointers...}: base = pointer + 1
  HK_MASK = 3,      // header read by the parent: a brick block's mask, or the (pointer + 1,
                    // valid) pair of an SVDAG child descriptor
  HK_MASKLOAD = 4   // a one-block brick: load its 64-bit mask at the pointer
};

struct DepthInfo {
  int level;   // level index
  int j;       // depth inside the level (0 for Raw)
  int nk, hk;
  int cs;      // log2 side (voxels) of this depth's child cells
  int w[3];    // log2 children per axis (octree nodes: 1)
  bool arena;  // nodes of this depth are stored (false for the voxel depth of a brick)
};

struct Layout {
  std::vector<DepthInfo> d;
  int brick_b = 2;  // log2 side of a brick block (2 unless a Raw exponent of the last level is < 2)
};

Layout make_layout(const Spec& s);
// Depths walking the paper's own layout (hvf_paper.cpp): one per Raw/DF level, L per
// SVO/SVDAG level, with the NK_P* kinds at the levels' last depths.
Layout make_paper_layout(const Spec& s);

// ------------------------------------------------------------------ built word buffer
struct Built {
  // With per-depth regions (Spec::regions) the nodes of depth d occupy words
  // [depth_offset[d], depth_offset[d + 1]) and every pointer word is an index relative to
  // depth_offset[t] - REGION_BIAS, t the depth it points into, so each region stays below
  // 2^32 words while the whole buffer may be larger (the paper's multiple buffers with
  // indirection, Sec. 3.3: the indirection is the per-depth region table). The bias keeps
  // every pointer above 0, the empty marker.
  bool regions = false;
  std::vector<uint32_t> words;
  std::vector<uint64_t> depth_nodes, depth_offset, depth_words, level_nodes;
  uint64_t nvox = 0;
};

hvf_status build_words(const Spec& s, const Layout& L, const uint64_t* codes, size_t n, Built& out,
                       std::string& err);
// The paper's layout (hvf_paper.cpp); depth_nodes / depth_offset stay zero (its nodes are in
// construction order, not grouped by depth).
hvf_status build_paper_words(const Spec& s, const Layout& L, const uint64_t* codes, size_t n, Built& out,
                             std::string& err);

// ------------------------------------------------------------------ device descriptor
// One packed word per depth: nk | hk << 4 | cs << 8 | wx << 12 | wy << 16 | wz << 20.
// pop_lut: 4 bits per h in [0, 16): the deepest depth whose node side exceeds 2^h, i.e.
// the depth a walk returns to when its position changes in bit h (node sides shrink
// strictly with depth, and every depth below the root is cubic).
// stacked: bit d set = depth d keeps a node-stack slot (slot index = number of stacked
// depths above d); all ones when every depth does. A pop to a depth without a slot restores the deepest stacked ancestor
// and descends again along the current cell position.
// lds_words: leading buffer words each block stages in LDS (0 = none); a multiple of 4.
struct DevFormat {
  const uint32_t* buf;
  int32_t ext[3];
  int32_t ndepth;
  uint64_t pop_lut;
  uint32_t stacked;
  uint32_t nslots;
  uint32_t lds_words;
  uint32_t regions;  // 1: per-depth regions; word index of region d's start in rbase[d]
  uint32_t dinfo[HVF_MAX_DEPTH];
  uint64_t rbase[HVF_MAX_DEPTH];
};

constexpr uint64_t REGION_BIAS = 16;
// Per-depth regions of a built buffer (no-op unless B.regions): rbase[d] = depth_offset[d] - REGION_BIAS.
void set_regions(DevFormat& F, const Built& B);

// Split schedule scratch: survivor counters (one per launch that fills a list, the first
// launch and each restart round), then one survivor list of n entries (8 bytes each), or
// two used in turn when there are restart rounds.
constexpr uint32_t HVF_SPLIT_MAX_ROUNDS = 6;
constexpr size_t HVF_SPLIT_HEAD_WORDS = 8;
inline size_t split_scratch_words(size_t n, uint32_t rounds) {
  return HVF_SPLIT_HEAD_WORDS + (rounds ? 4 : 2) * n;
}

// Largest prefix a schedule may stage in LDS (32 KiB; the node stack takes at most 32 KiB
// more, so a block stays within 64 KiB).
constexpr uint32_t HVF_LDS_PREFIX_MAX_WORDS = 8192;

// Words staged for lds_depths top depths: the start of depth lds_depths (depths are stored
// in order, each 64-byte aligned), or the whole buffer rounded down to 4 words when every
// depth is staged. Returns false if that exceeds HVF_LDS_PREFIX_MAX_WORDS.
bool lds_prefix_words(const Layout& L, const Built& B, int lds_depths, uint32_t* words);

// Check a word buffer read from a file before any kernel walks it: every depth offset is
// inside the buffer and 16-word aligned, and every word index the walk can read from any
// node it can reach (pointers, child descriptors, cells, blocks) is inside the buffer.
// False with a message otherwise.
bool validate_words(const Layout& L, const Built& B, std::string& err);

// Stack-slot mask of a layout: every depth, or with restart-sv only the root depth of each
// level; stack_depth > 0 further keeps only depths < stack_depth (depth 0 always).
uint32_t stacked_mask(const Layout& L, bool restart_sv, int stack_depth);
void set_stacked(DevFormat& F, uint32_t mask);

DevFormat make_devformat(const Layout& L, const Spec& s, const uint32_t* dbuf);

// Compile-time format families: bit k (k < 16) = node kind k may occur, bit 16 + h =
// header kind h may occur. Trace kernels are instantiated per family so code for absent
// kinds is not compiled in; a volume uses the first family that covers its layout.
constexpr uint32_t fam_nk(int k) { return 1u << k; }
constexpr uint32_t fam_hk(int h) { return 1u << (16 + h); }
constexpr uint32_t FAM_DAG_BRICK = fam_nk(NK_DAG_INNER) | fam_nk(NK_OCT_PTR) | fam_nk(NK_BLOCKS) | fam_nk(NK_CELLS) |
                                   fam_hk(HK_DAG) | fam_hk(HK_MASK) | fam_hk(HK_RAW) | fam_hk(HK_MASKLOAD);
constexpr uint32_t FAM_SVO_BRICK = fam_nk(NK_SVO_INNER) | fam_nk(NK_OCT_PTR) | fam_nk(NK_BLOCKS) | fam_nk(NK_CELLS) |
                                   fam_hk(HK_SVO) | fam_hk(HK_MASK) | fam_hk(HK_RAW) | fam_hk(HK_MASKLOAD);
constexpr uint32_t FAM_RAW_BRICK = fam_nk(NK_RAW_PTR) | fam_nk(NK_BLOCKS) | fam_nk(NK_CELLS) | fam_hk(HK_RAW) |
                                   fam_hk(HK_MASK) | fam_hk(HK_MASKLOAD);
constexpr uint32_t FAM_OCTREE = fam_nk(NK_SVO_INNER) | fam_nk(NK_DAG_INNER) | fam_nk(NK_OCT_PTR) |
                                fam_nk(NK_OCT_FINAL) | fam_hk(HK_SVO) | fam_hk(HK_DAG) | fam_hk(HK_MASK);
constexpr uint32_t FAM_RAW_OCTREE = FAM_OCTREE | fam_nk(NK_RAW_PTR) | fam_hk(HK_RAW);
constexpr uint32_t FAM_DF_BRICK = FAM_RAW_BRICK | fam_nk(NK_DF_PTR) | fam_nk(NK_DF_BLOCKS);
constexpr uint32_t FAM_DF_OCTREE = FAM_RAW_OCTREE | fam_nk(NK_DF_PTR);
constexpr uint32_t FAM_ALL = 0x1FFu | (0x1Fu << 16);
constexpr uint32_t FAM_NODF = FAM_ALL & ~(fam_nk(NK_DF_PTR) | fam_nk(NK_DF_BLOCKS));
constexpr uint32_t FAM_BRICK = fam_nk(NK_BLOCKS) | fam_nk(NK_CELLS) | fam_hk(HK_RAW) | fam_hk(HK_MASK) |
                               fam_hk(HK_MASKLOAD);
// SVO and SVDAG levels mixed above a brick.
constexpr uint32_t FAM_OCT_BRICK = FAM_DAG_BRICK | FAM_SVO_BRICK;
// The paper's own layout (--paper-layout): Raw, DF, SVO and SVDAG levels as the paper
// stores them. Binary layouts never need its NK_P* kinds, so they never land here.
constexpr uint32_t FAM_PAPER = fam_nk(NK_RAW_PTR) | fam_nk(NK_PRAW_VOX) | fam_nk(NK_PDF_PTR) | fam_nk(NK_PDF_VOX) |
                               fam_nk(NK_SVO_INNER) | fam_nk(NK_OCT_PTR) | fam_nk(NK_OCT_FINAL) |
                               fam_nk(NK_PSVO_TERM) | fam_nk(NK_PDAG_TERM) | fam_hk(HK_RAW) | fam_hk(HK_SVO) |
                               fam_hk(HK_DAG);
// Kernels for buffers with per-depth regions (Spec::regions): every kind, region-relative reads.
constexpr uint32_t FAM_REGIONS = 1u << 30;
constexpr int FAMILY_REGIONS = 12;  // family index of those kernels (after the FAMILIES table)
constexpr uint32_t FAMILIES[] = {FAM_BRICK,    FAM_DAG_BRICK, FAM_SVO_BRICK, FAM_RAW_BRICK, FAM_OCTREE, FAM_RAW_OCTREE,
                                 FAM_DF_BRICK, FAM_DF_OCTREE, FAM_OCT_BRICK, FAM_NODF,      FAM_PAPER,  FAM_ALL};
constexpr int NUM_FAMILIES = 12;
// Batched launches mixing both layouts.
constexpr uint32_t FAM_ANY = FAM_ALL | FAM_PAPER;
// Families whose kernels take every depth to be cubic (w equal on the three axes: the root
// is an octree level, and levels below the first are cubic), and the one whose depths all
// have w = 1 (octree levels only). family_of assigns them only to layouts that are.
constexpr bool fam_cubic(uint32_t f) {
  return f == FAM_DAG_BRICK || f == FAM_SVO_BRICK || f == FAM_OCTREE || f == FAM_OCT_BRICK;
}
constexpr bool fam_w1(uint32_t f) { return f == FAM_OCTREE; }

// Index into FAMILIES of the first family covering the layout.
int family_of(const Layout& L);
// Family index of a volume: FAMILY_REGIONS for per-depth regions, else family_of(layout); and
// the family's kind-set value.
int volume_family(const Spec& s, const Layout& L);
uint32_t family_value(int family);
// Whether the layout has a distance-field depth.
bool has_df(const Layout& L);
// Kind set of a volume for the batched kernel: 2 in the paper's layout, 1 with a
// distance-field depth, else 0.
inline int batch_kinds(const Spec& s, const Layout& L) { return s.paper ? 2 : (has_df(L) ? 1 : 0); }
// Kernel code of a batched launch: the widest kind set of its volumes (batch_kinds), or,
// when every volume falls in one brick-final family (common_family: that family's index,
// else -1), that family's own kernel: 3 SVDAG over a brick, 4 SVO over a brick, 5 both over
// a brick, 6 Raw over a brick.
// Batches holding a volume with per-depth regions take code 7, the region-aware kernel
// with every node kind.
inline int batch_kernel_code(int kinds, int common_family, bool regions) {
  if (regions) return 7;
  switch (common_family) {
    case 1: return 3;
    case 2: return 4;
    case 8: return 5;
    case 3: return 6;
    default: return kinds;
  }
}

// One batch of the batched launch: a volume and its ray / hit arrays. Rays of all
// batches form one index space; batch b owns indices [first, first + n).
struct BatchItem {
  const uint32_t* buf;
  const void* rays;  // float4 pairs
  void* hits;        // int4
  uint64_t pop_lut;
  uint32_t first;
  uint32_t n;
  int32_t ext[3];
  int32_t ndepth;
  uint32_t stacked;
  uint32_t pad;
  const uint64_t* rtab;  // per-depth region starts on the device (volumes with regions), else null
};
constexpr int HVF_BATCH_MAX_ITEMS = 256;

}  // namespace hvf

// The opaque handle.
struct hvf_volume {
  hvf::Spec spec;
  hvf::Layout layout;
  hvf::Built built;
  uint32_t* dbuf = nullptr;  // device copy of built.words
  int device = -1;
  hvf_schedule sched{0, 16, 8, 0, 4, 0, 0, 0};
  uint32_t* dcounters = nullptr;  // device ray counters for persistent launches (a ring)
  std::atomic<unsigned> counter_next{0};
  // Guards the lazily made device copy and counters against concurrent first traces.
  std::mutex dev_mu;
  // Split schedule on the legacy default stream: one survivor list reused by every call
  // there (that stream orders them), grown on demand, held by split_mu while a call
  // enqueues its kernels. Calls on other streams allocate their own.
  std::mutex split_mu;
  uint32_t* split_buf = nullptr;
  size_t split_words = 0;
  // A volume built on the device keeps built.words empty until a caller reads the host
  // copy (hvf_words, hvf_save); host_words() downloads it then, once, under host_mu.
  mutable std::mutex host_mu;
  bool host_pending = false;
  size_t pending_words = 0;
};

namespace hvf {
// Host copy of the word buffer (downloads it first for a device-built volume).
hvf_status host_words(const hvf_volume* v);
// Number of words of the buffer, whether or not the host copy is present.
size_t word_count(const hvf_volume* v);
}  // namespace hvf

constexpr int HVF_NUM_COUNTERS = 64;
// Zero words allocated after a device word buffer, so 8- and 16-byte reads that start at
// any word of the buffer stay inside the allocation.
constexpr size_t HVF_BUFFER_PAD_WORDS = 4;

namespace hvf {
// A volume with per-depth regions keeps its table of 64-bit region starts (as
// DevFormat::rbase) on the device right after its word buffer and the buffer's spare words,
// at an even word index, for kernels that hold many volumes (batches, the server).
inline size_t region_table_word(size_t nwords) { return (nwords + HVF_BUFFER_PAD_WORDS + 1) & ~(size_t)1; }
// That table's device address, or null (no regions, or not uploaded).
inline const uint64_t* device_region_table(const hvf_volume* v) {
  if (!v->built.regions || !v->dbuf) return nullptr;
  return reinterpret_cast<const uint64_t*>(v->dbuf + region_table_word(word_count(v)));
}
}  // namespace hvf

// Thread-local error text.
void hvf_set_error(const std::string& s);
