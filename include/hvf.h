/*
 * hvf.h -- ray intersection through hybrid voxel formats on AMD Instinct MI355X (gfx950).
 *
 * A hybrid voxel format is an ordered list of levels, each a base format: a Raw grid
 * R(W,H,D) of 2^W x 2^H x 2^D cells, a sparse voxel octree S(L) or a sparse voxel DAG
 * G(L) of depth L (Hybrid Voxel Formats, Sec. 3.1-3.2 and the table of implemented
 * formats). A cell of an upper level is a sub-volume stored in the next level's format;
 * a cell of the last level is a single voxel. Every level below the first must be a
 * cube (Sec. 5). The whole format lives in one buffer of 32-bit words whose word 0
 * holds the root pointer (Sec. 3.3, Sec. 4.1); this limits a format to 2^32 words.
 *
 * The query (Sec. 4.2): for each ray, the first occupied voxel along it.
 *
 * Coordinates are in finest-voxel units: the volume is [0,Nx) x [0,Ny) x [0,Nz) and voxel
 * (x,y,z) is the box [x,x+1) x [y,y+1) x [z,z+1). A ray is o + t*d for t in [tmin, tmax].
 * Numerics, shared bit-for-bit by every entry point: inv_a = 1/d_a (fp32, correctly
 * rounded); an axis with a non-finite inv_a is parallel; the crossing time of integer
 * plane p is T_a(p) = (float(p) - o_a) * inv_a (two rounded fp32 ops, never fused);
 * max(a,b) = a<b ? b : a and min(a,b) = b<a ? b : a. The ray is clipped to
 * [t0, t1) = [max(tmin, entry), min(tmax, exit)). Voxel v is visited iff
 * e(v) < x(v), where e(v) = max(t0, max_a T_a(near_a)) and x(v) = min(t1, min_a T_a(far_a))
 * over non-parallel axes, and a parallel axis needs v_a == floor(o_a). The result is the
 * visited occupied voxel of least e(v), reported with t = e(v). Rays with a NaN or
 * infinite origin or direction component, or a zero direction, miss.
 *
 * Errors: every hvf_status-returning call returns HVF_OK or an error code and leaves its
 * out-parameters untouched on error; hvf_last_error() gives a thread-local message.
 */
#ifndef HVF_H
#define HVF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One ray, 32 bytes, in grid units. tmax may be +inf. */
typedef struct hvf_ray {
  float ox, oy, oz, tmin;
  float dx, dy, dz, tmax;
} hvf_ray;

/* One result, 16 bytes. Hit: voxel (x,y,z) >= 0 and its entry time t.
 * Miss: x = y = z = -1, t = +inf. The hit flag is (x >= 0). */
typedef struct hvf_hit {
  int32_t x, y, z;
  float t;
} hvf_hit;

typedef enum hvf_status {
  HVF_OK = 0,
  HVF_E_SPEC = 1,        /* malformed format spec, or a non-cubic level below the first */
  HVF_E_INPUT = 2,       /* null pointer, codes not strictly ascending or outside the volume */
  HVF_E_OVERFLOW = 3,    /* the built format would need 2^32 words or more */
  HVF_E_NOMEM = 4,       /* host or device allocation failed, or a memory budget is exceeded */
  HVF_E_DEVICE = 5,      /* a HIP runtime error; the message names it */
  HVF_E_UNSUPPORTED = 6, /* a valid request the library does not implement */
  HVF_E_STATE = 7        /* call not valid in the object's current state */
} hvf_status;

typedef struct hvf_volume hvf_volume; /* opaque; immutable once built */

#define HVF_MAX_LEVELS 8
#define HVF_MAX_DEPTH 16

/* Summary of a built volume. Level kinds: 'R', 'D', 'S', 'G'. */
typedef struct hvf_info {
  int32_t num_levels;
  char kinds[HVF_MAX_LEVELS];
  int32_t level_exp[HVF_MAX_LEVELS][3]; /* log2 cells per axis of each level */
  int32_t extent_log2[3];               /* log2 voxels per axis of the whole volume */
  int32_t whole_level_dedup;
  int32_t num_depths;                   /* node depths of the traversal (Raw: 1, S/G(L): L) */
  uint64_t num_words;                   /* words in the buffer, including word 0 */
  uint64_t level_nodes[HVF_MAX_LEVELS]; /* nodes (octree levels) or arrays (Raw) per level */
  uint64_t depth_nodes[HVF_MAX_DEPTH];
  uint64_t depth_offset[HVF_MAX_DEPTH]; /* first word of each depth: depths are stored in order */
  uint64_t num_voxels;                  /* occupied voxels */
  int32_t level_maxdist[HVF_MAX_LEVELS]; /* DF levels: the maximum stored distance M; else 0 */
  uint32_t kernel_family;               /* template argument of the trace kernels this volume
                                           launches (node/header kinds compiled in) */
  int32_t paper_layout;                 /* 1: built with --paper-layout (the paper's word
                                           layout, Sec. 3.3); 0: the library's own layout */
  int32_t depth_buffers;                /* 1: per-depth regions: the words of depth d are
                                           [depth_offset[d], depth_offset[d + 1]) and every
                                           pointer word p to a node of depth t stands for
                                           word depth_offset[t] - 16 + p (0 stays "empty") */
} hvf_info;

/* How a trace is scheduled on the device. Results never depend on it.
 * persistent = 0: one lane per ray, one launch-sized grid.
 * persistent = 1: a grid sized to the device (at most blocks_per_cu 256-thread blocks per
 *   CU when blocks_per_cu > 0); each wave refills its idle lanes from a global ray counter
 *   whenever at least `refill` of its 64 lanes are idle, checking after every `inner`
 *   traversal steps.
 * sort = 1: trace rays in the order of a coherence key (origin cell of side 2^sort_bits
 *   voxels in Morton order, then direction octant) computed and sorted on the device;
 *   results are still written at each ray's own index.
 * split = K > 0 (a power of two, 2..64; needs persistent = 0 and sort = 0): every ray walks
 *   at most split_budget steps; a ray still walking then has the rest of its interval,
 *   [t, t1), cut into K segments that K lanes walk side by side from the root in a second
 *   launch, and its result is that of the first segment with one. K is an upper bound:
 *   the second launch halves it until the survivors' segments fit its grid's lanes. This shortens the few
 *   long walks that otherwise keep a launch's last waves busy. With split_rounds = R > 0,
 *   R restart rounds run in between: the rays still walking restart from the root at
 *   their t, packed densely, for split_budget, 2 split_budget, ... 2^(R-1) split_budget
 *   steps each; only the rays still walking after the last round are cut into segments.
 * steal = P > 0 (a power of two, 1..64; needs persistent = 0, sort = 0 and split = 0): one
 *   lane per ray, and every P steps each wave with at least steal_idle (1..64) idle lanes
 *   hands them the rest of walks still running in the wave. A walk whose rest [t, t1) is longer than the
 *   time the ray takes to cross steal_len voxels (1..2^20) along its fastest axis forks at
 *   the exit time e of one of its ancestor nodes: it keeps [t, e), and an idle lane
 *   continues the walk from e exactly as the walk would have, with a copy of its node
 *   stack, so no step is walked twice. A ray's result is its parts' hit of least t, kept
 *   per ray in LDS; parts behind a hit stop. Lanes past the last ray of a launch help too.
 *   This keeps lanes busy while a wave's longest walks finish.
 * interleave = 1 (needs persistent = 0, sort = 0 and split = 0): lane l of wave w of the
 *   launch takes ray l * W + w, W = ceil(n / 64), so each wave holds rays from all over the
 *   batch instead of 64 neighbours; hits are still written at each ray's index. This evens
 *   out the work per wave when the walk lengths of neighbouring rays are correlated (the
 *   secondary rays of one image), and costs coherent batches their locality.
 * rays_per_wave = R (0 meaning 64, else 1..64; R < 64 needs steal > 0 and interleave = 1):
 *   each wave starts with R rays (lane l < R of wave w takes ray l * W + w, W = ceil(n / R))
 *   and its other lanes start idle, taking forks from the first step on. A launch of few
 *   rays then spreads over W waves instead of ceil(n / 64): more waves per SIMD to hide
 *   each step's latency, at the cost of forks. */
typedef struct hvf_schedule {
  int32_t persistent;
  int32_t refill;
  int32_t inner;
  int32_t sort;
  int32_t sort_bits;
  int32_t blocks_per_cu;
  int32_t stack_depth; /* > 0: keep node-stack slots only for depths < stack_depth and
                          re-descend from the deepest kept ancestor on a deeper pop */
  int32_t lds_depths;  /* > 0: every block first copies the nodes of the top lds_depths
                          depths (a prefix of the buffer, at most 32 KiB) into LDS and
                          reads them there; HVF_E_INPUT if the prefix is larger */
  int32_t split;        /* 0, or K: see above */
  int32_t split_budget; /* steps of the first launch when split > 0 (1..2^20) */
  int32_t split_rounds; /* restart rounds of the split schedule (0..6; needs split > 0) */
  int32_t steal;        /* 0, or P: see above */
  int32_t steal_len;    /* voxels; shorter rests are not forked (steal > 0) */
  int32_t steal_idle;   /* idle lanes a wave needs before it forks walks (steal > 0) */
  int32_t interleave;   /* 0 or 1: see above */
  int32_t rays_per_wave; /* 0 (= 64) or 1..64: see above */
} hvf_schedule;

/* Build a volume on the host (Sec. 4.1).
 * format_spec: e.g. "G(7) R(4,4,4) --whole-level-dedup"; R(k^3) means R(k,k,k).
 *   Levels (table of implemented formats, Sec. 3.2): R(W,H,D) Raw grid, D(W,H,D,M) distance
 *   field (a Raw grid whose empty cells also store their L1 distance to the nearest
 *   non-empty cell, capped at M, 1 <= M <= 99; Sec. 3.3, 4.1, 4.2), S(L) SVO, G(L) SVDAG.
 *   With a DF level above the last the buffer is limited to 2^31 words.
 *   --whole-level-dedup: one de-duplication map per SVDAG level (Sec. 4.3).
 *   --restart-sv: restarting sparse-voxel intersection (Sec. 4.3): inside SVO/SVDAG levels
 *   no per-lane node stack is kept; after leaving a node the walk descends again from the
 *   level's root along the current position. Results are unchanged.
 *   --paper-layout: store the format in the paper's own word layout (Sec. 3.3, 4.1) instead
 *   of the library's: each level's child sub-volumes written before it, in Morton order of
 *   the cells; Raw cells and SVO/SVDAG leaves hold terminating integers (a pointer, or an
 *   occupied voxel's RGBA word 0xFFFFFFFF); an SVO node is (pointer to its children, masks),
 *   an SVDAG node its masks followed by one pointer per child; a DF cell is (terminating
 *   integer, capped distance). Results are unchanged; the buffer is larger for Raw- and
 *   SVO-final formats and smaller for deep SVDAGs. Not with --restart-sv (HVF_E_UNSUPPORTED)
 *   or short stacks or staged LDS depths (HVF_E_INPUT); hvf_build_device builds it too;
 *   batches and the server take such volumes, alone or mixed with the library's layout.
 * morton, n: strictly ascending Morton codes of the occupied voxels (host memory; x is
 *   bit 0, y bit 1, z bit 2 of each 3-bit group), all inside the volume. Not retained.
 * out: receives a new handle owned by the caller (release with hvf_free).
 * Errors: HVF_E_SPEC, HVF_E_INPUT, HVF_E_OVERFLOW, HVF_E_NOMEM, HVF_E_UNSUPPORTED.
 * Makes no HIP call. */
hvf_status hvf_build(const char* format_spec, const uint64_t* morton, size_t n, hvf_volume** out);

/* Build a volume on the device (Sec. 4.1) from Morton codes already in device memory.
 * The word buffer, statistics and host copy are identical to hvf_build's for the same
 * spec and codes; the nodes of every depth come from the codes by flag, scan and sort
 * passes on hip_stream (a hipStream_t, or NULL for the null stream), and SVDAG nodes are
 * de-duplicated by sorted content hashes, confirmed word by word.
 * format_spec: as for hvf_build, distance-field levels included (their capped distances
 *   come from separable relaxations along x, y and z on the device), and --paper-layout:
 *   the paper's write order (every node after its children's sub-trees) is computed from
 *   per-node subtree word counts, summed bottom-up and turned into offsets top-down; an
 *   SVDAG child or leaf is stored if it is the first equal one of its sub-volume (or level)
 *   in that order; --paper-layout is not combined with --depth-buffers (HVF_E_UNSUPPORTED).
 *   With --depth-buffers, or by itself once the library's layout reaches 2^32 words (2^31
 *   with a DF pointer grid), the buffer is split into per-depth regions with
 *   region-relative pointers, exactly as hvf_build does.
 * d_morton, n: device pointer to n strictly ascending Morton codes (x bit 0, y bit 1,
 *   z bit 2 of each 3-bit group), all inside the volume; n < 2^31. Read only, not retained.
 * out: receives a new handle owned by the caller (release with hvf_free); its device
 *   buffer is already resident on the current device (no upload needed).
 * Synchronises hip_stream before returning; temporary device memory (about 40 bytes per
 * code) is freed before returning. The host copy of the words (hvf_words, hvf_save) is
 * downloaded from the device buffer when first read.
 * Errors: HVF_E_SPEC, HVF_E_INPUT (null pointers, codes not ascending or outside the
 * volume), HVF_E_OVERFLOW, HVF_E_NOMEM, HVF_E_DEVICE, HVF_E_UNSUPPORTED (2^31 codes or more). */
hvf_status hvf_build_device(const char* format_spec, const uint64_t* d_morton, size_t n, void* hip_stream,
                            hvf_volume** out);

/* Copy the word buffer to device memory owned by the handle, on hip_stream (a
 * hipStream_t, or NULL for the null stream). Called implicitly by the first trace.
 * Errors: HVF_E_INPUT, HVF_E_NOMEM, HVF_E_DEVICE. */
hvf_status hvf_upload(hvf_volume* vol, void* hip_stream);

/* Concurrency: traces of one volume may run concurrently, on any streams and from any
 * host threads, with any schedules. Sorting takes per-call scratch from the stream-ordered
 * allocator. Splitting on the legacy default stream (NULL) reuses one survivor list per
 * volume, which that stream's ordering protects; on other streams, or when another host
 * thread holds the list, it takes per-call scratch as sorting does. At most 64 persistent
 * traces of one volume may be in flight at once. hvf_set_schedule and hvf_autotune must
 * not run concurrently with traces of the same volume. */

/* Trace n rays (Sec. 4.2). d_rays, d_hits: device pointers to n hvf_ray / hvf_hit,
 * caller-owned. Asynchronous on hip_stream; the caller synchronises. Uploads the volume
 * first if needed. n == 0 is a no-op. Errors: HVF_E_INPUT, HVF_E_DEVICE, HVF_E_NOMEM.
 * vol is not const: a trace may upload the buffer and create the volume's trace scratch
 * (persistent ray counters, the split survivor list) on first use, under the volume's
 * lock; the occupancy and the words never change. */
hvf_status hvf_trace(hvf_volume* vol, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits, void* hip_stream);

/* hvf_trace with an explicit schedule (NULL: the volume's current schedule). */
hvf_status hvf_trace_sched(hvf_volume* vol, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits,
                           const hvf_schedule* sched, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): hvf_trace_sched for a split schedule
 * (sched->split > 0) whose survivor lists live in a fixed device array of the library
 * instead of memory allocated per call. The array holds HVF_NOALLOC_MAX_RAYS rays' lists
 * (about 32 MiB per GPU, kept until the process ends); each GPU the library runs on has
 * its own. Hits are identical to hvf_trace_sched's with the same schedule.
 * vol: uploaded already (hvf_upload, or any earlier trace): HVF_E_STATE otherwise, since
 *   the upload allocates. d_rays, d_hits, n, hip_stream: as for hvf_trace.
 * Errors: HVF_E_INPUT (null pointers, sched NULL or without split, a schedule field out of
 * range, n > HVF_NOALLOC_MAX_RAYS), HVF_E_STATE, HVF_E_DEVICE. Makes no allocation: no
 * hipMalloc, hipFree or allocating library call. Calls that overlap on one GPU (concurrent
 * streams or host threads) share the array and race; the caller serialises them. */
#define HVF_NOALLOC_MAX_RAYS (1u << 21)
hvf_status hvf_trace_split_noalloc(hvf_volume* vol, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits,
                                   const hvf_schedule* sched, void* hip_stream);

/* Get / set the schedule hvf_trace uses for this volume (initially one lane per ray).
 * Not thread-safe against concurrent traces of the same volume. */
hvf_status hvf_get_schedule(const hvf_volume* vol, hvf_schedule* out);
hvf_status hvf_set_schedule(hvf_volume* vol, const hvf_schedule* sched);

/* Autotune: time candidate schedules (one lane per ray; short stacks of 2 and 4 depths;
 * persistent at full, 2 or 4 blocks per CU with refill thresholds 8/32 and 4 or 16 steps
 * between checks; sorted with cell sides 2^2, 2^4, 2^6; seven split schedules; five
 * stealing schedules; one lane per ray and the five stealing schedules again with
 * interleaved rays; the first of those with 32 and with 16 rays per wave), then the best
 * with the deepest LDS prefixes that fit, on the
 * caller's device ray sample; pick the fastest, store it as the volume's schedule and copy
 * it to *out (may be NULL). d_hits_scratch: n device hits, overwritten. Synchronises
 * hip_stream. Results never depend on the schedule chosen. */
hvf_status hvf_autotune(hvf_volume* vol, const hvf_ray* d_sample, size_t n, hvf_hit* d_hits_scratch,
                        hvf_schedule* out, void* hip_stream);

/* ---------------------------------------------------------------- batching
 * Many volumes (any formats and sizes) with ray batches of uneven size traced in one
 * persistent launch: a global counter hands out indices of the concatenated ray space,
 * idle lanes pick up the next rays (from whichever batch they fall in) whenever at least
 * `refill` of a wave's 64 lanes are idle. The launch (counter reset + kernel) is captured
 * once in a hipGraph and replayed by every hvf_batch_run. Each batch's hits are identical
 * to hvf_trace of that batch alone. */
typedef struct hvf_batch hvf_batch;

typedef struct hvf_batch_opts {
  int32_t refill;        /* 1..64 */
  int32_t inner;         /* traversal steps between refill checks, 1..4096 */
  int32_t blocks_per_cu; /* 0: as many as fit; else at most this many 256-thread blocks per CU */
  int32_t use_graph;     /* 1: capture and replay a hipGraph; 0: plain launches */
} hvf_batch_opts;

/* Describe a batched launch over m batches (1 <= m <= 256; total rays < 2^31): volume
 * vols[i] traces d_rays[i][0..n[i]) into d_hits[i]. The pointers are captured: the same
 * device buffers are read and written by every hvf_batch_run. Uploads the volumes.
 * Volumes must outlive the batch. opts may be NULL (defaults). Volumes with per-depth
 * regions (hvf_info.depth_buffers, e.g. past 2^32 words) may sit beside any others; the
 * launch then runs the region-aware kernel, which compiles every node kind in. */
hvf_status hvf_batch_create(hvf_volume* const* vols, const hvf_ray* const* d_rays, const size_t* n,
                            hvf_hit* const* d_hits, size_t m, const hvf_batch_opts* opts, hvf_batch** out);

/* Run (replay) the batched launch on hip_stream; asynchronous. */
hvf_status hvf_batch_run(hvf_batch* b, void* hip_stream);

/* Time candidate refill/inner/occupancy settings on the batch itself, keep the fastest
 * (re-capturing the graph) and copy it to *out (may be NULL). Synchronises hip_stream. */
hvf_status hvf_batch_autotune(hvf_batch* b, void* hip_stream, hvf_batch_opts* out);

/* Release a batch (waits for its device work to finish). NULL is ignored. */
void hvf_batch_free(hvf_batch* b);

/* ---------------------------------------------------------------- serving
 * A server keeps volumes resident in device memory and serves trace requests as they
 * arrive. Requests queue in arrival order and are admitted while fewer than max_slots are
 * in flight and the request's device footprint (48 bytes per ray, 256-byte granules) fits
 * in the free part of the memory budget; the rest wait. An engine thread packs every
 * admitted request into the next step (one batched persistent launch, with the ray upload
 * and hit download) on one of max_steps streams, so requests that arrive while others run
 * are admitted and overlap on the device. Each request's hits are identical to hvf_trace
 * of that request alone. Latency = submission to hits available in the caller's array. */
typedef struct hvf_server hvf_server;

#define HVF_SERVER_MAX_VOLUMES 1024

typedef struct hvf_serve_stats {
  uint64_t completed;
  double p50_ms, p99_ms, mean_ms, max_ms;
  uint64_t rays;
  double span_ms;  /* first submission to last completion */
  double mrays_s;  /* rays / span */
  uint64_t steps;
  uint64_t admission_waits;
  uint64_t peak_bytes, budget_bytes;
  uint64_t max_step_requests;
} hvf_serve_stats;

/* mem_budget_bytes: device (and pinned host staging) memory for in-flight requests.
 * max_slots: requests in flight at once (>= 1). max_steps: batched launches in flight at
 * once, each on its own stream (1..8). opts: kernel schedule (NULL: defaults; use_graph is
 * ignored). max_slots = max_steps = 1 serves one request at a time in arrival order. */
hvf_status hvf_server_create(size_t mem_budget_bytes, int max_slots, int max_steps, const hvf_batch_opts* opts,
                             hvf_server** out);
/* Make a volume resident (uploads it); it must outlive the server. Volumes with per-depth
 * regions are served like any other (steps holding one run the region-aware kernel). */
hvf_status hvf_server_add_volume(hvf_server* s, hvf_volume* vol, int* vol_id);
/* Queue a request: n host rays, results into n host hits. Non-blocking. Both arrays must
 * stay valid until the request completes. Rays in pinned host memory are copied to the
 * device directly; others are first copied into the server's pinned staging. hits may be
 * NULL: the results then stay in the server's staging (read them with
 * hvf_server_result) and keep their memory until hvf_server_release. HVF_E_NOMEM if the
 * request can never fit the budget. */
hvf_status hvf_server_submit(hvf_server* s, int vol_id, const hvf_ray* rays, size_t n, hvf_hit* hits,
                             uint64_t* req_id);
/* *done = 1 once the request has completed; its status is returned then (a request whose
 * step failed on the device completes with that error and never writes its hits). */
hvf_status hvf_server_poll(hvf_server* s, uint64_t req_id, int* done, double* latency_ms);
/* Results of a completed request submitted with hits == NULL (valid until released). */
hvf_status hvf_server_result(hvf_server* s, uint64_t req_id, const hvf_hit** hits);
/* Forget a completed request; frees its memory if the server held its results. */
hvf_status hvf_server_release(hvf_server* s, uint64_t req_id);
hvf_status hvf_server_wait(hvf_server* s, uint64_t req_id, double* latency_ms);
/* Wait until every submitted request has completed. */
hvf_status hvf_server_drain(hvf_server* s);
/* Testing the error path: the next n steps (n >= 0) fail at launch, before any device work,
 * as a step whose upload or launch fails does. Their requests complete with HVF_E_DEVICE,
 * their memory and slots are returned, and the server refuses new requests afterwards. */
hvf_status hvf_server_fail_steps(hvf_server* s, int n);
hvf_status hvf_server_stats(hvf_server* s, hvf_serve_stats* out);
/* Finish queued work, then release the server (not the volumes). NULL is ignored. */
void hvf_server_destroy(hvf_server* s);

/* Counting variant of hvf_trace, for byte accounting: the same traversal and results,
 * and for ray i the word index of each format load it makes, in order, in
 * d_log[i * cap + k] for k < cap, with the total number of loads in d_count[i] (it may
 * exceed cap; the log then holds the first cap), and, if d_steps is not NULL, the number
 * of traversal steps in d_steps[i]. d_log (n * cap uint32), d_count and d_steps (n uint32)
 * are caller-owned device buffers. Slower than hvf_trace; not for timing. */
hvf_status hvf_trace_count(hvf_volume* vol, const hvf_ray* d_rays, size_t n, hvf_hit* d_hits, uint32_t* d_log,
                           uint32_t cap, uint32_t* d_count, uint32_t* d_steps, void* hip_stream);

/* Synchronous convenience form: host ray and hit arrays, staged through device memory. */
hvf_status hvf_trace_host(hvf_volume* vol, const hvf_ray* rays, size_t n, hvf_hit* hits);

/* Sizes and per-level / per-depth node counts. */
hvf_status hvf_info_get(const hvf_volume* vol, hvf_info* out);

/* Copy the word buffer (host copy) into words[0..cap); *n_words receives its length. */
hvf_status hvf_words(const hvf_volume* vol, uint32_t* words, size_t cap, size_t* n_words);

/* Save / load a built volume: the construction's output file (Sec. 4.1 writes the built
 * format to an output file that the renderer then loads). The file holds a magic, the
 * spec, the word count, the per-depth and per-level statistics, the words and an FNV-1a
 * checksum. hvf_load returns a new handle owned by the caller. It refuses (HVF_E_INPUT) a
 * file whose checksum, spec or statistics do not match, and one in which any word index
 * a walk can read (a pointer, child descriptor, cell or block of any node reachable from
 * the root) or any depth offset lies past the buffer, so no kernel reads outside it. */
hvf_status hvf_save(const hvf_volume* vol, const char* path);
hvf_status hvf_load(const char* path, hvf_volume** out);

/* Release a handle and its host and device memory. NULL is ignored. */
void hvf_free(hvf_volume* vol);

const char* hvf_status_string(hvf_status s);
const char* hvf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HVF_H */
