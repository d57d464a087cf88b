// gconn_internal.hpp -- host-side shared declarations of the gconn library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>
#include <string>

#include "../../include/gconn.h"

namespace gconn {

// Work classes of the finish phase (and of top-down BFS levels): a vertex
// with at most kSmallDeg edges is handled by one lane, one with at most
// kMedDeg edges by one wave64, and larger ones are cut into kSeg-edge
// segments, one wave each.  Small and medium vertices are appended to
// kSubLists sub-lists (chosen by the 64-vertex group of the appending wave) so
// that the append counters are spread over many addresses: on this chip
// atomics to a single address serialise at ~11 ns each.
constexpr uint32_t kSmallDeg = 32;
constexpr uint32_t kMedDeg = 1024;
constexpr uint32_t kSeg = 1024;
constexpr uint32_t kSubLists = 64;
constexpr uint32_t kCntPad = 32;      // words between two work-list counters
constexpr uint32_t kMaxLmaxSamples = 4096;
constexpr int kRoundsPerSync = 8;        // device-side early-exit rounds per host check
constexpr uint32_t kRoundSlots = 64;     // ring of per-round "changed" flags
constexpr uint64_t kMaxRounds = 1u << 24;

// Device control block at the start of every workspace (zeroed per call by a
// kernel, never by hipMemsetAsync, so a captured graph replays correctly).
struct Ctrl {
  uint32_t lmax;
  uint32_t seg_count;
  uint32_t done;
  uint32_t err;
  uint32_t bfs_source;
  uint32_t comp_min;
  uint32_t frontier_count[2];
  uint32_t queue_cursor;              // BFS bitmap -> queue rebuild
  uint32_t pad0;
  unsigned long long edge_count;      // materialised finish edges (SV/LT/LP)
  unsigned long long frontier_edges[2];
  unsigned long long explored_edges;
  unsigned long long stat_sampled;
  unsigned long long stat_active;
  unsigned long long stat_finish_edges;
  unsigned long long stat_hooks;
  // work-list counters, one 128-byte line each: atomics on words of one line
  // are performed one after another, so packed counters would serialise the
  // appends of every wave in the launch
  uint32_t small_cnt[kSubLists * kCntPad];
  uint32_t medium_cnt[kSubLists * kCntPad];
  uint32_t changed[kRoundSlots];
  uint32_t kx_queue[8];               // XCD-bucketed k-out: per-XCD work-item cursors
  // BFS sampling, decided on the device level by level
  uint32_t bfs_mode;                  // this level: 0 finished, 1 top-down, 2 bottom-up
  uint32_t bfs_convert;               // 1: queue -> bitmap first, 2: bitmap -> queue first
  uint32_t bfs_as_queue;              // the current frontier is held as a queue
  uint32_t bfs_levels;                // levels run
};

struct WsLayout {
  size_t ctrl = 0;
  size_t P = 0;       // parent array when the caller gives no labels buffer
  size_t small = 0;   // small-vertex sub-lists (uint32[kSubLists][sub_cap])
  size_t medium = 0;  // medium-vertex sub-lists (uint32[kSubLists][sub_cap])
  size_t segs = 0;    // hub segments (uint2[seg_cap])
  size_t hooks = 0;   // Union-Hooks claim array (uint32[n])
  size_t prev = 0;    // round-start parents (SV, LT)
  size_t esrc = 0;    // materialised edges (SV, LT, LP)
  size_t edst = 0;
  size_t visited = 0; // BFS bitmap
  size_t fr_bits0 = 0, fr_bits1 = 0;  // BFS frontier bitmaps
  size_t queue0 = 0, queue1 = 0;      // BFS frontier queues
  size_t bfs_stripes = 0;             // BFS per-level counter stripes
  size_t bfs_slots = 0;               // BFS per-workgroup argmax / minimum slots
  size_t resid = 0;   // k-out pre-link: residual sampled edges (uint2[n])
  size_t words = 0;   // Union-JTB (rank, parent) words (uint64[n])
  size_t roots = 0;   // Union-JTB flat roots after sampling (uint32[n])
  size_t mins = 0;    // Union-JTB component minima for the labels (uint32[n])
  size_t kx_src = 0;  // XCD-bucketed k-out: residual records, first endpoint (uint32[chunks][2048])
  size_t kx_dst = 0;  //   second endpoint (same layout)
  size_t kx_root = 0; //   root of the first endpoint's pre-link tree (same layout)
  size_t kx_hdr = 0;  //   records per (chunk, XCD group) (uint32[chunks][8])
  size_t lrec_src = 0;  // local-first k-out: leaving edges by range and level (uint32)
  size_t lrec_dst = 0;
  size_t lrec_hdr = 0;  //   per range: number of records
  size_t probe = 0;     // automatic k-out: the locality probe's counts
  uint32_t sub_cap = 0;
  uint64_t seg_cap = 0;
  uint64_t edge_cap = 0;
  size_t total = 0;
};

// Rules that need a per-vertex claim array (LinkCtx::H, kEmpty-filled):
// Union-Hooks' hooks and Union-Rem-Lock's locks.
inline bool needs_claims(int link) {
  return link == GCONN_LINK_HOOKS || link == GCONN_LINK_REM_LOCK;
}

// Thread-local error reporting.
void set_error(const std::string& msg);
void clear_error();
gconn_status fail(gconn_status s, const std::string& msg);
gconn_status hip_fail(hipError_t e, const char* what);

#define GCONN_HIP(call)                                        \
  do {                                                         \
    hipError_t _e = (call);                                    \
    if (_e != hipSuccess) return ::gconn::hip_fail(_e, #call); \
  } while (0)

#define GCONN_LAUNCHED(what)                                    \
  do {                                                          \
    hipError_t _e = hipGetLastError();                          \
    if (_e != hipSuccess) return ::gconn::hip_fail(_e, what);   \
  } while (0)

#define GCONN_TRY(expr)                      \
  do {                                       \
    gconn_status _s = (expr);                \
    if (_s != GCONN_OK) return _s;           \
  } while (0)

// Option / graph validation (host only; no device access).
gconn_status check_options(const gconn_options& o);
gconn_status check_graph(const gconn_graph* g);
gconn_status check_device_ptr(const void* p, const char* name);
gconn_status check_device_ready();
bool is_union_find(int link);

// Workspace planning for one static run.
WsLayout plan_workspace(const gconn_graph& g, const gconn_options& o, bool forest, bool labels);

// The static pipeline (sampling, L_max, finish, finalisation) on parent array
// P (n entries).  fu/fv nullable (forest).  labels: write canonical labels into
// P at the end (finalisation) when true.
gconn_status run_static(const gconn_graph& g, uint32_t* P, uint32_t* fu, uint32_t* fv,
                        bool finalize, uint8_t* ws, const WsLayout& L, const gconn_options& o,
                        gconn_stats* stats, hipStream_t s);

// Synchronous check of a graph's offsets and ids; uses ctrl->err.
gconn_status validate_graph(const gconn_graph& g, Ctrl* ctrl, uint32_t block, hipStream_t s);

// Union-JTB (gconn_jtb.hip): the same pipeline over 64-bit (rank, parent)
// words.  words: the word array to use (nullable: the workspace's own); P
// receives canonical labels when finalize is set.
WsLayout plan_workspace_jtb(const gconn_graph& g, const gconn_options& o, bool forest, bool labels);
gconn_status run_static_jtb(const gconn_graph& g, uint32_t* P, uint32_t* fu, uint32_t* fv,
                            bool finalize, uint8_t* ws, const WsLayout& L, const gconn_options& o,
                            gconn_stats* stats, hipStream_t s, uint64_t* words);
gconn_status launch_jtb_init(uint64_t* W, uint32_t n, hipStream_t s);
gconn_status launch_jtb_insert(const gconn_options& o, uint64_t* W, const uint32_t* src,
                               const uint32_t* dst, uint64_t k, hipStream_t s);
// kind: nullable (plain query batch); else a mixed batch's queries only.
gconn_status launch_jtb_query(const gconn_options& o, uint64_t* W, const uint8_t* kind,
                              const uint32_t* a, const uint32_t* b, uint64_t q, uint8_t* out,
                              hipStream_t s);
gconn_status launch_jtb_mixed(const gconn_options& o, uint64_t* W, const uint8_t* kind,
                              const uint32_t* a, const uint32_t* b, uint64_t count, uint8_t* out,
                              hipStream_t s);
// Canonical labels (component minima) from the words; scratch: n entries.
gconn_status launch_jtb_labels(const uint64_t* W, uint32_t n, uint32_t* labels, uint32_t* scratch,
                               hipStream_t s);

// Incremental helpers implemented next to the static kernels.
gconn_status launch_iota(uint32_t* P, uint32_t n, hipStream_t s);
gconn_status launch_fill(uint32_t* p, uint32_t value, uint64_t count, hipStream_t s);
gconn_status launch_finalize(uint32_t* P, uint32_t n, uint32_t* labels, hipStream_t s);
gconn_status launch_insert(const gconn_options& o, uint32_t* P, uint32_t* H, const uint32_t* src,
                           const uint32_t* dst, uint64_t k, hipStream_t s);
// Clear the control block and set P[v] = v (one kernel).
gconn_status reset_ctrl_and_parents(Ctrl* ctrl, uint32_t* P, uint32_t n, hipStream_t s);
// Many-graph pipeline and autotuner step (gconn_batch.hip).
gconn_status batch_workspace_size(const gconn_batch* b, size_t* bytes);
gconn_status run_batch(const gconn_batch* b, uint32_t* labels_out, void* workspace,
                       size_t workspace_bytes, const gconn_class_options* classes,
                       uint32_t num_classes, uint32_t lmax_samples, uint64_t seed,
                       gconn_stats* stats, hipStream_t s);
gconn_status autotune(const gconn_graph* graphs, uint32_t num_graphs,
                      const gconn_options* candidates, uint32_t num_candidates, uint32_t reps,
                      uint32_t* labels_scratch, void* workspace, size_t workspace_bytes,
                      hipStream_t s, uint32_t* best, double* times_ms);
// Synchronous id check of a pair list (ids < n); uses ctrl as scratch.
gconn_status validate_pairs(const uint32_t* a, const uint32_t* b, uint64_t k, uint32_t n,
                            Ctrl* ctrl, hipStream_t s);
gconn_status launch_query(const gconn_options& o, uint32_t* P, const uint32_t* a,
                          const uint32_t* b, uint64_t q, uint8_t* out, hipStream_t s);
// Mixed batch: the inserts (kind 0), then the queries (kind 1; out 0 for inserts).
gconn_status launch_mixed(const gconn_options& o, uint32_t* P, uint32_t* H, const uint8_t* kind,
                          const uint32_t* a, const uint32_t* b, uint64_t count, uint8_t* out,
                          hipStream_t s);
// Synchronous check that every kind is 0 or 1; uses ctrl as scratch.
gconn_status validate_kinds(const uint8_t* kind, uint64_t count, Ctrl* ctrl, hipStream_t s);

// Phase profiler (thread-local; HIP events on the caller's stream).
enum Phase : int {
  kPhaseInit = 0, kPhaseSample, kPhaseCompress, kPhaseLmax, kPhaseGather, kPhaseFinish,
  kPhaseFinalize, kPhaseCount
};
bool profiling();
gconn_status prof_mark(int phase, bool begin, hipStream_t s);
void prof_count_run();
gconn_status profile_enable(int on);
gconn_status profile_read(gconn_phase_times* out, int reset);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

inline uint32_t grid_for(uint64_t items, uint32_t block, uint32_t cap = 1u << 20) {
  uint64_t g = (items + block - 1) / block;
  if (g == 0) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

}  // namespace gconn
