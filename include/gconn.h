/*
 * gconn.h -- C ABI of the MI355X (gfx950) graph-connectivity library.
 *
 * Implements the connectivity design space of Hong, Dhulipala and Shun,
 * "Exploring the Design Space of Static and Incremental Graph Connectivity
 * Algorithms on GPUs" (PACT 2020): a sampling phase (k-out, hook-based, BFS),
 * the most frequent label L_max, a finish phase over the vertices whose label
 * is not L_max (union-find variants with CAS linking, Shiloach-Vishkin,
 * Liu-Tarjan, label propagation) with on-the-fly or separate tree compression,
 * label finalisation, spanning-forest recording, and incremental batches of
 * edge insertions and connectivity queries.
 *
 * Conventions shared by every entry point
 *  - Vertex ids are uint32 in [0, n) with n <= 0xFFFFFFFE (0xFFFFFFFF is the
 *    "empty" sentinel of forest slots and hook arrays).  Edge counts are uint64.
 *  - Every array argument named "device" is memory the caller allocated on the
 *    current HIP device (hipMalloc, or a torch CUDA tensor); the library never
 *    allocates device memory except where a function says so, and never frees
 *    caller memory.  The caller keeps ownership of every buffer.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *    enqueued on it and the call returns without waiting unless the function
 *    says otherwise; results are valid once the stream has been synchronised.
 *    Workspace contents are scratch: do not reuse a workspace on another
 *    stream while a call using it may still run.
 *  - Argument errors are detected on the host before anything is enqueued and
 *    return GCONN_EINVAL (message in gconn_last_error()).  HIP launch errors
 *    return GCONN_EDEVICE.  Nothing throws across the ABI.
 *  - Self-loops and duplicate edges are allowed everywhere.  n == 0 or m == 0
 *    is a valid input (labels are then the identity).
 *  - CSR rows must be sorted ascending when a sampler that reads "the first"
 *    edges of a vertex is used (k-out, hook-based); results are still exact if
 *    they are not, only the sampled subset changes.
 */
#ifndef GCONN_H
#define GCONN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gconn_status {
  GCONN_OK = 0,
  GCONN_EINVAL = -1,       /* bad argument (null pointer, id range, option)      */
  GCONN_ENOMEM = -2,       /* caller workspace smaller than gconn_workspace_size */
  GCONN_EDEVICE = -3,      /* HIP runtime / launch error                          */
  GCONN_ENODEV = -4,       /* no HIP device, or not a gfx950 device               */
  GCONN_EBUSY = -5,        /* admission refused (serving)                         */
  GCONN_ETIMEOUT = -6,     /* bounded wait expired                                */
  GCONN_EUNSUPPORTED = -7  /* option combination without a correct algorithm     */
} gconn_status;

/* Graph formats (Notation: COO edge array; CSR Offsets[n+1] + Edges[m]). */
enum { GCONN_CSR = 0, GCONN_COO = 1 };

/* Sampling phase (Sampling Algorithms; Appendix A.1). */
enum {
  GCONN_SAMPLE_NONE = 0,
  GCONN_SAMPLE_KOUT = 1, /* union-find over k edges per vertex, then full compress */
  GCONN_SAMPLE_HB = 2,   /* hook to the first neighbour, then first N edges of roots */
  GCONN_SAMPLE_BFS = 3   /* direction-optimising BFS from the largest-degree vertex */
};

/* Finish (link) algorithm (Finish Algorithms; Appendix A.2-A.4). */
enum {
  GCONN_LINK_ASYNC = 0,   /* Union-Async: CAS the larger root onto the smaller     */
  GCONN_LINK_HOOKS = 1,   /* Union-Hooks: CAS on a hooks array, then plain write   */
  GCONN_LINK_EARLY = 2,   /* Union-Early: walk both paths, hook on reaching a root */
  GCONN_LINK_REM_CAS = 3, /* Union-Rem-CAS: Rem's algorithm with CAS + splice rule */
  GCONN_LINK_ECL = 4,     /* ECL-CC's rule: Union-Async, halving finds, separate
                             full-compress pass                                    */
  GCONN_LINK_SV = 5,      /* root-based Shiloach-Vishkin (writeMin + full shortcut) */
  GCONN_LINK_LT = 6,      /* Liu-Tarjan rule set, variant in lt_variant            */
  GCONN_LINK_LP = 7,      /* label propagation                                     */
  GCONN_LINK_AFFOREST = 8, /* G_Afforest: Afforest's link (walk two levels, CAS a
                             root under the lower side), separate full compress   */
  GCONN_LINK_REM_LOCK = 9, /* Union-Rem-Lock: Rem's algorithm, the root link made
                             under a per-vertex try-lock (wave-safe: a lane that
                             gets the lock finishes and releases it in the same
                             step, so lanes of one wave never wait on each other) */
  GCONN_LINK_JTB = 10     /* Union-JTB: randomized linking by rank (Jayanti, Tarjan
                             and Boix-Adsera); parent and rank share one 64-bit word
                             updated by 64-bit CAS, ties broken by a seeded random
                             key; finds are FIND_NAIVE (FindSimple) or
                             FIND_TWO_TRY_SPLIT.  Roots are not component minima,
                             so labels come from a separate minimum reduction.
                             Sampling: none or k-out (one lane per vertex; the
                             schedule, pre-link and local-first options do not
                             apply); the workspace holds the words (8 bytes per
                             vertex).  Not in batched or served calls.         */
};

/* On-the-fly compression inside Find (Appendix A.2, find options). */
enum {
  GCONN_FIND_NAIVE = 0,    /* no compression                                 */
  GCONN_FIND_SPLIT = 1,    /* path splitting with CAS (AtomicSplit)          */
  GCONN_FIND_HALVE = 2,    /* path halving with CAS (AtomicHalve)            */
  GCONN_FIND_COMPRESS = 3, /* full path compression (not for Union-Rem-CAS)  */
  GCONN_FIND_TWO_TRY_SPLIT = 4 /* Union-JTB only: two splitting CAS tries at each
                                  vertex of the walk before moving on       */
};

/* Splice rule of Union-Rem-CAS at a non-root (Appendix A.2, splice options). */
/* SPLICE_ATOMIC: Rem's splice, done with a CAS (Appendix A.2, Union-Rem-CAS
 * splice options): a non-root r_u whose parent is above P[r_v] is re-hung
 * under P[r_v] and the walk continues from its old parent.  Correct when
 * unions and queries are separated, which every call of this library is
 * (static runs; epoch-fenced incremental batches). */
enum { GCONN_SPLICE_SPLIT_ONE = 0, GCONN_SPLICE_HALVE_ONE = 1, GCONN_SPLICE_ATOMIC = 2 };

/* Liu-Tarjan variants, in the paper's order (Appendix A.4): connect rule
 * C(onnect)/P(arentConnect)/E(xtendedConnect), update rule U(pdate)/R(ootUpdate),
 * shortcut S(hortcut)/F(ullShortcut), optional A(lter). */
enum {
  GCONN_LT_CUSA = 0, GCONN_LT_CRSA, GCONN_LT_PUSA, GCONN_LT_PRSA, GCONN_LT_PUS, GCONN_LT_PRS,
  GCONN_LT_EUSA, GCONN_LT_EUS, GCONN_LT_CUFA, GCONN_LT_CRFA, GCONN_LT_PUFA, GCONN_LT_PRFA,
  GCONN_LT_PUF, GCONN_LT_PRF, GCONN_LT_EUFA, GCONN_LT_EUF, GCONN_LT_COUNT
};

/* A graph resident in device memory.
 *  CSR: offsets[n+1] (uint32 or uint64, offsets_64 says which; offsets[0] = 0,
 *       non-decreasing, offsets[n] = m) and nbrs[m]; a symmetric graph stores
 *       every undirected edge in both rows (the paper's inputs are symmetrised).
 *  COO: nbrs = src[m], dst[m]: one entry per undirected edge is enough. */
typedef struct gconn_graph {
  int32_t format;        /* GCONN_CSR or GCONN_COO                  */
  int32_t offsets_64;    /* CSR only: 1 = uint64 offsets, 0 = uint32 */
  uint32_t n;            /* number of vertices                       */
  uint32_t reserved;
  uint64_t m;            /* CSR entries, or COO edges                */
  const void* offsets;   /* device, CSR only                         */
  const uint32_t* nbrs;  /* device: CSR neighbours, or COO sources   */
  const uint32_t* dst;   /* device: COO destinations (NULL for CSR)  */
} gconn_graph;

typedef struct gconn_options {
  int32_t sample;        /* GCONN_SAMPLE_*                      (default KOUT)   */
  int32_t link;          /* GCONN_LINK_*                        (default ASYNC)  */
  int32_t find;          /* GCONN_FIND_*                        (default SPLIT)  */
  int32_t splice;        /* GCONN_SPLICE_* (Union-Rem-CAS only) (default SPLIT_ONE) */
  int32_t lt_variant;    /* GCONN_LT_* (GCONN_LINK_LT only)     (default PRF)    */
  uint32_t k;            /* k-out: edges sampled per vertex     (default 2)      */
  uint32_t hb_n;         /* hook-based: first N edges of roots  (default 4)      */
  uint32_t lmax_samples; /* vertices sampled for L_max, 1..4096 (default 1024)   */
  uint64_t seed;         /* seeds the L_max sample and random k-out choices      */
  int32_t kout_random;   /* 0: first k edges; 1: first edge + k-1 uniform picks  */
  int32_t validate;      /* 1: check the graph on the device first (synchronous) */
  int32_t block;         /* threads per workgroup, multiple of 64, <= 1024 (256) */
  int32_t schedule;      /* k-out kernel shape: 0 automatic (default): for first
                            k <= 2 a probe of 4096 seeded vertices decides on
                            the device -- the local-first passes (kout_local)
                            when at least a quarter of the sampled edges stay
                            inside their vertex's id range and the graph spans
                            at least 64 ranges (meshes and other graphs whose
                            ids follow their geometry), else persistent lanes
                            with the next vertex's row prefetched (the only
                            choice for k > 2 or random picks); 1 one lane per
                            vertex, 2 lane-refill step machine (Union-Rem-CAS,
                            first-k, uint32 offsets; else as 0), 3 two-stage
                            pipeline: the next vertex's neighbour parents
                            loaded during the current unions (Union-Rem-CAS
                            with SplitAtomicOne / HalveAtomicOne, first k <= 2;
                            else as 0), 4 two passes: a streaming pass writes
                            every vertex's sampled neighbours to a slot array,
                            then the union pass runs over the slots, so its
                            lanes start on unions at once (first k <= 2; else
                            as 0), 5 flat: the pre-link pass (kout_prelink),
                            then a pass that points every vertex at its
                            pre-link tree's root, then the union pass over
                            the remaining sampled edges, starting from roots
                            (first k <= 2; else as 0), 6 XCD-bucketed: the
                            pre-link and flattening, then the remaining
                            sampled edges grouped by the XCD whose share of
                            the ids holds their second endpoint and united by
                            workgroups running on that XCD (first k <= 2;
                            else as 0)                                     (0) */
  int32_t atomic_compress; /* path-compression and splice writes (FindSplit,
                            FindHalve, SplitAtomicOne, HalveAtomicOne, the
                            Union-Early splice): 1 CAS as in the atomic rules,
                            0 relaxed agent-scope stores (they only ever move
                            a non-root's parent to one of its ancestors)  (1) */
  int32_t kout_prelink;  /* first-k k-out with k <= 2: 1 links every vertex to
                            its smallest sampled neighbour, when that is smaller,
                            with one plain store before any union runs (each
                            vertex is still a root and the only writer of its
                            own slot), and sends only its other sampled edge(s)
                            through the union rule; 0 unites every sampled edge.
                            Same partition either way.                     (0) */
  int32_t kout_local;    /* first-k k-out with k <= 2: 1 unites, in LDS, the
                            sampled edges whose endpoints both lie in the same
                            id range (one workgroup per range; the largest
                            power of two up to 32768 vertices whose parents
                            fit the device's LDS), then unites each distinct
                            pair of range-local roots that the edges leaving a
                            range join, once -- for graphs whose ids are
                            local, such as grids and meshes.  Same partition.
                            Overrides kout_prelink.                         (0) */
} gconn_options;

/* Counters filled when a stats pointer is passed (the call then synchronises
 * the stream before returning).  Host memory. */
typedef struct gconn_stats {
  uint64_t sampled_edges;   /* neighbour entries read by the sampling phase
                               (BFS: the row entries of the visited vertices)   */
  uint64_t active_vertices; /* vertices gathered for the finish (label != L_max) */
  uint64_t finish_edges;    /* neighbour entries read by the finish (SV/LT/LP: first round) */
  uint64_t hooks;           /* successful root links (union-find rules)         */
  uint64_t rounds;          /* SV / LT / LP rounds, or BFS levels               */
  uint32_t lmax;            /* most frequent sampled label (0xFFFFFFFF: none)   */
  uint32_t bfs_source;      /* BFS sampling source (0xFFFFFFFF: none)           */
} gconn_stats;

/* Fills *opt with the defaults listed above. */
void gconn_options_default(gconn_options* opt);

/* Bytes of device workspace gconn_cc / gconn_spanning_forest need for this
 * graph and options (want_forest = 1 for the spanning forest; want_labels = 0
 * when the forest call gets labels_out == NULL).  opt may be NULL (defaults). */
gconn_status gconn_workspace_size(const gconn_graph* g, const gconn_options* opt, int want_forest,
                                  int want_labels, size_t* bytes);

/* Static connectivity (Alg. "GConn for Static Connectivity"): labels_out[v]
 * (device, n entries, caller-owned) receives the minimum vertex id of v's
 * component.  labels_out doubles as the parent array during the run.
 * workspace: device, >= gconn_workspace_size(g, opt, 0, 1) bytes, 256-byte
 * aligned.  COO input uses the finish phase only (sampling needs CSR).
 * The call returns without waiting, except for the iterative parts whose
 * length depends on the data: SV, LT and LP run their rounds, and BFS
 * sampling its levels, eight at a time on the device (each round or level
 * decides on the device whether to run, and does nothing once the work is
 * done), with one host check of the stop flag per eight. */
gconn_status gconn_cc(const gconn_graph* g, uint32_t* labels_out, void* workspace,
                      size_t workspace_bytes, const gconn_options* opt, gconn_stats* stats,
                      void* stream);

/* gconn_cc without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops that must not call
 * hipMalloc, harnesses that forbid it).  Same arguments and results as
 * gconn_cc minus the workspace: the pipeline runs in a scratch array of
 * GCONN_NOALLOC_SCRATCH_BYTES that the library holds in device memory, one per
 * device, from the first use until the process ends.  The call allocates
 * nothing (no hipMalloc, no hipFree, no allocating library routine).
 * Returns GCONN_ENOMEM, before enqueuing anything, when gconn_workspace_size
 * for this graph and these options exceeds the scratch size (with 16 entries
 * per vertex: about n <= 2.7M vertices for the default automatic k-out
 * schedule, which keeps room for the local-first passes, and about n <= 8.1M
 * with schedule 1), and GCONN_EUNSUPPORTED while phase
 * profiling is on.  Every call on one device shares that device's scratch
 * array and leaves it holding its own intermediate state (each run clears what
 * it needs with kernels): calls that may overlap on one device -- on
 * different streams, or from different threads -- race and must be
 * serialised by the caller. */
#define GCONN_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
gconn_status gconn_cc_noalloc(const gconn_graph* g, uint32_t* labels_out,
                              const gconn_options* opt, gconn_stats* stats, void* stream);

/* Spanning forest (Alg. "GConn for Spanning Forest"): for every vertex r that
 * stops being a root, fu[r], fv[r] (device, n entries each) receive the input
 * edge that linked it; other slots hold 0xFFFFFFFF.  Exactly n - c slots are
 * filled (c = number of components).  labels_out (device, nullable) receives
 * the canonical labels as in gconn_cc.  Root-based finishes only: union-find
 * rules and SV (LT, LP, and Union-Rem-CAS / Rem-Lock with SPLICE_ATOMIC
 * return GCONN_EUNSUPPORTED). */
gconn_status gconn_spanning_forest(const gconn_graph* g, uint32_t* fu, uint32_t* fv,
                                   uint32_t* labels_out, void* workspace, size_t workspace_bytes,
                                   const gconn_options* opt, gconn_stats* stats, void* stream);

/* Incremental connectivity (Alg. "GConn for Incremental Connectivity").
 * The handle is host memory created by gconn_inc_create; it keeps the parent
 * array `parent_buf` (device, n_max entries, caller-owned, must outlive the
 * handle) and uses `workspace` (device, >= gconn_inc_workspace_size bytes,
 * caller-owned, must outlive the handle).  If `initial` is non-NULL its graph
 * (n <= n_max) is connected first with gconn_cc's pipeline.  Batches are
 * totally ordered on the handle's stream: a query batch sees exactly the
 * inserts enqueued before it.  A handle is not thread-safe.  With
 * GCONN_LINK_JTB the forest lives in the workspace as 64-bit (rank, parent)
 * words and parent_buf is scratch for gconn_inc_labels. */
typedef struct gconn_inc gconn_inc;

gconn_status gconn_inc_workspace_size(uint32_t n_max, const gconn_graph* initial,
                                      const gconn_options* opt, size_t* bytes);
gconn_status gconn_inc_create(uint32_t n_max, uint32_t* parent_buf, const gconn_graph* initial,
                              void* workspace, size_t workspace_bytes, const gconn_options* opt,
                              void* stream, gconn_inc** out);
/* Insert k edges (src[i], dst[i]) (device arrays, ids < n_max). */
gconn_status gconn_inc_insert_batch(gconn_inc* h, const uint32_t* src, const uint32_t* dst,
                                    uint64_t k, void* stream);
/* out[i] (device, q bytes) = 1 iff a[i] and b[i] are connected, else 0. */
gconn_status gconn_inc_query_batch(gconn_inc* h, const uint32_t* a, const uint32_t* b, uint64_t q,
                                   uint8_t* out, void* stream);
/* Mixed batch (Alg. "GConn for Incremental Connectivity": a batch mixes
 * inserts and queries).  kind[i] (device, count bytes) is GCONN_REQ_INSERT for
 * the edge (a[i], b[i]) and GCONN_REQ_QUERY for the pair (a[i], b[i]).  Every
 * insert of the batch is applied first, then every query is answered, so the
 * answers are deterministic: out[i] (device, count bytes) = 1 iff element i is
 * a query whose endpoints are connected once all of the batch's inserts (and
 * the earlier batches) are in; 0 for inserts.  Any other kind value is
 * GCONN_EINVAL when options.validate is set, and undefined otherwise. */
gconn_status gconn_inc_mixed_batch(gconn_inc* h, const uint8_t* kind, const uint32_t* a,
                                   const uint32_t* b, uint64_t count, uint8_t* out, void* stream);
/* labels_out (device, n_max entries) = canonical labels of the current graph. */
gconn_status gconn_inc_labels(gconn_inc* h, uint32_t* labels_out, void* stream);
/* Frees the host handle only (no device memory is owned). */
gconn_status gconn_inc_destroy(gconn_inc* h);

/* ------------------------------------------------------------- many graphs
 * Many independent graphs connected by one pipeline run (one launch per phase
 * for all of them).  Graph g owns the vertex range [vbase[g], vbase[g+1]) of
 * one concatenated CSR whose neighbour ids are global (vbase[g] + local id);
 * its edges must stay inside its range.  Every vbase[g] is a multiple of 64
 * (pad with isolated vertices), so each 64-vertex tile belongs to one graph.
 * Each graph gets its own L_max (the paper's sampling/finish split, per
 * graph), and each graph class its own sampling and union-find rule, chosen
 * per class by a caller or by gconn_autotune and dispatched inside the same
 * kernels. */
#define GCONN_MAX_CLASSES 64

typedef struct gconn_batch {
  uint32_t num_graphs;         /* G                                                */
  uint32_t n;                  /* vbase[G]: all vertices, padding included         */
  uint64_t m;                  /* total CSR entries                                */
  const uint64_t* offsets;     /* device, n + 1 (global)                           */
  const uint32_t* nbrs;        /* device, m global neighbour ids                   */
  const uint32_t* vbase;       /* device, G + 1: vbase[0] = 0, multiples of 64     */
  const uint8_t* graph_class;  /* device, G class indices (NULL: every graph in 0) */
  uint32_t block;              /* threads per workgroup of every batch kernel:
                                  0 = 256, else a multiple of 64 in [64, 1024]     */
  uint32_t reserved;
} gconn_batch;

typedef struct gconn_class_options {
  int32_t sample;    /* GCONN_SAMPLE_NONE, GCONN_SAMPLE_KOUT (first k edges) or
                        GCONN_SAMPLE_HB (hook to the first neighbour, then the
                        first k edges of the vertices that stayed roots)         */
  int32_t link;      /* GCONN_LINK_ASYNC, GCONN_LINK_REM_CAS or GCONN_LINK_EARLY    */
  int32_t find;      /* GCONN_FIND_NAIVE, _SPLIT or _HALVE                          */
  int32_t splice;    /* GCONN_SPLICE_* (Union-Rem-CAS)                              */
  uint32_t k;        /* k-out edges per vertex, or hook-based N (1..64)             */
  uint32_t reserved;
} gconn_class_options;

gconn_status gconn_cc_batch_workspace_size(const gconn_batch* b, size_t* bytes);

/* labels_out (device, n entries, caller-owned) receives, for every vertex v of
 * graph g, the minimum LOCAL id (id - vbase[g]) of v's component in graph g;
 * padding vertices get their own local id.  classes: host array of
 * num_classes (1..GCONN_MAX_CLASSES) entries.  lmax_samples / seed: as in
 * gconn_options.  Asynchronous on `stream` (synchronous if stats != NULL). */
gconn_status gconn_cc_batch(const gconn_batch* b, uint32_t* labels_out, void* workspace,
                            size_t workspace_bytes, const gconn_class_options* classes,
                            uint32_t num_classes, uint32_t lmax_samples, uint64_t seed,
                            gconn_stats* stats, void* stream);

/* Autotuner step: times every candidate option set on every given graph
 * (one warm-up, then `reps` timed runs each, HIP events on `stream`) and
 * writes the index of the candidate with the smallest total to *best and the
 * totals (ms) to times_ms (host, num_candidates entries, nullable).
 * labels_scratch: device, at least max n entries.  workspace: device, large
 * enough for every candidate on every graph.  Synchronous. */
gconn_status gconn_autotune(const gconn_graph* graphs, uint32_t num_graphs,
                            const gconn_options* candidates, uint32_t num_candidates,
                            uint32_t reps, uint32_t* labels_scratch, void* workspace,
                            size_t workspace_bytes, void* stream, uint32_t* best,
                            double* times_ms);

/* Captured pipelines (HIP graphs).  gconn_cc_capture / gconn_cc_batch_capture
 * validate their arguments exactly as gconn_cc / gconn_cc_batch do, then
 * record the whole launch sequence of one run into a HIP graph (on a private
 * stream; nothing runs yet) and instantiate it.  gconn_exec_launch replays it
 * on `stream` with one launch: the same pointers, sizes and options, reading
 * whatever the input buffers hold at that time, writing labels_out again.
 * Launch-bound callers (small graphs, many repeats) save the per-kernel launch
 * cost.  Only pipelines with no host round trip can be captured: union-find
 * finishes (no SV, LT or LP) with k-out, hook-based or no sampling (BFS checks
 * its stop flag on the host every eight levels), options.validate = 0, no
 * statistics, and phase profiling off -- anything else is GCONN_EUNSUPPORTED.  The caller keeps
 * every buffer alive while the handle exists; replays on one handle must not
 * overlap (they share the workspace).  Host-owned handle. */
typedef struct gconn_exec gconn_exec;
gconn_status gconn_cc_capture(const gconn_graph* g, uint32_t* labels_out, void* workspace,
                              size_t workspace_bytes, const gconn_options* opt, gconn_exec** out);
gconn_status gconn_cc_batch_capture(const gconn_batch* b, uint32_t* labels_out, void* workspace,
                                    size_t workspace_bytes, const gconn_class_options* classes,
                                    uint32_t num_classes, uint32_t lmax_samples, uint64_t seed,
                                    gconn_exec** out);
gconn_status gconn_exec_launch(gconn_exec* e, void* stream);
gconn_status gconn_exec_destroy(gconn_exec* e);

/* ------------------------------------------------------------- serving
 * A request loop over one resident parent array (incremental connectivity
 * served online).  Clients submit insert or query batches from host memory
 * at any time; a worker thread admits them in submission order while the
 * caller's device arena (and a pinned host staging area of the same size the
 * server allocates) has room for their data -- admission by HBM footprint --
 * copies them to the device and runs them on several HIP streams.  Requests of
 * the same kind that follow each other form an epoch and overlap on the device
 * (inserts commute; queries only read connectivity); the first request of a
 * new epoch, and every request after it in that epoch, waits on events
 * recorded on every stream when the epoch began, so a query batch sees exactly
 * the inserts submitted before it and no later one.  Each request's answers
 * are therefore the same whether it runs alone or in a mix.  The server's
 * streams have default priority. */
typedef struct gconn_server gconn_server;

enum { GCONN_REQ_INSERT = 0, GCONN_REQ_QUERY = 1 };

typedef struct gconn_server_config {
  uint32_t n_max;          /* vertices (ids < n_max)                                */
  uint32_t streams;        /* device streams for overlap, 1..16 (0 -> 4)            */
  uint64_t arena_bytes;    /* device arena = in-flight budget; insert of k edges
                              needs 8k bytes, query of q pairs 9q (each rounded up
                              to 256)                                                */
  gconn_options options;   /* union-find rule for inserts, find rule for queries   */
} gconn_server_config;

typedef struct gconn_request_info {
  int32_t kind;            /* GCONN_REQ_*                                           */
  int32_t status;          /* gconn_status of the request                           */
  uint64_t count;          /* edges or pairs                                        */
  uint64_t epoch;          /* epoch number it ran in                                */
  double submit_us;        /* microseconds since server creation                    */
  double admit_us;
  double done_us;          /* result visible on the host                            */
} gconn_request_info;

/* parent_buf: device, n_max entries; arena: device, arena_bytes; both
 * caller-owned and kept until gconn_server_destroy.  The parent array is
 * initialised here (P[v] = v). */
gconn_status gconn_server_create(const gconn_server_config* cfg, uint32_t* parent_buf,
                                 void* arena, gconn_server** out);
/* Copies nothing yet: a, b (host, count entries) and out (host, count bytes,
 * queries only: 1 iff connected) must stay valid until the request is done.
 * Pageable buffers go through the server's pinned staging area; buffers that
 * are pinned already (hipHostMalloc, torch pin_memory) are read and written
 * by the copy engines directly, with no host copy.  Returns GCONN_EINVAL, and
 * queues nothing, for a request larger than the arena or one holding a vertex
 * id >= n_max (submission scans the ids on the host whatever
 * options.validate says: the parent array is shared by every client, so one
 * bad id must not reach the kernels).  Thread-safe. */
gconn_status gconn_server_submit(gconn_server* s, int kind, const uint32_t* a, const uint32_t* b,
                                 uint64_t count, uint8_t* out, uint64_t* ticket);
/* Blocks until the request is done or timeout_s (< 0: no limit) elapses
 * (GCONN_ETIMEOUT).  info (nullable) receives its record. */
gconn_status gconn_server_wait(gconn_server* s, uint64_t ticket, double timeout_s,
                               gconn_request_info* info);
/* Blocks until every submitted request is done. */
gconn_status gconn_server_drain(gconn_server* s);
/* Drains, stops the worker, frees host resources (not the caller's buffers). */
gconn_status gconn_server_destroy(gconn_server* s);

/* Per-phase device time of the static pipeline (gconn_cc, gconn_spanning_forest,
 * the initial graph of gconn_inc_create).  While profiling is enabled on the
 * calling thread, each phase is bracketed by HIP events recorded on the call's
 * own stream; gconn_profile_read waits for those events and adds up the
 * elapsed times (milliseconds).  Disabled by default. */
typedef struct gconn_phase_times {
  double init_ms;      /* control block, parent array, forest slots, hooks   */
  double sample_ms;    /* sampling kernels (k-out, hook-based, BFS levels)    */
  double compress_ms;  /* full compression after sampling                     */
  double lmax_ms;      /* most frequent label                                 */
  double gather_ms;    /* vertex gathering (active lists)                     */
  double finish_ms;    /* finish phase, every round included                  */
  double finalize_ms;  /* label finalisation (or ECL-CC's compress pass)      */
  uint64_t runs;       /* pipeline runs accumulated                           */
} gconn_phase_times;

/* on: 0 off; 1 every phase; otherwise a mask of the phases to bracket, bit
 * (p + 1) for the p-th field above (init = 0 ... finalize = 6), so a caller can
 * time one kernel with two events per run. */
gconn_status gconn_profile_enable(int on);
/* Fills *out with the totals since the last reset; reset = 1 clears them. */
gconn_status gconn_profile_read(gconn_phase_times* out, int reset);

/* Diagnostics: the chip's random-access ceilings, the yardstick of the union
 * passes (whose cost is the number of data-dependent 4-byte parent reads and
 * CASes the memory system serves per second, not streaming bandwidth).
 * Enqueues one kernel on `stream` that makes `accesses` (rounded down to a
 * multiple of 8 * lanes) random 4-byte accesses to table[0, words): kind 0
 * cached loads, 1 device-coherent loads, 2 CAS of each word's value to
 * itself (the table must hold table[i] == i, and is left unchanged).
 * sink (device, sink_words >= 256 entries) receives one word per lane;
 * lanes = sink_words rounded down to a multiple of 256.  words must be a power of
 * two.  Time it with events on the same stream. */
gconn_status gconn_diag_random_access(uint32_t* table, uint64_t words, int kind,
                                      uint64_t accesses, uint32_t* sink, uint32_t sink_words,
                                      void* stream);

const char* gconn_status_string(gconn_status s);
/* Message for the most recent failure on the calling thread ("" if none). */
const char* gconn_last_error(void);
/* Library version string. */
const char* gconn_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GCONN_H */
