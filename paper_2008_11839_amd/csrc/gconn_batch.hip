// gconn_batch.hip -- many independent graphs in one pipeline run, and the
// autotuner's timing step.
//
// The graphs are concatenated (global ids); graph boundaries are multiples of
// 64, so one wave iteration over 64 consecutive vertices belongs to one graph
// and reads its graph id once from a tile table.  The pipeline is the static
// one -- init, k-out sampling, L_max, compress + gather, union-find finish,
// finalisation -- run once for all graphs, with two per-graph differences: an
// L_max per graph (one workgroup samples each graph), and a sampling switch
// and union-find rule per graph class, selected at run time inside the kernels
// from a small table passed by value.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "gconn_device.hpp"
#include "gconn_internal.hpp"
#include "gconn_rules.hpp"

namespace gconn {

// Union-find rules available per class, by rule id: 0-2 Union-Async with
// FindNaive / FindSplit / FindHalve, 3-5 Union-Rem-CAS with SplitAtomicOne and
// those finds, 6-8 the same with HalveAtomicOne, 9-11 Union-Early, 12-14
// Union-Rem-CAS with Rem's SpliceAtomic (unions and finds are never concurrent
// in a batch run: sampling, gathering and finishing are separate kernels).

__device__ __forceinline__ bool unite_by_id(uint32_t rid, const LinkCtx& c, uint32_t u,
                                            uint32_t v) {
  switch (rid) {
    case 0: return Rule<kUnionAsync, kFindNaive, 0>::unite(c, u, v);
    case 1: return Rule<kUnionAsync, kFindSplit, 0>::unite(c, u, v);
    case 2: return Rule<kUnionAsync, kFindHalve, 0>::unite(c, u, v);
    case 3: return Rule<kUnionRemCas, kFindNaive, kSpliceSplitOne>::unite(c, u, v);
    case 4: return Rule<kUnionRemCas, kFindSplit, kSpliceSplitOne>::unite(c, u, v);
    case 5: return Rule<kUnionRemCas, kFindHalve, kSpliceSplitOne>::unite(c, u, v);
    case 6: return Rule<kUnionRemCas, kFindNaive, kSpliceHalveOne>::unite(c, u, v);
    case 7: return Rule<kUnionRemCas, kFindSplit, kSpliceHalveOne>::unite(c, u, v);
    case 8: return Rule<kUnionRemCas, kFindHalve, kSpliceHalveOne>::unite(c, u, v);
    case 9: return Rule<kUnionEarly, kFindNaive, 0>::unite(c, u, v);
    case 10: return Rule<kUnionEarly, kFindSplit, 0>::unite(c, u, v);
    case 11: return Rule<kUnionEarly, kFindHalve, 0>::unite(c, u, v);
    case 12: return Rule<kUnionRemCas, kFindNaive, kSpliceAtomic>::unite(c, u, v);
    case 13: return Rule<kUnionRemCas, kFindSplit, kSpliceAtomic>::unite(c, u, v);
    default: return Rule<kUnionRemCas, kFindHalve, kSpliceAtomic>::unite(c, u, v);
  }
}

struct BatchClass {
  uint32_t sample;  // 0 none, 1 k-out, 2 hook-based
  uint32_t rule;    // rule id
  uint32_t k;       // k-out: edges per vertex; hook-based: N, the edges of step 2
  uint32_t pad;
};
struct BatchClasses {
  BatchClass c[GCONN_MAX_CLASSES];
};

__device__ __forceinline__ const BatchClass& class_of(const BatchClasses& cl,
                                                      const uint8_t* graph_class, uint32_t g) {
  return cl.c[graph_class ? graph_class[g] : 0];
}

// tile t (64 vertices) -> graph id: a workgroup per graph writes its tiles
// (one thread per graph took a sequential pass over a million-vertex graph's
// 15,625 tiles)
__global__ void k_batch_tiles(const uint32_t* __restrict__ vbase, uint32_t G, uint32_t* tile_graph) {
  for (uint32_t g = blockIdx.x; g < G; g += gridDim.x) {
    const uint32_t lo = vbase[g] >> 6, hi = vbase[g + 1] >> 6;
    for (uint32_t t = lo + threadIdx.x; t < hi; t += blockDim.x) tile_graph[t] = g;
  }
}

__global__ void k_batch_sample(const uint64_t* __restrict__ off, const uint32_t* __restrict__ nbrs,
                               uint32_t n, const uint32_t* __restrict__ tile_graph,
                               const uint8_t* __restrict__ graph_class, BatchClasses cl, LinkCtx lc,
                               Ctrl* stats) {
  unsigned long long sampled = 0;
  // Tiles are visited in a scrambled order (odd multiplier modulo the next
  // power of two, out-of-range values skipped): the tiles of one small graph
  // would otherwise all run at the same moment, and its few smallest ids --
  // every vertex's first sampled neighbours -- would take all their CASes at
  // once.  Scrambled, a graph's unions spread over the whole launch.
  const uint64_t tiles = ((uint64_t)n + 63) >> 6;
  uint64_t span = 1;
  while (span < tiles) span <<= 1;
  constexpr uint64_t kNoTile = ~0ull;
  uint64_t t = wave_index();
  // next tile of this wave in the scrambled order (uniform over the wave)
  auto advance = [&]() -> uint64_t {
    while (t < span) {
      const uint64_t tile = (t * 0x9E3779B97F4A7C15ull) & (span - 1);
      t += wave_count();
      if (tile < tiles) return tile;
    }
    return kNoTile;
  };
  // a tile's graph, the lane's row bounds and first two neighbours: loaded for
  // the next tile before the current tile's unions run, so that they are in
  // flight together (the batch's n is a multiple of 64: every lane's vertex
  // exists, padding vertices have empty rows)
  struct Row {
    uint64_t b, d;
    uint32_t w0, w1, g;
  };
  auto fetch = [&](uint64_t tile, Row& r) {
    r.b = r.d = 0;
    r.w0 = r.w1 = r.g = 0;
    if (tile == kNoTile) return;
    const uint64_t v = (tile << 6) + lane();
    r.g = tile_graph[tile];
    r.b = off[v];
    r.d = off[v + 1] - r.b;
    if (r.d > 0) r.w0 = nbrs[r.b];
    if (r.d > 1) r.w1 = nbrs[r.b + 1];
  };
  uint64_t cur = advance();
  Row rc;
  fetch(cur, rc);
  while (cur != kNoTile) {
    const uint64_t nxt = advance();
    Row rn;
    fetch(nxt, rn);
    const BatchClass& bc = class_of(cl, graph_class, rc.g);
    if (bc.sample) {  // uniform over the wave: one graph per tile
      const uint64_t v = (cur << 6) + lane();
      uint32_t take = (uint32_t)(rc.d < bc.k ? rc.d : bc.k);
      // hook-based step 2: only the vertices step 1 left as roots (degree 0,
      // or first neighbour not smaller -- decided from the graph, not from P)
      if (bc.sample == 2 && (rc.d == 0 || rc.w0 < v)) take = 0;
      for (uint32_t j = 0; j < take; ++j) {
        const uint32_t w = j == 0 ? rc.w0 : j == 1 ? rc.w1 : nbrs[rc.b + j];
        unite_by_id(bc.rule, lc, (uint32_t)v, w);
      }
      sampled += take;
    }
    cur = nxt;
    rc = rn;
  }
  if (stats) {
    sampled = wave_sum(sampled);
    if (lane() == 0 && sampled) atomicAdd(&stats->stat_sampled, sampled);
  }
}

// Hook-based sampling, step 1, for the tiles of hook-based classes (Sampling
// Algorithms, HB): P[v] = min(v, first neighbour).  Every vertex is still a
// root and its lane the only writer of its slot, so this is a plain store.
__global__ void k_batch_hb1(const uint64_t* __restrict__ off, const uint32_t* __restrict__ nbrs,
                            uint32_t n, const uint32_t* __restrict__ tile_graph,
                            const uint8_t* __restrict__ graph_class, BatchClasses cl, uint32_t* P,
                            Ctrl* stats) {
  // four tiles per wave step: their graphs and classes are looked up
  // together (the lookups are uniform over the wave), then the hook-based
  // tiles among them do their one store per vertex
  unsigned long long took = 0, linked = 0;
  const uint64_t tiles = (uint64_t)n >> 6;  // n is a multiple of 64
  for (uint64_t t0 = wave_index() * 4; t0 < tiles; t0 += wave_count() * 4) {
    uint32_t g[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) g[j] = t0 + j < tiles ? tile_graph[t0 + j] : 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (t0 + j >= tiles || class_of(cl, graph_class, g[j]).sample != 2) continue;  // uniform
      const uint64_t v = ((t0 + j) << 6) + lane();
      const uint64_t b = off[v];
      if (off[v + 1] > b) {
        ++took;
        const uint32_t w = nbrs[b];
        if (w < v) {
          P[v] = w;
          ++linked;
        }
      }
    }
  }
  if (stats) {
    took = wave_sum(took);
    linked = wave_sum(linked);
    if (lane() == 0) {
      if (took) atomicAdd(&stats->stat_sampled, took);
      if (linked) atomicAdd(&stats->stat_hooks, linked);
    }
  }
}

// One workgroup per graph: the most frequent root over a seeded sample of the
// graph's vertices (smallest label on ties), or none without sampling.
constexpr uint32_t kBatchLmaxTable = 2 * kMaxLmaxSamples;
__global__ void __launch_bounds__(1024) k_batch_lmax(const uint32_t* P,
                                                     const uint32_t* __restrict__ vbase,
                                                     const uint8_t* __restrict__ graph_class,
                                                     BatchClasses cl, uint32_t samples,
                                                     uint64_t seed, uint32_t* lmax) {
  __shared__ uint32_t keys[kBatchLmaxTable];
  __shared__ uint32_t cnts[kBatchLmaxTable];
  __shared__ unsigned long long best;
  const uint32_t g = blockIdx.x;
  const uint32_t lo = vbase[g], ng = vbase[g + 1] - lo;
  if (!class_of(cl, graph_class, g).sample || ng == 0) {
    if (threadIdx.x == 0) lmax[g] = kEmpty;
    return;
  }
  for (uint32_t i = threadIdx.x; i < kBatchLmaxTable; i += blockDim.x) {
    keys[i] = kEmpty;
    cnts[i] = 0;
  }
  if (threadIdx.x == 0) best = 0;
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < samples; j += blockDim.x) {
    const uint32_t hi = (uint32_t)(splitmix64_at(seed, j) >> 32);
    const uint32_t v = lo + (uint32_t)(((uint64_t)hi * ng) >> 32);
    const uint32_t label = root_plain(P, v);
    uint32_t h = (label * 2654435761u) & (kBatchLmaxTable - 1);
    for (;;) {
      const uint32_t prev = atomicCAS(&keys[h], kEmpty, label);
      if (prev == kEmpty || prev == label) {
        atomicAdd(&cnts[h], 1u);
        break;
      }
      h = (h + 1) & (kBatchLmaxTable - 1);
    }
  }
  __syncthreads();
  unsigned long long mine = 0;
  for (uint32_t i = threadIdx.x; i < kBatchLmaxTable; i += blockDim.x)
    if (keys[i] != kEmpty) {
      const unsigned long long key = ((unsigned long long)cnts[i] << 32) | (kEmpty - keys[i]);
      mine = key > mine ? key : mine;
    }
  mine = wave_max(mine);
  if (lane() == 0) atomicMax(&best, mine);
  __syncthreads();
  if (threadIdx.x == 0) lmax[g] = best ? kEmpty - (uint32_t)(best & 0xFFFFFFFFu) : kEmpty;
}

// Compress (sampled classes) + vertex gathering against the graph's own L_max.
__global__ void k_batch_gather(const uint64_t* __restrict__ off, uint32_t* P, uint32_t n,
                               const uint32_t* __restrict__ tile_graph,
                               const uint8_t* __restrict__ graph_class, BatchClasses cl,
                               const uint32_t* __restrict__ lmax, Ctrl* c, WorkLists wl,
                               int want_stats) {
  // Four consecutive vertices per lane (one tile, so one graph): their row
  // bounds and parents are loaded together and their root walks advance in
  // lockstep, so a wave keeps several independent loads in flight.  L is the
  // root of the graph's largest sampled tree (k_batch_lmax walked to it and
  // no link runs before the finish), so a walk that reaches it stops there.
  // The work-list appends then go tile by tile, 64 consecutive vertices per
  // append as the finish expects (its lanes read consecutive rows): lane l
  // takes vertex 64 j + l of the wave's four tiles from the lane holding it.
  unsigned long long act = 0, edges = 0;
  for (uint64_t base = wave_base() * 4; base < n; base += wave_stride() * 4) {
    const uint64_t v0 = base + 4 * lane();
    const bool live = v0 < n;  // n is a multiple of 64: then v0 + 3 < n too
    const uint32_t g = live ? tile_graph[v0 >> 6] : 0u;
    const bool sampled = live && class_of(cl, graph_class, g).sample != 0;
    const uint32_t L = live ? lmax[g] : kEmpty;
    uint64_t o[5];
    uint32_t p[4], r[4];
#pragma unroll
    for (int j = 0; j < 5; ++j) o[j] = live ? off[v0 + j] : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      p[j] = sampled ? P[v0 + j] : (uint32_t)(v0 + j);
      r[j] = p[j];
    }
    bool walk[4], more = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      walk[j] = sampled && p[j] != v0 + j && p[j] != L;
      more = more || walk[j];
    }
    while (more) {
      more = false;
      uint32_t q[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) q[j] = walk[j] ? P[r[j]] : r[j];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (walk[j]) {
          if (q[j] == r[j]) {
            walk[j] = false;
          } else {
            r[j] = q[j];
            walk[j] = q[j] != L;
          }
        }
        more = more || walk[j];
      }
    }
    uint32_t degs[4], act_mask = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (live && r[j] != p[j]) P[v0 + j] = r[j];
      degs[j] = live ? (uint32_t)(o[j + 1] - o[j]) : 0u;
      if (degs[j] > 0 && r[j] != L) act_mask |= 1u << j;
    }
    const uint32_t src_k = lane() & 3;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const uint32_t from = 16 * t + (lane() >> 2);  // the lane holding vertex 64 t + lane
      uint32_t d = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t x = __shfl(degs[j], from);
        d = src_k == (uint32_t)j ? x : d;
      }
      const bool active = (__shfl(act_mask, from) >> src_k) & 1u;
      const uint64_t v = base + 64 * t + lane();
      wl_push(wl, c, (base >> 6) + t, (uint32_t)v, d, active);
      act += active ? 1 : 0;
      edges += active ? d : 0;
    }
  }
  if (want_stats) {
    act = wave_sum(act);
    edges = wave_sum(edges);
    if (lane() == 0) {
      if (act) atomicAdd(&c->stat_active, act);
      if (edges) atomicAdd(&c->stat_finish_edges, edges);
    }
  }
}

__global__ void k_batch_finish(const uint64_t* __restrict__ off, const uint32_t* __restrict__ nbrs,
                               WorkLists wl, const Ctrl* c, const uint32_t* __restrict__ tile_graph,
                               const uint8_t* __restrict__ graph_class, BatchClasses cl,
                               LinkCtx lc) {
  __shared__ uint32_t pre_s[kSubLists + 1], pre_m[kSubLists + 1];
  wl_prefix(c->small_cnt, pre_s);
  wl_prefix(c->medium_cnt, pre_m);
  __syncthreads();
  const uint32_t S = pre_s[kSubLists], M = pre_m[kSubLists], G = c->seg_count;
  for (uint64_t i = gtid(); i < S; i += wave_stride()) {
    const uint32_t u = wl_get(wl.small, wl.cap, pre_s, (uint32_t)i);
    const uint32_t rid = class_of(cl, graph_class, tile_graph[u >> 6]).rule;
    const uint64_t e = off[u + 1];
    for (uint64_t x = off[u]; x < e; ++x) unite_by_id(rid, lc, u, nbrs[x]);
  }
  for (uint64_t w = wave_index(); w < M; w += wave_count()) {
    const uint32_t u = wl_get(wl.medium, wl.cap, pre_m, (uint32_t)w);
    const uint32_t rid = class_of(cl, graph_class, tile_graph[u >> 6]).rule;
    const uint64_t e = off[u + 1];
    for (uint64_t x = off[u] + lane(); x < e; x += 64) unite_by_id(rid, lc, u, nbrs[x]);
  }
  for (uint64_t s = wave_index(); s < G; s += wave_count()) {
    const uint2 sg = wl.segs[s];
    const uint32_t rid = class_of(cl, graph_class, tile_graph[sg.x >> 6]).rule;
    const uint64_t b = off[sg.x] + (uint64_t)sg.y * kSeg;
    uint64_t e = off[sg.x + 1];
    if (e > b + kSeg) e = b + kSeg;
    for (uint64_t x = b + lane(); x < e; x += 64) unite_by_id(rid, lc, sg.x, nbrs[x]);
  }
}

// labels_out[v] = root(v) - vbase[g]: per-graph local labels.
// Four tiles per wave step, a vertex of each per lane, their root walks in
// lockstep; the batch's n is a multiple of 64.
__global__ void k_batch_finalize(const uint32_t* P, uint32_t n,
                                 const uint32_t* __restrict__ tile_graph,
                                 const uint32_t* __restrict__ vbase, uint32_t* out) {
  const uint64_t tiles = (uint64_t)n >> 6;
  for (uint64_t t0 = wave_index() * 4; t0 < tiles; t0 += wave_count() * 4) {
    uint32_t lo[4], r[4];
    uint64_t v[4];
    bool live[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      live[j] = t0 + j < tiles;  // uniform over the wave
      v[j] = ((t0 + j) << 6) + lane();
      lo[j] = live[j] ? vbase[tile_graph[t0 + j]] : 0u;
      r[j] = live[j] ? P[v[j]] : 0u;
    }
    bool more = true;
    while (more) {
      more = false;
      uint32_t q[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) q[j] = live[j] ? P[r[j]] : r[j];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (q[j] != r[j]) {
          r[j] = q[j];
          more = true;
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (live[j]) out[v[j]] = r[j] - lo[j];
  }
}

namespace {

struct BatchLayout {
  size_t ctrl = 0, P = 0, tiles = 0, lmax = 0, small = 0, medium = 0, segs = 0, total = 0;
  uint32_t sub_cap = 0;
};

BatchLayout plan_batch(const gconn_batch& b) {
  BatchLayout L;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t p = at;
    at = align_up(at + (bytes ? bytes : 1), 256);
    return p;
  };
  const uint64_t n = b.n, m = b.m;
  L.ctrl = take(sizeof(Ctrl));
  L.P = take(4 * n);
  L.tiles = take(4 * (n / 64 + 1));
  L.lmax = take(4ull * b.num_graphs);
  const uint64_t groups = (n + 63) / 64;
  L.sub_cap = (uint32_t)(((groups + kSubLists - 1) / kSubLists + 1) * 64);
  L.small = take(4ull * kSubLists * L.sub_cap);
  L.medium = take(4ull * kSubLists * L.sub_cap);
  L.segs = take(8 * (2 * m / kSeg + 1));
  L.total = at;
  return L;
}

gconn_status rule_id(const gconn_class_options& c, uint32_t* rid) {
  int f = c.find;
  if (f < GCONN_FIND_NAIVE || f > GCONN_FIND_HALVE)
    return fail(GCONN_EUNSUPPORTED, "batched classes use FindNaive, FindSplit or FindHalve");
  switch (c.link) {
    case GCONN_LINK_ASYNC: *rid = (uint32_t)f; return GCONN_OK;
    case GCONN_LINK_REM_CAS:
      if (c.splice == GCONN_SPLICE_ATOMIC) {
        *rid = 12 + (uint32_t)f;
        return GCONN_OK;
      }
      if (c.splice != GCONN_SPLICE_SPLIT_ONE && c.splice != GCONN_SPLICE_HALVE_ONE)
        return fail(GCONN_EINVAL, "class splice out of range");
      *rid = 3 + (c.splice == GCONN_SPLICE_HALVE_ONE ? 3u : 0u) + (uint32_t)f;
      return GCONN_OK;
    case GCONN_LINK_EARLY: *rid = 9 + (uint32_t)f; return GCONN_OK;
    default:
      return fail(GCONN_EUNSUPPORTED, "batched classes use Union-Async, Union-Rem-CAS or Union-Early");
  }
}

gconn_status check_batch(const gconn_batch* b) {
  if (!b) return fail(GCONN_EINVAL, "batch is NULL");
  if (b->num_graphs == 0) return fail(GCONN_EINVAL, "batch has no graphs");
  if (b->n % 64 != 0) return fail(GCONN_EINVAL, "batch n must be a multiple of 64 (pad graphs)");
  if (b->n > 0xFFFFFFC0u) return fail(GCONN_EINVAL, "batch n too large");
  if (b->n > 0) GCONN_TRY(check_device_ptr(b->offsets, "batch.offsets"));
  if (b->m > 0) GCONN_TRY(check_device_ptr(b->nbrs, "batch.nbrs"));
  GCONN_TRY(check_device_ptr(b->vbase, "batch.vbase"));
  if (b->graph_class) GCONN_TRY(check_device_ptr(b->graph_class, "batch.graph_class"));
  if (b->block != 0 && (b->block < 64 || b->block > 1024 || b->block % 64 != 0))
    return fail(GCONN_EINVAL, "batch.block must be 0 or a multiple of 64 in [64, 1024]");
  return GCONN_OK;
}

}  // namespace

gconn_status batch_workspace_size(const gconn_batch* b, size_t* bytes) {
  if (!b || !bytes) return fail(GCONN_EINVAL, "batch or bytes is NULL");
  *bytes = plan_batch(*b).total;
  return GCONN_OK;
}

gconn_status run_batch(const gconn_batch* b, uint32_t* labels_out, void* workspace,
                       size_t workspace_bytes, const gconn_class_options* classes,
                       uint32_t num_classes, uint32_t lmax_samples, uint64_t seed,
                       gconn_stats* stats, hipStream_t s) {
  GCONN_TRY(check_device_ready());
  GCONN_TRY(check_batch(b));
  if (!classes || num_classes == 0 || num_classes > GCONN_MAX_CLASSES)
    return fail(GCONN_EINVAL, "classes must hold 1..64 entries");
  if (lmax_samples < 1 || lmax_samples > kMaxLmaxSamples)
    return fail(GCONN_EINVAL, "lmax_samples must be in [1, 4096]");
  BatchClasses cl;
  std::memset(&cl, 0, sizeof(cl));
  for (uint32_t i = 0; i < num_classes; ++i) {
    const gconn_class_options& c = classes[i];
    if (c.sample != GCONN_SAMPLE_NONE && c.sample != GCONN_SAMPLE_KOUT &&
        c.sample != GCONN_SAMPLE_HB)
      return fail(GCONN_EUNSUPPORTED, "batched classes sample with k-out, hook-based or not at all");
    if (c.sample != GCONN_SAMPLE_NONE && (c.k < 1 || c.k > 64))
      return fail(GCONN_EINVAL, "class k (k-out edges, or hook-based N) must be in [1, 64]");
    cl.c[i].sample = c.sample == GCONN_SAMPLE_KOUT ? 1u : c.sample == GCONN_SAMPLE_HB ? 2u : 0u;
    cl.c[i].k = c.k;
    GCONN_TRY(rule_id(c, &cl.c[i].rule));
  }
  if (b->n > 0) GCONN_TRY(check_device_ptr(labels_out, "labels_out"));
  const BatchLayout L = plan_batch(*b);
  if (workspace_bytes < L.total)
    return fail(GCONN_ENOMEM, "workspace has " + std::to_string(workspace_bytes) +
                                  " bytes, needs " + std::to_string(L.total));
  GCONN_TRY(check_device_ptr(workspace, "workspace"));
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(GCONN_EINVAL, "workspace must be 256-byte aligned");

  uint8_t* ws = static_cast<uint8_t*>(workspace);
  Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
  uint32_t* P = reinterpret_cast<uint32_t*>(ws + L.P);
  uint32_t* tiles = reinterpret_cast<uint32_t*>(ws + L.tiles);
  uint32_t* lmax = reinterpret_cast<uint32_t*>(ws + L.lmax);
  WorkLists wl;
  wl.small = reinterpret_cast<uint32_t*>(ws + L.small);
  wl.medium = reinterpret_cast<uint32_t*>(ws + L.medium);
  wl.segs = reinterpret_cast<uint2*>(ws + L.segs);
  wl.cap = L.sub_cap;
  LinkCtx lc;
  lc.P = P;
  lc.H = nullptr;
  lc.fu = lc.fv = nullptr;
  lc.hooks = stats ? &ctrl->stat_hooks : nullptr;
  lc.atomic_compress = 1;  // compression writes are CAS in the batch
  Ctrl* st = stats ? ctrl : nullptr;
  const uint32_t n = b->n, G = b->num_graphs, block = b->block ? b->block : 256;

  GCONN_TRY(reset_ctrl_and_parents(ctrl, P, n, s));
  k_batch_tiles<<<std::max<uint32_t>(1, std::min<uint32_t>(G, 65535)), 256, 0, s>>>(b->vbase, G,
                                                                                   tiles);
  GCONN_LAUNCHED("k_batch_tiles");
  if (n > 0 && b->m > 0) {
    bool any_hb = false;
    for (uint32_t i = 0; i < num_classes; ++i) any_hb = any_hb || cl.c[i].sample == 2;
    if (any_hb) {
      k_batch_hb1<<<std::min<uint32_t>(grid_for(n / 4, block), 8192), block, 0, s>>>(
          b->offsets, b->nbrs, n, tiles, b->graph_class, cl, P, st);
      GCONN_LAUNCHED("k_batch_hb1");
    }
    const uint32_t sgrid = persistent_grid(k_batch_sample, block);
    k_batch_sample<<<sgrid, block, 0, s>>>(b->offsets, b->nbrs, n, tiles, b->graph_class, cl, lc, st);
    GCONN_LAUNCHED("k_batch_sample");
    k_batch_lmax<<<G, 1024, 0, s>>>(P, b->vbase, b->graph_class, cl, lmax_samples, seed, lmax);
    GCONN_LAUNCHED("k_batch_lmax");
    k_batch_gather<<<grid_for(n / 4, block), block, 0, s>>>(b->offsets, P, n, tiles, b->graph_class, cl,
                                                      lmax, ctrl, wl, stats ? 1 : 0);
    GCONN_LAUNCHED("k_batch_gather");
    const uint32_t fgrid = persistent_grid(k_batch_finish, block);
    k_batch_finish<<<fgrid, block, 0, s>>>(b->offsets, b->nbrs, wl, ctrl, tiles, b->graph_class, cl,
                                          lc);
    GCONN_LAUNCHED("k_batch_finish");
  }
  if (n > 0) {
    k_batch_finalize<<<grid_for(n / 4, block), block, 0, s>>>(P, n, tiles, b->vbase, labels_out);
    GCONN_LAUNCHED("k_batch_finalize");
  }
  if (stats) {
    Ctrl h;
    GCONN_HIP(hipMemcpyAsync(&h, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    GCONN_HIP(hipStreamSynchronize(s));
    std::memset(stats, 0, sizeof(*stats));
    stats->sampled_edges = h.stat_sampled;
    stats->active_vertices = h.stat_active;
    stats->finish_edges = h.stat_finish_edges;
    stats->hooks = h.stat_hooks;
    stats->lmax = 0xFFFFFFFFu;
    stats->bfs_source = 0xFFFFFFFFu;
  }
  return GCONN_OK;
}

gconn_status autotune(const gconn_graph* graphs, uint32_t num_graphs,
                      const gconn_options* candidates, uint32_t num_candidates, uint32_t reps,
                      uint32_t* labels_scratch, void* workspace, size_t workspace_bytes,
                      hipStream_t s, uint32_t* best, double* times_ms) {
  if (!graphs || num_graphs == 0 || !candidates || num_candidates == 0 || !best)
    return fail(GCONN_EINVAL, "graphs, candidates and best are required");
  if (reps == 0) reps = 1;
  hipEvent_t a = nullptr, z = nullptr;
  GCONN_HIP(hipEventCreate(&a));
  GCONN_HIP(hipEventCreate(&z));
  double best_ms = 0;
  gconn_status st = GCONN_OK;
  for (uint32_t c = 0; c < num_candidates && st == GCONN_OK; ++c) {
    double total = 0;
    for (uint32_t gi = 0; gi < num_graphs && st == GCONN_OK; ++gi) {
      st = gconn_cc(&graphs[gi], labels_scratch, workspace, workspace_bytes, &candidates[c],
                    nullptr, s);  // warm-up
      if (st != GCONN_OK) break;
      if (hipEventRecord(a, s) != hipSuccess) { st = hip_fail(hipGetLastError(), "hipEventRecord"); break; }
      for (uint32_t r = 0; r < reps && st == GCONN_OK; ++r)
        st = gconn_cc(&graphs[gi], labels_scratch, workspace, workspace_bytes, &candidates[c],
                      nullptr, s);
      if (st != GCONN_OK) break;
      float ms = 0;
      if (hipEventRecord(z, s) != hipSuccess || hipEventSynchronize(z) != hipSuccess ||
          hipEventElapsedTime(&ms, a, z) != hipSuccess) {
        st = hip_fail(hipGetLastError(), "autotune timing");
        break;
      }
      total += ms;
    }
    if (st != GCONN_OK) break;
    if (times_ms) times_ms[c] = total;
    if (c == 0 || total < best_ms) {
      best_ms = total;
      *best = c;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(z);
  return st;
}

}  // namespace gconn
