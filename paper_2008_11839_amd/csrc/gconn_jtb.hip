// gconn_jtb.hip -- static and incremental connectivity with Union-JTB
// (randomized linking by rank over 64-bit (rank, parent) words; the rule is in
// gconn_jtb.hpp).  The pipeline follows the static algorithm (Alg. "GConn for
// Static Connectivity"): k-out sampling with the same union rule, flattening
// and L_max, the finish over the vertices whose root is not L_max, then
// canonical labels.  Because linking by rank does not keep the smallest id at
// the root, the last step reduces every component to its minimum vertex.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "gconn_device.hpp"
#include "gconn_jtb.hpp"

namespace gconn {

namespace {

// Root of x by pointer jumping over the words, after a kernel boundary (no
// concurrent links).
__device__ __forceinline__ uint32_t jtb_root_plain(const uint64_t* W, uint32_t x) {
  uint32_t p = jtb_parent(W[x]);
  while (p != x) {
    x = p;
    p = jtb_parent(W[x]);
  }
  return x;
}

// Clears the control block (block 0) and makes every vertex a rank-0 root;
// empties the forest slots when they are given; sets M to the identity when
// it is given (the component minima of the final labelling start there).
__global__ void k_jtb_init(Ctrl* c, uint64_t* W, uint32_t n, uint32_t* fu, uint32_t* fv,
                           uint32_t* M) {
  if (c && blockIdx.x == 0) {
    uint32_t* w = reinterpret_cast<uint32_t*>(c);
    for (uint32_t i = threadIdx.x; i < sizeof(Ctrl) / 4; i += blockDim.x) w[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
      c->lmax = kEmpty;
      c->bfs_source = kEmpty;
      c->comp_min = kEmpty;
    }
  }
  for (uint64_t v = gtid(); v < n; v += wave_stride()) {
    W[v] = jtb_word((uint32_t)v, 0);
    if (M) M[v] = (uint32_t)v;
    if (fu) {
      fu[v] = kEmpty;
      fv[v] = kEmpty;
    }
  }
}

// k-out sampling (Alg. k-out sampling) with Union-JTB: every vertex unites
// with its first k neighbours, or with its first one and k - 1 picks drawn
// uniformly from its row by SplitMix64 (one lane per vertex).
template <int F, typename OffT>
__global__ void k_jtb_kout(const OffT* __restrict__ off, const uint32_t* __restrict__ nbrs,
                           uint32_t n, uint32_t k, int random, uint64_t seed, JtbCtx c,
                           Ctrl* stats) {
  for (uint64_t base = wave_base(); base < n; base += wave_stride()) {
    const uint64_t v = base + lane();
    uint32_t took = 0;
    if (v < n) {
      const uint64_t b = off[v], deg = (uint64_t)off[v + 1] - b;
      took = (uint32_t)(deg < k ? deg : k);
      for (uint32_t j = 0; j < took; ++j) {
        uint64_t x = b + j;
        if (random && j > 0) {
          const uint64_t r = splitmix64_at(seed, v * (uint64_t)k + j) >> 32;
          x = b + ((r * deg) >> 32);
        }
        jtb_unite<F>(c, (uint32_t)v, nbrs[x]);
      }
    }
    if (stats) {
      const unsigned long long s = wave_sum(took);
      if (lane() == 0 && s) atomicAdd(&stats->stat_sampled, s);
    }
  }
}

// Full compression into a separate array: R[v] = root(v).
__global__ void k_jtb_flatten(const uint64_t* W, uint32_t* R, uint32_t n) {
  for (uint64_t v = gtid(); v < n; v += wave_stride()) R[v] = jtb_root_plain(W, (uint32_t)v);
}

// GetMostFrequentLabel over the flat roots R: the same seeded vertex sample
// as the 32-bit pipeline; the mode wins, the smallest root on ties.  One
// block; every thread counts how often its sample's root occurs among all
// samples (samples <= 4096, so at most 16M comparisons from LDS).
__global__ void __launch_bounds__(1024) k_jtb_lmax(const uint32_t* R, uint32_t n, uint32_t samples,
                                                   uint64_t seed, Ctrl* c) {
  __shared__ uint32_t lab[kMaxLmaxSamples];
  __shared__ unsigned long long best;
  if (threadIdx.x == 0) best = 0;
  for (uint32_t j = threadIdx.x; j < samples; j += blockDim.x) {
    const uint32_t hi = (uint32_t)(splitmix64_at(seed, j) >> 32);
    lab[j] = R[((uint64_t)hi * n) >> 32];
  }
  __syncthreads();
  unsigned long long mine = 0;
  for (uint32_t j = threadIdx.x; j < samples; j += blockDim.x) {
    uint32_t cnt = 0;
    for (uint32_t i = 0; i < samples; ++i) cnt += lab[i] == lab[j] ? 1u : 0u;
    const unsigned long long key = ((unsigned long long)cnt << 32) | (kEmpty - lab[j]);
    mine = key > mine ? key : mine;
  }
  mine = wave_max(mine);
  if (lane() == 0) atomicMax(&best, mine);
  __syncthreads();
  if (threadIdx.x == 0 && best) c->lmax = kEmpty - (uint32_t)(best & 0xFFFFFFFFu);
}

// Vertex gathering: active = degree > 0 and (no sampling, or root != L_max).
// One lane per vertex; the active vertices go to the degree-class work lists.
template <typename OffT>
__global__ void k_jtb_gather(const OffT* __restrict__ off, const uint32_t* R, uint32_t n, Ctrl* c,
                             WorkLists wl, int sampled, int want_stats) {
  const uint32_t lmax = sampled ? c->lmax : kEmpty;
  unsigned long long act = 0, edges = 0;
  for (uint64_t base = wave_base(); base < n; base += wave_stride()) {
    const uint64_t v = base + lane();
    const bool valid = v < n;
    const uint64_t deg = valid ? (uint64_t)off[v + 1] - off[v] : 0;
    const bool active = valid && deg > 0 && (!sampled || R[v] != lmax);
    wl_push(wl, c, base >> 6, (uint32_t)v, deg, active);
    act += active ? 1 : 0;
    edges += active ? deg : 0;
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

// Finish (Alg. union-find meta-algorithm) over the work lists: small vertices
// one lane each, medium vertices one wave each, hub segments one wave each.
template <int F, typename OffT>
__global__ void k_jtb_finish(const OffT* __restrict__ off, const uint32_t* __restrict__ nbrs,
                             WorkLists wl, const Ctrl* c, JtbCtx jc) {
  __shared__ uint32_t pre_s[kSubLists + 1], pre_m[kSubLists + 1];
  wl_prefix(c->small_cnt, pre_s);
  wl_prefix(c->medium_cnt, pre_m);
  __syncthreads();
  const uint32_t S = pre_s[kSubLists], M = pre_m[kSubLists], G = c->seg_count;
  for (uint64_t i = gtid(); i < S; i += wave_stride()) {
    const uint32_t u = wl_get(wl.small, wl.cap, pre_s, (uint32_t)i);
    const uint64_t e = off[u + 1];
    for (uint64_t x = off[u]; x < e; ++x) jtb_unite<F>(jc, u, nbrs[x]);
  }
  for (uint64_t w = wave_index(); w < M; w += wave_count()) {
    const uint32_t u = wl_get(wl.medium, wl.cap, pre_m, (uint32_t)w);
    const uint64_t e = off[u + 1];
    for (uint64_t x = off[u] + lane(); x < e; x += 64) jtb_unite<F>(jc, u, nbrs[x]);
  }
  for (uint64_t s = wave_index(); s < G; s += wave_count()) {
    const uint2 sg = wl.segs[s];
    const uint64_t b = (uint64_t)off[sg.x] + (uint64_t)sg.y * kSeg;
    uint64_t e = off[sg.x + 1];
    if (e > b + kSeg) e = b + kSeg;
    for (uint64_t x = b + lane(); x < e; x += 64) jtb_unite<F>(jc, sg.x, nbrs[x]);
  }
}

// One union per pair (COO finish, incremental inserts).
template <int F>
__global__ void k_jtb_pairs(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b,
                            uint64_t m, JtbCtx jc) {
  for (uint64_t e = gtid(); e < m; e += wave_stride()) jtb_unite<F>(jc, a[e], b[e]);
}

template <int F>
__global__ void k_jtb_unite_kind(const uint8_t* __restrict__ kind, const uint32_t* __restrict__ a,
                                 const uint32_t* __restrict__ b, uint64_t m, JtbCtx jc) {
  for (uint64_t e = gtid(); e < m; e += wave_stride())
    if (kind[e] == GCONN_REQ_INSERT) jtb_unite<F>(jc, a[e], b[e]);
}

// Connectivity queries: out[i] = find(a[i]) == find(b[i]).  kind: nullable;
// when given, only entries of kind "query" are answered (0 for the others).
template <int F>
__global__ void k_jtb_query(const uint8_t* __restrict__ kind, const uint32_t* __restrict__ a,
                            const uint32_t* __restrict__ b, uint64_t q, uint64_t* W, uint8_t* out) {
  for (uint64_t i = gtid(); i < q; i += wave_stride()) {
    uint8_t r = 0;
    if (!kind || kind[i] == GCONN_REQ_QUERY) {
      uint64_t wa, wb;
      r = (uint8_t)(jtb_find<F>(W, a[i], kNoWord, &wa) == jtb_find<F>(W, b[i], kNoWord, &wb));
    }
    out[i] = r;
  }
}

// Canonical labels, pass 1: L[v] = root(v), and M[r] = the minimum over the
// component of root r (M starts as the identity).  Only vertices below their
// root can lower M[r].  In a wave, the lowest such lane of each root holds
// that root's smallest id in the wave (ids rise with the lane), so one lane
// per distinct root writes; it skips the atomic when M[r] is already at most
// its id (M only decreases, so any value read is an upper bound of the current
// one).  The grid runs roughly in id order, so the giant component's minimum
// lands early and later waves skip.
__global__ void k_jtb_roots_min(const uint64_t* W, uint32_t* L, uint32_t* M, uint32_t n) {
  for (uint64_t base = wave_base(); base < n; base += wave_stride()) {
    const uint64_t v = base + lane();
    uint32_t r = 0;
    if (v < n) {
      r = jtb_root_plain(W, (uint32_t)v);
      L[v] = r;
    }
    bool pending = v < n && v < r;
    unsigned long long mask = __ballot(pending);
    while (mask) {
      const uint32_t leader = __ffsll(mask) - 1;
      const uint32_t root = __shfl(r, leader);
      if (lane() == leader && ld(&M[root]) > (uint32_t)v) amin(&M[root], (uint32_t)v);
      if (pending && r == root) pending = false;
      mask = __ballot(pending);
    }
  }
}

// Pass 2: L[v] = M[L[v]].
__global__ void k_jtb_relabel(uint32_t* L, const uint32_t* M, uint32_t n) {
  for (uint64_t v = gtid(); v < n; v += wave_stride()) L[v] = M[L[v]];
}

template <class Fn>
gconn_status with_jtb_find(int find_rule, Fn&& fn) {
  if (find_rule == GCONN_FIND_TWO_TRY_SPLIT)
    return fn(std::integral_constant<int, kJtbFindTwoTrySplit>{});
  return fn(std::integral_constant<int, kJtbFindSimple>{});
}

// M: n entries; m_ready: M already holds the identity (else it is set here).
gconn_status jtb_labels(const uint64_t* W, uint32_t n, uint32_t* labels, uint32_t* M, uint32_t block,
                        bool m_ready, hipStream_t s) {
  const uint32_t grid = grid_for(n, block);
  if (!m_ready) GCONN_TRY(launch_iota(M, n, s));
  k_jtb_roots_min<<<grid, block, 0, s>>>(W, labels, M, n);
  GCONN_LAUNCHED("k_jtb_roots_min");
  k_jtb_relabel<<<grid, block, 0, s>>>(labels, M, n);
  GCONN_LAUNCHED("k_jtb_relabel");
  return GCONN_OK;
}

// Salt of the tie-breaking keys: the high half of SplitMix64's first output
// for the seed.
uint32_t jtb_salt(uint64_t seed) {
  uint64_t z = seed + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return (uint32_t)((z ^ (z >> 31)) >> 32);
}

}  // namespace

WsLayout plan_workspace_jtb(const gconn_graph& g, const gconn_options& o, bool forest,
                            bool labels) {
  (void)o;
  WsLayout L;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t p = at;
    at = align_up(at + (bytes ? bytes : 1), 256);
    return p;
  };
  const uint64_t n = g.n, m = g.m;
  L.ctrl = take(sizeof(Ctrl));
  if (forest && !labels) L.P = take(4 * n);
  L.words = take(8 * n);
  L.roots = take(4 * n);
  if (labels) L.mins = take(4 * n);
  if (g.format == GCONN_CSR) {
    // one push call per 64-vertex group; group g goes to sub-list g % kSubLists
    const uint64_t groups = (n + 63) / 64;
    L.sub_cap = (uint32_t)(((groups + kSubLists - 1) / kSubLists + 1) * 64);
    L.small = take(4ull * kSubLists * L.sub_cap);
    L.medium = take(4ull * kSubLists * L.sub_cap);
    L.seg_cap = 2 * m / kSeg + 1;
    L.segs = take(8 * L.seg_cap);
  }
  L.total = at;
  return L;
}

gconn_status run_static_jtb(const gconn_graph& g, uint32_t* P, uint32_t* fu, uint32_t* fv,
                            bool finalize, uint8_t* ws, const WsLayout& L, const gconn_options& o,
                            gconn_stats* stats, hipStream_t s, uint64_t* words) {
  const uint32_t n = g.n;
  const uint32_t block = (uint32_t)o.block;
  Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
  uint64_t* W = words ? words : reinterpret_cast<uint64_t*>(ws + L.words);
  uint32_t* R = reinterpret_cast<uint32_t*>(ws + L.roots);
  JtbCtx jc{W, fu, fv, stats ? &ctrl->stat_hooks : nullptr, jtb_salt(o.seed)};
  const bool csr = g.format == GCONN_CSR;
  const bool sampled = csr && o.sample == GCONN_SAMPLE_KOUT;
  prof_count_run();
  GCONN_TRY(prof_mark(kPhaseInit, true, s));
  uint32_t* M = finalize ? reinterpret_cast<uint32_t*>(ws + L.mins) : nullptr;
  k_jtb_init<<<grid_for(std::max<uint32_t>(n, 1), block), block, 0, s>>>(ctrl, W, n, fu, fv, M);
  GCONN_LAUNCHED("k_jtb_init");
  GCONN_TRY(prof_mark(kPhaseInit, false, s));
  if (o.validate && (g.m > 0 || csr)) GCONN_TRY(validate_graph(g, ctrl, block, s));
  if (n > 0 && g.m > 0) {
    GCONN_TRY(with_jtb_find(o.find, [&](auto fc) -> gconn_status {
      constexpr int F = decltype(fc)::value;
      if (!csr) {
        GCONN_TRY(prof_mark(kPhaseFinish, true, s));
        k_jtb_pairs<F><<<grid_for(g.m, block), block, 0, s>>>(g.nbrs, g.dst, g.m, jc);
        GCONN_LAUNCHED("k_jtb_pairs");
        return prof_mark(kPhaseFinish, false, s);
      }
      WorkLists wl;
      wl.small = reinterpret_cast<uint32_t*>(ws + L.small);
      wl.medium = reinterpret_cast<uint32_t*>(ws + L.medium);
      wl.segs = reinterpret_cast<uint2*>(ws + L.segs);
      wl.cap = L.sub_cap;
      auto body = [&](auto* off) -> gconn_status {
        using OffT = std::remove_const_t<std::remove_pointer_t<decltype(off)>>;
        if (sampled) {
          GCONN_TRY(prof_mark(kPhaseSample, true, s));
          k_jtb_kout<F, OffT><<<grid_for(n, block), block, 0, s>>>(
              off, g.nbrs, n, o.k, o.kout_random, o.seed, jc, stats ? ctrl : nullptr);
          GCONN_LAUNCHED("k_jtb_kout");
          GCONN_TRY(prof_mark(kPhaseSample, false, s));
          GCONN_TRY(prof_mark(kPhaseCompress, true, s));
          k_jtb_flatten<<<grid_for(n, block), block, 0, s>>>(W, R, n);
          GCONN_LAUNCHED("k_jtb_flatten");
          GCONN_TRY(prof_mark(kPhaseCompress, false, s));
          GCONN_TRY(prof_mark(kPhaseLmax, true, s));
          k_jtb_lmax<<<1, 1024, 0, s>>>(R, n, o.lmax_samples, o.seed, ctrl);
          GCONN_LAUNCHED("k_jtb_lmax");
          GCONN_TRY(prof_mark(kPhaseLmax, false, s));
        }
        GCONN_TRY(prof_mark(kPhaseGather, true, s));
        k_jtb_gather<OffT><<<grid_for(n, block), block, 0, s>>>(off, R, n, ctrl, wl,
                                                                sampled ? 1 : 0, stats ? 1 : 0);
        GCONN_LAUNCHED("k_jtb_gather");
        GCONN_TRY(prof_mark(kPhaseGather, false, s));
        GCONN_TRY(prof_mark(kPhaseFinish, true, s));
        const uint32_t grid = persistent_grid(k_jtb_finish<F, OffT>, block);
        k_jtb_finish<F, OffT><<<grid, block, 0, s>>>(off, g.nbrs, wl, ctrl, jc);
        GCONN_LAUNCHED("k_jtb_finish");
        return prof_mark(kPhaseFinish, false, s);
      };
      if (g.offsets_64) return body(static_cast<const uint64_t*>(g.offsets));
      return body(static_cast<const uint32_t*>(g.offsets));
    }));
  }
  if (finalize && n > 0) {
    GCONN_TRY(prof_mark(kPhaseFinalize, true, s));
    GCONN_TRY(jtb_labels(W, n, P, M, block, true, s));
    GCONN_TRY(prof_mark(kPhaseFinalize, false, s));
  }
  if (stats) {
    Ctrl h;
    GCONN_HIP(hipMemcpyAsync(&h, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    GCONN_HIP(hipStreamSynchronize(s));
    stats->sampled_edges = h.stat_sampled;
    stats->active_vertices = h.stat_active;
    stats->finish_edges = h.stat_finish_edges;
    stats->hooks = h.stat_hooks;
    stats->rounds = 0;
    stats->lmax = h.lmax;
    stats->bfs_source = kEmpty;
  }
  return GCONN_OK;
}

gconn_status launch_jtb_init(uint64_t* W, uint32_t n, hipStream_t s) {
  if (n == 0) return GCONN_OK;
  k_jtb_init<<<grid_for(n, 256), 256, 0, s>>>(nullptr, W, n, nullptr, nullptr, nullptr);
  GCONN_LAUNCHED("k_jtb_init");
  return GCONN_OK;
}

gconn_status launch_jtb_insert(const gconn_options& o, uint64_t* W, const uint32_t* src,
                               const uint32_t* dst, uint64_t k, hipStream_t s) {
  const uint32_t block = (uint32_t)o.block;
  const JtbCtx jc{W, nullptr, nullptr, nullptr, jtb_salt(o.seed)};
  return with_jtb_find(o.find, [&](auto fc) -> gconn_status {
    constexpr int F = decltype(fc)::value;
    k_jtb_pairs<F><<<grid_for(k, block), block, 0, s>>>(src, dst, k, jc);
    GCONN_LAUNCHED("k_jtb_pairs");
    return GCONN_OK;
  });
}

gconn_status launch_jtb_query(const gconn_options& o, uint64_t* W, const uint8_t* kind,
                              const uint32_t* a, const uint32_t* b, uint64_t q, uint8_t* out,
                              hipStream_t s) {
  const uint32_t block = (uint32_t)o.block;
  return with_jtb_find(o.find, [&](auto fc) -> gconn_status {
    constexpr int F = decltype(fc)::value;
    k_jtb_query<F><<<grid_for(q, block), block, 0, s>>>(kind, a, b, q, W, out);
    GCONN_LAUNCHED("k_jtb_query");
    return GCONN_OK;
  });
}

gconn_status launch_jtb_mixed(const gconn_options& o, uint64_t* W, const uint8_t* kind,
                              const uint32_t* a, const uint32_t* b, uint64_t count, uint8_t* out,
                              hipStream_t s) {
  const uint32_t block = (uint32_t)o.block;
  const JtbCtx jc{W, nullptr, nullptr, nullptr, jtb_salt(o.seed)};
  return with_jtb_find(o.find, [&](auto fc) -> gconn_status {
    constexpr int F = decltype(fc)::value;
    k_jtb_unite_kind<F><<<grid_for(count, block), block, 0, s>>>(kind, a, b, count, jc);
    GCONN_LAUNCHED("k_jtb_unite_kind");
    k_jtb_query<F><<<grid_for(count, block), block, 0, s>>>(kind, a, b, count, W, out);
    GCONN_LAUNCHED("k_jtb_query");
    return GCONN_OK;
  });
}

gconn_status launch_jtb_labels(const uint64_t* W, uint32_t n, uint32_t* labels, uint32_t* scratch,
                               hipStream_t s) {
  if (n == 0) return GCONN_OK;
  return jtb_labels(W, n, labels, scratch, 256, false, s);
}

}  // namespace gconn
