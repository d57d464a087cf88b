// gconn_static.hip -- kernels and host pipeline of static connectivity and
// spanning forest on gfx950 (Alg. "GConn for Static Connectivity" and
// "GConn for Spanning Forest": init, sampling, L_max, finish, finalisation).
//
// Execution shape.  Streaming passes over the n vertices use one lane per
// vertex in wave-uniform grid-stride loops (every lane of a wave runs the same
// number of iterations, so wave-wide ballots, scans and shuffles are safe).
// Vertex gathering (the active set: label != L_max, degree > 0) fills three
// work classes: one lane per small vertex with its edges walked serially (the
// edge-reorganisation goal: no same-vertex CAS conflicts inside a wave), one
// wave per medium vertex, one wave per 1024-edge segment of a hub.
//
// The k-out sampler for Union-Rem-CAS runs as a lane-refill step machine:
// each lane owns a contiguous range of vertices and, every iteration, does one
// step of its current union (one round of at most two loads, then at most one
// CAS), moving on to its next edge or vertex as soon as a union ends.  Lanes
// of a wave therefore never wait for each other's union chains, and every
// iteration issues all lanes' loads together.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "gconn_device.hpp"
#include "gconn_internal.hpp"
#include "gconn_rules.hpp"

namespace gconn {

#ifndef GCONN_PF_PREFETCH_P
#define GCONN_PF_PREFETCH_P 0
#endif

// --------------------------------------------------------------- setup
// P[v] = v and empty forest slots, four vertices per lane with 16-byte stores;
// block 0 also clears the control block.
// Locality probe of the automatic k-out schedule, run by blocks 1..16 of
// k_init (so it costs no launch and no time of its own): 16 x 256 seeded
// vertices count their sampled edges (first k) and how many stay inside their
// vertex's id range of the local-first passes, one (inside, all) pair per
// block in `part`.  The sampling kernels read the pairs and decide the same
// way each (kout_local_chosen): the local passes when at least a quarter
// stay inside and the graph spans at least kProbeMinRanges ranges (one
// workgroup each: fewer cannot fill the chip), otherwise the one-pass kernel.
// A scrambled RMAT graph keeps about range/n of its sampled edges inside.
// Exact either way: the choice only picks the schedule.
constexpr uint32_t kProbeBlocks = 16;
constexpr uint32_t kProbeMinRanges = 64;

struct KoutProbe {
  const uint32_t* off32;  // one of the two offset arrays
  const uint64_t* off64;
  const uint32_t* nbrs;
  uint32_t* part;         // 2 * kProbeBlocks counts; null: no probe
  uint32_t k;
  uint32_t shift;         // log2 of the local-first range
  uint64_t seed;
};

// What the sampling kernels need to read the probe's decision.
struct KoutGate {
  const uint32_t* part;  // null: no gate (the kernel always runs)
  uint32_t n;
  uint32_t shift;
};

__device__ __forceinline__ bool kout_local_chosen(const KoutGate& g) {
  uint64_t loc = 0, tot = 0;
  for (uint32_t b = 0; b < kProbeBlocks; ++b) {
    loc += g.part[2 * b];
    tot += g.part[2 * b + 1];
  }
  const uint64_t ranges = ((uint64_t)g.n + (1ull << g.shift) - 1) >> g.shift;
  return tot > 0 && 4 * loc >= tot && ranges >= kProbeMinRanges;
}

// Block `b` (1..kProbeBlocks) of k_init: one sample per thread.
__device__ void kout_probe_block(const KoutProbe& pr, uint32_t n, uint32_t b) {
  __shared__ uint32_t s_loc, s_tot;
  if (threadIdx.x == 0) s_loc = s_tot = 0;
  __syncthreads();
  const uint64_t j = (uint64_t)(b - 1) * blockDim.x + threadIdx.x;
  const uint32_t v = (uint32_t)(((splitmix64_at(pr.seed, j) >> 32) * (uint64_t)n) >> 32);
  const uint64_t o0 = pr.off32 ? pr.off32[v] : pr.off64[v];
  const uint64_t o1 = pr.off32 ? pr.off32[v + 1] : pr.off64[v + 1];
  const uint32_t t = (uint32_t)(o1 - o0 < pr.k ? o1 - o0 : pr.k);
  uint32_t loc = 0;
  for (uint32_t i = 0; i < t; ++i) loc += (pr.nbrs[o0 + i] >> pr.shift) == (v >> pr.shift);
  if (t) {
    atomicAdd(&s_loc, loc);
    atomicAdd(&s_tot, t);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    pr.part[2 * (b - 1)] = s_loc;
    pr.part[2 * (b - 1) + 1] = s_tot;
  }
}

__global__ void k_init(Ctrl* c, uint32_t* P, uint32_t n, uint32_t* fu, uint32_t* fv, int vec,
                       KoutProbe probe) {
  if (blockIdx.x == 0) {
    uint32_t* w = reinterpret_cast<uint32_t*>(c);
    for (uint32_t i = threadIdx.x; i < sizeof(Ctrl) / 4; i += blockDim.x) w[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
      c->lmax = kEmpty;
      c->bfs_source = kEmpty;
      c->comp_min = kEmpty;
    }
  }
  if (probe.part && blockIdx.x >= 1 && blockIdx.x <= kProbeBlocks)
    kout_probe_block(probe, n, blockIdx.x);
  const uint64_t quads = vec ? n / 4 : 0;  // vec: P, fu, fv are 16-byte aligned
  for (uint64_t q = gtid(); q < quads; q += wave_stride()) {
    const uint32_t v = (uint32_t)(4 * q);
    reinterpret_cast<uint4*>(P)[q] = make_uint4(v, v + 1, v + 2, v + 3);
    if (fu) {
      reinterpret_cast<uint4*>(fu)[q] = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
      reinterpret_cast<uint4*>(fv)[q] = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
    }
  }
  for (uint64_t v = 4 * quads + gtid(); v < n; v += wave_stride()) {
    P[v] = (uint32_t)v;
    if (fu) {
      fu[v] = kEmpty;
      fv[v] = kEmpty;
    }
  }
}

__global__ void k_ctrl_init(Ctrl* c) {
  uint32_t* w = reinterpret_cast<uint32_t*>(c);
  for (uint32_t i = threadIdx.x; i < sizeof(Ctrl) / 4; i += blockDim.x) w[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    c->lmax = kEmpty;
    c->bfs_source = kEmpty;
    c->comp_min = kEmpty;
  }
}

__global__ void k_iota(uint32_t* P, uint32_t n) {
  for (uint64_t v = gtid(); v < n; v += wave_stride()) P[v] = (uint32_t)v;
}

__global__ void k_fill(uint32_t* p, uint32_t value, uint64_t count) {
  for (uint64_t i = gtid(); i < count; i += wave_stride()) p[i] = value;
}

__global__ void k_copy(uint32_t* dst, const uint32_t* src, uint64_t count) {
  for (uint64_t i = gtid(); i < count; i += wave_stride()) dst[i] = src[i];
}

template <typename OffT>
__global__ void k_validate_csr(const OffT* off, const uint32_t* nbrs, uint32_t n, uint64_t m,
                               Ctrl* c) {
  uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid == 0 && (off[0] != 0 || (uint64_t)off[n] != m)) c->err = 1;
  for (uint64_t v = tid; v < n; v += wave_stride())
    if (off[v + 1] < off[v]) c->err = 1;
  for (uint64_t e = tid; e < m; e += wave_stride())
    if (nbrs[e] >= n) c->err = 1;
}

__global__ void k_validate_ids(const uint32_t* a, const uint32_t* b, uint64_t m, uint32_t n,
                               Ctrl* c) {
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += wave_stride())
    if (a[e] >= n || b[e] >= n) c->err = 1;
}

// --------------------------------------------------------------- sampling
// k-out sampling (Sampling Algorithms; Appendix A.1): each vertex unites with
// its first k neighbours (or its first neighbour plus k-1 uniform picks).  One
// lane per vertex reads its leading neighbours together (CSR coalescing) and
// runs its unions serially (edge reorganisation).
template <class R, typename OffT>
__global__ void k_sample_kout(const OffT* __restrict__ off, const uint32_t* __restrict__ nbrs,
                              uint32_t n, uint32_t k, int random, uint64_t seed, LinkCtx lc,
                              Ctrl* stats) {
  unsigned long long sampled = 0;
  for (uint64_t base = wave_base(); base < n; base += wave_stride()) {
    const uint64_t v = base + lane();
    if (v >= n) continue;
    const uint64_t b = off[v], deg = (uint64_t)off[v + 1] - b;
    uint32_t take = (uint32_t)(deg < k ? deg : k);
    if (!random) {
      for (uint32_t j = 0; j < take; ++j) R::unite(lc, (uint32_t)v, nbrs[b + j]);
    } else if (deg > 0) {
      R::unite(lc, (uint32_t)v, nbrs[b]);
      for (uint32_t j = 1; j < k; ++j) {
        const uint32_t r = (uint32_t)(splitmix64_at(seed, v * k + j) >> 32);
        const uint64_t pick = ((uint64_t)r * deg) >> 32;
        R::unite(lc, (uint32_t)v, nbrs[b + pick]);
      }
      take = k;
    }
    sampled += take;
  }
  if (stats) {
    // every lane of the wave left the loop after the same iterations
    sampled = wave_sum(sampled);
    if (lane() == 0 && sampled) atomicAdd(&stats->stat_sampled, sampled);
  }
}

// Default k-out schedule: a persistent grid in which each lane walks vertices
// v, v + T, v + 2T, ... (T = resident lanes, so every iteration of a wave
// covers 64 consecutive vertices and their parent entries stay coalesced).
// The next vertex's row bounds and leading neighbours are loaded before the
// current vertex's unions run, so that random row-start fetch overlaps them.
template <class R, typename OffT>
__global__ void k_sample_kout_pf(const OffT* __restrict__ off, const uint32_t* __restrict__ nbrs,
                                 uint32_t n, uint32_t k, int random, uint64_t seed, LinkCtx lc,
                                 Ctrl* stats, KoutGate gate) {
  if (gate.part && kout_local_chosen(gate)) return;  // the automatic schedule chose the local passes
  const uint64_t T = wave_stride();
  uint64_t v = gtid();
  // row of v: start b, degree d, first two sampled neighbours
  auto fetch = [&](uint64_t x, uint64_t& b, uint64_t& d, uint32_t& w0, uint32_t& w1) {
    b = 0; d = 0; w0 = 0; w1 = 0;
    if (x >= n) return;
    b = off[x];
    d = (uint64_t)off[x + 1] - b;
    if (d > 0) w0 = nbrs[b];
    if (k > 1 && d > 0) {
      if (!random) {
        if (d > 1) w1 = nbrs[b + 1];
      } else {
        const uint32_t r = (uint32_t)(splitmix64_at(seed, x * k + 1) >> 32);
        w1 = nbrs[b + (((uint64_t)r * d) >> 32)];
      }
    }
  };
  uint64_t b, d;
  uint32_t w0, w1;
  fetch(v, b, d, w0, w1);
  unsigned long long sampled = 0;
  while (v < n) {
    const uint64_t nv = v + T;
    uint64_t nb, nd;
    uint32_t n0, n1;
    fetch(nv, nb, nd, n0, n1);
    if (d > 0) {
      const uint32_t take = random ? k : (uint32_t)(d < k ? d : k);
#if GCONN_PF_PREFETCH_P
      if constexpr (R::kUnion == kUnionRemCas) {
        // both neighbours' parents in flight together, from the L2 when cached
        const uint32_t p0 = ld(&lc.P[w0]);
        const uint32_t p1 = take > 1 ? ld(&lc.P[w1]) : kEmpty;
        R::unite_from(lc, (uint32_t)v, w0, kEmpty, p0);
        if (take > 1) R::unite_from(lc, (uint32_t)v, w1, kEmpty, p1);
      } else
#endif
      {
        R::unite(lc, (uint32_t)v, w0);
        if (take > 1) R::unite(lc, (uint32_t)v, w1);
      }
      for (uint32_t j = 2; j < take; ++j) {
        uint64_t pick = j;
        if (random) pick = ((uint64_t)(uint32_t)(splitmix64_at(seed, v * k + j) >> 32) * d) >> 32;
        R::unite(lc, (uint32_t)v, nbrs[b + pick]);
      }
      sampled += take;
    }
    v = nv;
    b = nb;
    d = nd;
    w0 = n0;
    w1 = n1;
  }
  if (stats) {
    // lanes leave the loop at different iterations; they have reconverged here
    sampled = wave_sum(sampled);
    if (lane() == 0 && sampled) atomicAdd(&stats->stat_sampled, sampled);
  }
}

// Two-stage pipelined k-out for Union-Rem-CAS (first k <= 2 edges): while a
// lane runs the unions of its vertex v, the parent entries of the next
// vertex and of its two sampled neighbours are already in flight, and so is
// the row of the vertex after that.  The unions start from those values: a
// parent value loaded earlier is one the slot has held, so it is an ancestor
// and a valid starting point; the hook CAS re-validates any root it acts on.
template <class R, typename OffT>
__global__ void k_sample_kout_pipe(const OffT* __restrict__ off, const uint32_t* __restrict__ nbrs,
                                   uint32_t n, uint32_t k, LinkCtx lc, Ctrl* stats) {
  const uint64_t T = wave_stride();
  const uint32_t* P = lc.P;
  // row of x: number of sampled entries and the first two (0 when absent:
  // P[0] is a valid address and its value is then ignored)
  auto row = [&](uint64_t x, uint32_t& t, uint32_t& a, uint32_t& b) {
    t = 0;
    a = 0;
    b = 0;
    if (x >= n) return;
    const uint64_t s = off[x], d = (uint64_t)off[x + 1] - s;
    t = (uint32_t)(d < k ? d : k);
    if (t > 0) a = nbrs[s];
    if (t > 1) b = nbrs[s + 1];
  };
  uint64_t v = gtid();
  uint32_t t, w0, w1;
  row(v, t, w0, w1);
  uint32_t p0 = ld(&P[w0]), p1 = ld(&P[w1]);
  uint32_t nt, n0, n1;
  row(v + T, nt, n0, n1);
  unsigned long long sampled = 0;
  while (v < n) {
    const uint64_t nv = v + T;
    // stage 2 for the next vertex, stage 1 for the one after
    const uint32_t q0 = ld(&P[n0]), q1 = ld(&P[n1]);
    uint32_t mt, m0, m1;
    row(nv + T, mt, m0, m1);
    if (t > 0) {
      R::unite_from(lc, (uint32_t)v, w0, kEmpty, p0);
      if (t > 1) R::unite_from(lc, (uint32_t)v, w1, kEmpty, p1);
      sampled += t;
    }
    v = nv;
    t = nt;
    w0 = n0;
    w1 = n1;
    p0 = q0;
    p1 = q1;
    nt = mt;
    n0 = m0;
    n1 = m1;
  }
  if (stats) {
    // lanes leave the loop at different iterations; they have reconverged here
    sampled = wave_sum(sampled);
    if (lane() == 0 && sampled) atomicAdd(&stats->stat_sampled, sampled);
  }
}

// k-out pre-link (first k <= 2 edges).  Runs before any union: every vertex v
// is still a root and this lane is the only writer of P[v], so linking v under
// its smallest sampled neighbour u < v is a plain store (it is a link of the
// root v by the edge (v, u), recorded in v's forest slot).  The other sampled
// edges of v (self-loops and repeats dropped) go to res[v] for the union pass.
// The partition after both passes is that of the sampled edge set, as with
// one union per sampled edge.
template <typename OffT>
__global__ void k_kout_prelink(const OffT* __restrict__ off, const uint32_t* __restrict__ nbrs,
                               uint32_t n, uint32_t k, uint32_t* P, uint2* res, uint32_t* fu,
                               uint32_t* fv, Ctrl* stats) {
  unsigned long long sampled = 0, linked = 0;
  for (uint64_t base = wave_base(); base < n; base += wave_stride()) {
    const uint64_t v = base + lane();
    if (v < n) {
      const uint64_t b = off[v], d = (uint64_t)off[v + 1] - b;
      uint32_t a = kEmpty, c = kEmpty;
      if (d > 0) a = nbrs[b];
      if (d > 1 && k > 1) c = nbrs[b + 1];
      sampled += d < k ? d : k;
      if (a == v) a = kEmpty;
      if (c == v || c == a) c = kEmpty;
      const uint32_t lo = a < c ? a : c, hi = a < c ? c : a;  // kEmpty sorts last
      uint2 r = make_uint2(kEmpty, kEmpty);
      if (lo < v) {
        P[v] = lo;
        if (fu) {
          fu[v] = (uint32_t)v;
          fv[v] = lo;
        }
        ++linked;
        r.x = hi;
      } else {
        r.x = lo;
        r.y = hi;
      }
      res[v] = r;
    }
  }
  if (stats) {
    // every lane of the wave ran the same iterations
    sampled = wave_sum(sampled);
    linked = wave_sum(linked);
    if (lane() == 0) {
      if (sampled) atomicAdd(&stats->stat_sampled, sampled);
      if (linked) atomicAdd(&stats->stat_hooks, linked);
    }
  }
}

// Local-first k-out (first k <= 2 edges).  Workgroup r owns the id range
// [r * range, (r + 1) * range): it unites the sampled edges with
// both endpoints in the range on a copy of the range's parents in LDS (LDS
// atomics: far cheaper than device atomics, and the range's trees never
// leave the CU), linking the larger local root under the smaller, so each
// local root is its local component's minimum.  It then writes every vertex's
// local root to P (a flat local forest) and sends the sampled edges that
// leave the range to res[v] for the union pass.  Runs on a freshly
// initialised P; the partition after both passes is the sampled one.  With
// local == 0 it only streams the rows: every sampled edge goes to res[v] and
// the union pass does all the linking (the two-pass schedule).  The range
// is a power of two chosen at launch: the largest the device's LDS per
// workgroup holds (4 bytes per vertex), up to kLocalRangeMax -- the wider it
// is, the fewer sampled edges of a mesh-like graph leave it.
#ifndef GCONN_LOCAL_RANGE_MAX
#define GCONN_LOCAL_RANGE_MAX 32768
#endif
constexpr uint32_t kLocalRangeMax = GCONN_LOCAL_RANGE_MAX;
constexpr uint32_t kLocalRangeMin = 8192;

__device__ __forceinline__ uint32_t lds_root(uint32_t* L, uint32_t x) {
  for (;;) {
    const uint32_t p = __hip_atomic_load(&L[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (p == x) return x;
    x = p;
  }
}

template <typename OffT>
__global__ void __launch_bounds__(1024) k_kout_local(const OffT* __restrict__ off,
                                                     const uint32_t* __restrict__ nbrs,
                                                     uint32_t n, uint32_t k, uint32_t shift,
                                                     uint32_t* P, uint2* res, uint32_t* rsrc,
                                                     uint32_t* rdst, uint32_t* rcnt,
                                                     uint32_t* fu, uint32_t* fv, int local,
                                                     Ctrl* stats, KoutGate gate) {
  extern __shared__ uint32_t L[];  // 2^shift entries
  __shared__ uint32_t nrec;
  if (gate.part && !kout_local_chosen(gate)) return;  // the one-pass kernel was chosen
  const uint32_t range = 1u << shift;
  const uint64_t lo = (uint64_t)blockIdx.x * range;
  const uint32_t len = (uint32_t)min<uint64_t>(range, n - lo);
  const uint64_t out = (uint64_t)blockIdx.x * 2 * range;  // this range's record block
  for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) L[i] = i;
  if (threadIdx.x == 0) nrec = 0;
  __syncthreads();
  unsigned long long sampled = 0, linked = 0;
  // Each lane takes four consecutive vertices per step.  Their row bounds
  // are loaded two steps ahead and their leading neighbours one step ahead,
  // so both are in flight while the current step's LDS unions run.
  const uint32_t stride = 4 * blockDim.x;
  auto load_bounds = [&](uint32_t i, uint64_t (&o)[5]) {
#pragma unroll
    for (int j = 0; j < 5; ++j) o[j] = i + j <= len ? (uint64_t)off[lo + i + j] : 0;
  };
  auto load_heads = [&](uint32_t i, const uint64_t (&o)[5], uint32_t (&w)[8]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint64_t d = i + j < len ? o[j + 1] - o[j] : 0;
      w[2 * j] = d > 0 ? nbrs[o[j]] : kEmpty;
      w[2 * j + 1] = (d > 1 && k > 1) ? nbrs[o[j] + 1] : kEmpty;
    }
  };
  uint64_t o[5], o1[5];
  uint32_t wv[8];
  uint32_t i0 = 4 * threadIdx.x;
  load_bounds(i0, o);
  load_heads(i0, o, wv);
  load_bounds(i0 + stride, o1);
  for (; i0 < len; i0 += stride) {
    uint64_t o2[5];
    uint32_t w1[8];
    load_bounds(i0 + 2 * stride, o2);
    load_heads(i0 + stride, o1, w1);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t i = i0 + j;
      if (i >= len) break;
      const uint64_t v = lo + i;
      const uint64_t d = o[j + 1] - o[j];
      const uint32_t t = (uint32_t)(d < k ? d : k);
      sampled += t;
      uint2 r = make_uint2(kEmpty, kEmpty);
      for (uint32_t e2 = 0; e2 < t; ++e2) {
        const uint32_t w = e2 == 0 ? wv[2 * j] : wv[2 * j + 1];
        if (!local || w < lo || w >= lo + len) {  // leaves the range: global union pass
          if (local) {
            const uint32_t at = atomicAdd(&nrec, 1u);
            rsrc[out + at] = (uint32_t)v;
            rdst[out + at] = w;
          } else if (e2 == 0) {
            r.x = w;
          } else {
            r.y = w;
          }
          continue;
        }
        // local union of i and w - lo (min-linking, CAS on the larger root)
        uint32_t a = lds_root(L, i), c = lds_root(L, (uint32_t)(w - lo));
        while (a != c) {
          const uint32_t hi = a > c ? a : c, low = a > c ? c : a;
          uint32_t e = hi;
          if (__hip_atomic_compare_exchange_strong(&L[hi], &e, low, __ATOMIC_RELAXED,
                                                   __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP)) {
            ++linked;
            if (fu) {
              fu[lo + hi] = (uint32_t)v;
              fv[lo + hi] = w;
            }
            break;
          }
          a = lds_root(L, e);
          c = lds_root(L, low);
        }
      }
      if (!local) res[v] = r;
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      o[j] = o1[j];
      o1[j] = o2[j];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) wv[j] = w1[j];
  }
  __syncthreads();
  if (local) {
    for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
      const uint32_t r = lds_root(L, i);
      if (r != i) P[lo + i] = (uint32_t)lo + r;
    }
    if (threadIdx.x == 0) rcnt[blockIdx.x] = nrec;
  }
  if (stats) {
    sampled = wave_sum(sampled);
    linked = wave_sum(linked);
    if (lane() == 0) {
      if (sampled) atomicAdd(&stats->stat_sampled, sampled);
      if (linked) atomicAdd(&stats->stat_hooks, linked);
    }
  }
}

// Union pass of the local-first k-out over one range's leaving edges (one
// workgroup per range).  After the local pass every vertex points at its
// range-local root, so an edge (v, w) joins the sets of a = P[v] and b = P[w];
// on a mesh most of a range's leaving edges join the same few pairs of local
// roots.  Each distinct pair is united once: an LDS hash set of the pairs
// lets only the first lane that brings a pair run the union (when the set is
// full the lane unites anyway).  Uniting a and b joins the same sets as
// uniting v and w (P[x] only ever holds members of x's set); a spanning
// forest records the edge (v, w) itself.  (Pointing the united roots at their
// final roots afterwards was measured slower: the compression pass that
// follows reaches the roots anyway.)
// 8192 slots (64 KB of LDS): against 16384 (128 KB, one workgroup per CU)
// the 2D grid's call takes 0.435 instead of 0.461 ms and the 3D grid's 0.623
// instead of 0.674; 4096 and fewer slots overflow on the 3D grid's ranges.
// Splitting a range's records over several workgroups, each with a smaller
// set, was slower on both (a pair is then united once per workgroup).
constexpr uint32_t kPairSlots = 8192;

template <class R>
__global__ void __launch_bounds__(1024) k_kout_pairs(const uint32_t* __restrict__ rsrc,
                                                     const uint32_t* __restrict__ rdst,
                                                     const uint32_t* __restrict__ rcnt,
                                                     uint32_t shift, LinkCtx lc,
                                                     KoutGate gate) {
  extern __shared__ unsigned long long H[];  // kPairSlots keys, ~0 = empty
  if (gate.part && !kout_local_chosen(gate)) return;
  for (uint32_t i = threadIdx.x; i < kPairSlots; i += blockDim.x) H[i] = ~0ull;
  __syncthreads();
  const uint32_t cnt = rcnt[blockIdx.x];
  const uint64_t base = (uint64_t)blockIdx.x * 2 * (1ull << shift);
  for (uint32_t j0 = 0; j0 < cnt; j0 += blockDim.x) {
    const uint32_t j = j0 + threadIdx.x;
    bool fresh = false;
    uint32_t v = 0, w = 0, a = 0, b = 0;
    if (j < cnt) {
      v = rsrc[base + j];
      w = rdst[base + j];
      a = ld(&lc.P[v]);
      b = ld(&lc.P[w]);
      if (a != b) {
        const unsigned long long key = a < b ? ((unsigned long long)a << 32) | b
                                             : ((unsigned long long)b << 32) | a;
        uint32_t h = (uint32_t)((key * 0x9e3779b97f4a7c15ull) >> 50) & (kPairSlots - 1);
        fresh = true;  // unless found, or the probe runs out (then unite anyway)
        for (int probe = 0; probe < 32; ++probe) {
          unsigned long long e = ~0ull;
          if (__hip_atomic_compare_exchange_strong(&H[h], &e, key, __ATOMIC_RELAXED,
                                                   __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP))
            break;  // inserted: this lane unites the pair
          if (e == key) {
            fresh = false;  // another lane has this pair
            break;
          }
          h = (h + 1) & (kPairSlots - 1);
        }
      }
    }
    if (fresh) R::unite_pair(lc, a, b, v, w);
  }
}

// Union pass over the residual sampled edges of the pre-link.
template <class R>
__global__ void k_kout_residual(const uint2* __restrict__ res, uint32_t n, LinkCtx lc) {
  for (uint64_t v = gtid(); v < n; v += wave_stride()) {
    const uint2 r = res[v];
    if (r.x != kEmpty) R::unite(lc, (uint32_t)v, r.x);
    if (r.y != kEmpty) R::unite(lc, (uint32_t)v, r.y);
  }
}

// Flattening of the pre-link forest (the flat k-out schedule): every vertex
// is pointed straight at its tree's root before the residual unions run, so
// those start from roots instead of walking the pre-link chains once per
// union.  No link runs in this pass and every write stores a root that is an
// ancestor of the slot's vertex, so reads may be cached and stale; the writes
// are agent-scope stores (two waves can share a line of P).
__global__ void k_flatten(uint32_t* P, uint32_t n) {
  for (uint64_t v = gtid(); v < n; v += wave_stride()) {
    const uint32_t p = ld(&P[v]);
    if (p == v) continue;
    uint32_t r = p, q = ld(&P[p]);
    while (q != r) {
      r = q;
      q = ld(&P[r]);
    }
    if (r != p) st(&P[v], r);
  }
}

// Residual union pass of the flat schedule: both endpoints' parents are loaded
// together before the unions run (a parent value the slot has held is a valid
// start for the root-based rules; the splice rule re-reads them itself).
template <class R>
__global__ void k_kout_residual_flat(const uint2* __restrict__ res, uint32_t n, LinkCtx lc) {
  for (uint64_t v = gtid(); v < n; v += wave_stride()) {
    const uint2 r = res[v];
    if (r.x == kEmpty) continue;  // r.y is empty too
    const uint32_t pv = ld(&lc.P[v]);
    const uint32_t p0 = ld(&lc.P[r.x]);
    const uint32_t p1 = r.y != kEmpty ? ld(&lc.P[r.y]) : kEmpty;
    R::unite_from(lc, (uint32_t)v, r.x, pv, p0);
    if (r.y != kEmpty) R::unite_from(lc, (uint32_t)v, r.y, pv, p1);
  }
}

// --------------------------------------------------------------- XCD-bucketed k-out
// First-k k-out (k <= 2) arranged so that the union pass's parent reads stay
// in the L2 of the XCD that makes them.  An MI355X has eight XCDs, each with
// a private 4 MB L2, and a parent read that misses it costs a 128-byte line
// across the fabric.  Three kernels:
//  * k_kx_stream: one workgroup per 1024-vertex chunk reads the rows' first k
//    neighbours and writes P[v] -- the pre-link of v under its smallest
//    sampled neighbour when that is smaller (v is a root and this lane its
//    only writer, so a plain store), else v itself -- and v's forest slots.
//    The other sampled edges of the chunk ("residual", at most two per
//    vertex) go to the chunk's record block, sorted into eight groups by the
//    XCD that will unite them: edge (v, w) goes to group (w >> shift) & 7, so
//    each XCD reads the parents of one eighth of the ids (interleaved ranges
//    of 2^shift vertices, which spreads the low-id skew of sorted rows).
//  * k_kx_flatten: per chunk, every vertex is pointed at its pre-link root,
//    and every record's first endpoint is replaced by that root (the original
//    endpoint is kept aside for spanning forests).
//  * k_kx_unite: a persistent grid.  Each workgroup reads the id of the XCD
//    it runs on and takes work items (kKxItem chunks' records of one group)
//    from that XCD's queue, then from the others once it is empty, and unites
//    each record with the configured rule.
// The partition after the three passes is that of the sampled edge set.
constexpr uint32_t kKxChunk = 1024;         // vertices per chunk: 256 lanes x 4
constexpr uint32_t kKxCap = 2 * kKxChunk;   // residual records per chunk
constexpr uint32_t kKxGroups = 8;           // record groups: one per XCD
constexpr uint32_t kKxItem = 16;            // chunks per work item of the union pass

// Id of the XCD running the calling wave (hardware register XCC_ID, id 20 on
// gfx940 and later, bits [3:0]), folded into [0, 8).
__device__ __forceinline__ uint32_t xcc_id() {
  return (uint32_t)__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kKxGroups - 1);
}

template <typename OffT>
__global__ void __launch_bounds__(256) k_kx_stream(const OffT* __restrict__ off,
                                                   const uint32_t* __restrict__ nbrs, uint32_t n,
                                                   uint32_t k, uint32_t shift, uint32_t* P,
                                                   uint32_t* fu, uint32_t* fv, uint32_t* rsrc,
                                                   uint32_t* rdst, uint32_t* hdr, int vec,
                                                   Ctrl* stats) {
  // vec: bit 0 -- P, fu, fv are 16-byte aligned; bit 1 -- uint32 offsets are
  __shared__ uint32_t cnt[kKxGroups], pos[kKxGroups + 1];
  __shared__ uint32_t s_src[kKxCap], s_dst[kKxCap];
  const uint64_t base = (uint64_t)blockIdx.x * kKxChunk;
  if (threadIdx.x < kKxGroups) cnt[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t v0 = base + 4ull * threadIdx.x;
  // row starts of the lane's four vertices (and the end of the last)
  uint64_t o[5];
  if ((vec & 2) && v0 + 4 <= n && sizeof(OffT) == 4) {
    const uint4 a = *reinterpret_cast<const uint4*>(off + v0);
    o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
    o[4] = off[v0 + 4];
  } else {
#pragma unroll
    for (int j = 0; j < 5; ++j) o[j] = v0 + j <= n ? (uint64_t)off[v0 + j] : 0;
  }
  uint32_t w0[4], w1[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint64_t d = v0 + j < n ? o[j + 1] - o[j] : 0;
    w0[j] = d > 0 ? nbrs[o[j]] : kEmpty;
    w1[j] = (d > 1 && k > 1) ? nbrs[o[j] + 1] : kEmpty;
  }
  uint32_t par[4], lo_[4], rec[8], slot[8];
  unsigned long long sampled = 0, linked = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t v = (uint32_t)(v0 + j);
    const uint64_t d = v0 + j < n ? o[j + 1] - o[j] : 0;
    sampled += d < k ? d : k;
    const uint32_t a = w0[j] == v ? kEmpty : w0[j];
    const uint32_t c = (w1[j] == v || w1[j] == a) ? kEmpty : w1[j];
    const uint32_t lo = a < c ? a : c, hi = a < c ? c : a;  // kEmpty sorts last
    if (lo < v) {
      par[j] = lo;
      lo_[j] = lo;
      ++linked;
      rec[2 * j] = hi;
      rec[2 * j + 1] = kEmpty;
    } else {
      par[j] = v;
      lo_[j] = kEmpty;
      rec[2 * j] = lo;
      rec[2 * j + 1] = hi;
    }
  }
#pragma unroll
  for (int r = 0; r < 8; ++r)
    slot[r] = rec[r] != kEmpty ? atomicAdd(&cnt[(rec[r] >> shift) & (kKxGroups - 1)], 1u) : 0u;
  // parents and forest slots of the four vertices
  if ((vec & 1) && v0 + 4 <= n) {
    *reinterpret_cast<uint4*>(P + v0) = make_uint4(par[0], par[1], par[2], par[3]);
    if (fu) {
      const uint32_t v = (uint32_t)v0;
      *reinterpret_cast<uint4*>(fu + v0) =
          make_uint4(lo_[0] != kEmpty ? v : kEmpty, lo_[1] != kEmpty ? v + 1 : kEmpty,
                     lo_[2] != kEmpty ? v + 2 : kEmpty, lo_[3] != kEmpty ? v + 3 : kEmpty);
      *reinterpret_cast<uint4*>(fv + v0) = make_uint4(lo_[0], lo_[1], lo_[2], lo_[3]);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (v0 + j < n) {
        P[v0 + j] = par[j];
        if (fu) {
          fu[v0 + j] = lo_[j] != kEmpty ? (uint32_t)(v0 + j) : kEmpty;
          fv[v0 + j] = lo_[j];
        }
      }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t at = 0;
    for (uint32_t g = 0; g < kKxGroups; ++g) {
      pos[g] = at;
      at += cnt[g];
    }
    pos[kKxGroups] = at;
  }
  if (threadIdx.x < kKxGroups) hdr[(uint64_t)blockIdx.x * kKxGroups + threadIdx.x] = cnt[threadIdx.x];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 8; ++r)
    if (rec[r] != kEmpty) {
      const uint32_t at = pos[(rec[r] >> shift) & (kKxGroups - 1)] + slot[r];
      s_src[at] = (uint32_t)(v0 + r / 2);
      s_dst[at] = rec[r];
    }
  __syncthreads();
  const uint32_t total = pos[kKxGroups];
  const uint64_t out = (uint64_t)blockIdx.x * kKxCap;
  for (uint32_t i = threadIdx.x; i < total; i += blockDim.x) {
    rsrc[out + i] = s_src[i];
    rdst[out + i] = s_dst[i];
  }
  if (stats) {
    sampled = wave_sum(sampled);
    linked = wave_sum(linked);
    if (lane() == 0) {
      if (sampled) atomicAdd(&stats->stat_sampled, sampled);
      if (linked) atomicAdd(&stats->stat_hooks, linked);
    }
  }
}

// Pre-link roots of one chunk: P[v] is pointed at its root (only this
// workgroup writes the chunk's parent words, and no link runs in this kernel,
// so every value any lane reads is an ancestor), and each residual record gets
// the root of its first endpoint (rroot, same layout as the records).
__global__ void __launch_bounds__(256) k_kx_flatten(uint32_t* P, uint32_t n,
                                                    const uint32_t* __restrict__ rsrc,
                                                    const uint32_t* __restrict__ hdr,
                                                    uint32_t* rroot) {
  __shared__ uint32_t R[kKxChunk];
  const uint64_t base = (uint64_t)blockIdx.x * kKxChunk;
  const uint32_t len = (uint32_t)min<uint64_t>(kKxChunk, n - base);
  uint32_t p[4], r[4];
  bool done[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t i = 4 * threadIdx.x + j;
    p[j] = i < len ? P[base + i] : 0u;
    r[j] = p[j];
    done[j] = i >= len || p[j] == base + i;
  }
  // the four chases advance together (independent loads in flight)
  for (;;) {
    bool more = false;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (!done[j]) {
        const uint32_t q = ld(&P[r[j]]);
        if (q == r[j]) done[j] = true;
        else r[j] = q;
        more = more || !done[j];
      }
    if (!more) break;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t i = 4 * threadIdx.x + j;
    if (i < len) {
      R[i] = r[j];
      if (r[j] != p[j]) P[base + i] = r[j];
    }
  }
  __syncthreads();
  const uint32_t* h = hdr + (uint64_t)blockIdx.x * kKxGroups;
  uint32_t total = 0;
#pragma unroll
  for (uint32_t g = 0; g < kKxGroups; ++g) total += h[g];
  const uint64_t at = (uint64_t)blockIdx.x * kKxCap;
  for (uint32_t i = threadIdx.x; i < total; i += blockDim.x) rroot[at + i] = R[rsrc[at + i] - base];
}

// Union pass over the residual records, XCD by XCD (see above).  Each lane
// takes two records at a time and loads both endpoints' parents of both
// before uniting them (a parent value a slot has held is a valid start for
// the root-based rules).
template <class R>
__global__ void __launch_bounds__(256) k_kx_unite(const uint32_t* __restrict__ rsrc,
                                                  const uint32_t* __restrict__ rdst,
                                                  const uint32_t* __restrict__ rroot,
                                                  const uint32_t* __restrict__ hdr,
                                                  uint32_t chunks, int from_vertex, Ctrl* c,
                                                  LinkCtx lc) {
  __shared__ uint32_t s_item, s_grp;
  __shared__ uint32_t seg[kKxItem], pre[kKxItem + 1];
  const uint32_t items = (chunks + kKxItem - 1) / kKxItem;
  const uint32_t home = xcc_id();
  uint32_t tried = 0;  // thread 0 only: queues found empty, in order from home
  for (;;) {
    if (threadIdx.x == 0) {
      uint32_t t = kEmpty, g = home;
      while (tried < kKxGroups) {
        g = (home + tried) & (kKxGroups - 1);
        t = atomicAdd(&c->kx_queue[g], 1u);
        if (t < items) break;
        t = kEmpty;
        ++tried;
      }
      s_item = t;
      s_grp = g;
    }
    __syncthreads();
    const uint32_t item = s_item, g = s_grp;
    if (item == kEmpty) break;
    if (threadIdx.x < 64) {
      // the group's segment in each chunk of the item, and a prefix of the lengths
      const uint32_t ch = item * kKxItem + lane();
      uint32_t start = 0, cnt = 0;
      if (lane() < kKxItem && ch < chunks) {
        const uint32_t* h = hdr + (uint64_t)ch * kKxGroups;
        for (uint32_t x = 0; x < g; ++x) start += h[x];
        cnt = h[g];
      }
      uint32_t total;
      const uint32_t ex = wave_exclusive(cnt, &total);
      if (lane() < kKxItem) {
        seg[lane()] = start;
        pre[lane()] = ex;
      }
      if (lane() == 0) pre[kKxItem] = total;
    }
    __syncthreads();
    const uint32_t total = pre[kKxItem];
    auto locate = [&](uint32_t j) -> uint64_t {
      uint32_t lo = 0, hi = kKxItem;  // pre[lo] <= j < pre[hi]
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= j) lo = mid;
        else hi = mid;
      }
      return (uint64_t)(item * kKxItem + lo) * kKxCap + seg[lo] + (j - pre[lo]);
    };
    for (uint32_t j = threadIdx.x; j < total; j += 2 * blockDim.x) {
      const uint32_t j2 = j + blockDim.x;
      const uint64_t i1 = locate(j);
      const uint64_t i2 = j2 < total ? locate(j2) : i1;
      const uint32_t r1 = __builtin_nontemporal_load(&rroot[i1]);
      const uint32_t w1 = __builtin_nontemporal_load(&rdst[i1]);
      const uint32_t r2 = __builtin_nontemporal_load(&rroot[i2]);
      const uint32_t w2 = __builtin_nontemporal_load(&rdst[i2]);
      const uint32_t e1 = (from_vertex || lc.fu) ? __builtin_nontemporal_load(&rsrc[i1]) : r1;
      const uint32_t e2 = (from_vertex || lc.fu) ? __builtin_nontemporal_load(&rsrc[i2]) : r2;
      const uint32_t pw1 = ld(&lc.P[w1]), pw2 = ld(&lc.P[w2]);
      if (from_vertex) {
        // from the endpoint itself, whose parent was the root r (flattened)
        R::unite_edge(lc, e1, w1, r1, pw1, e1);
        if (j2 < total) R::unite_edge(lc, e2, w2, r2, pw2, e2);
      } else {
        const uint32_t pr1 = ld(&lc.P[r1]), pr2 = ld(&lc.P[r2]);
        R::unite_edge(lc, r1, w1, pr1, pw1, e1);
        if (j2 < total) R::unite_edge(lc, r2, w2, pr2, pw2, e2);
      }
    }
    __syncthreads();
  }
}

// The same first-k sampling with Union-Rem-CAS as a lane-refill step machine
// (uint32 offsets).  Each iteration: pick at most two addresses from the
// lane's state, load them together, decide, issue at most one CAS, update the
// state.  States: OFF (row bounds of the next vertex), NBR (its next two
// sampled neighbours), REM (compare P[ru], P[rv]; hook ru if it is a root),
// SPL (one splice step at ru: split or halve), CMP1/CMP2 (one FindSplit /
// FindHalve step of the trailing compression of u, then of v).  Every state
// either finishes a union, strictly lowers ru or the compression cursor, or
// continues from a fresh CAS result, so each lane terminates.
template <int F, int S>
__global__ void __launch_bounds__(256) k_sample_kout_rem_sm(const uint32_t* __restrict__ off,
                                                            const uint32_t* __restrict__ nbrs,
                                                            uint32_t n, uint32_t k, LinkCtx lc,
                                                            Ctrl* stats) {
  enum : uint32_t { OFF, NBR, REM, SPL, CMP1, CMP2, DONE };
  uint32_t* __restrict__ P = lc.P;
  const uint64_t T = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t chunk = (n + T - 1) / T;
  uint64_t vtx = gtid() * chunk;
  const uint64_t vend = min((uint64_t)n, vtx + chunk);
  uint32_t st = vtx < vend ? OFF : DONE;
  uint32_t b = 0, take = 0, j = 0, wnext = 0, have_next = 0;
  uint32_t u = 0, v = 0, ru = 0, rv = 0, pru = 0, prv = 0, x = 0, xp = 0, side = 0;
  unsigned long long sampled = 0, hooks = 0;
  while (st != DONE) {
    // ---- one load round
    const uint32_t* a0;
    const uint32_t* a1 = nullptr;
    switch (st) {
      case OFF: a0 = off + vtx; a1 = off + vtx + 1; break;
      case NBR: a0 = nbrs + b + j; if (j + 1 < take) a1 = nbrs + b + j + 1; break;
      case REM: a0 = P + ru; a1 = P + rv; break;
      case SPL: a0 = P + pru; break;
      case CMP1: a0 = P + x; break;
      default: a0 = P + xp; break;  // CMP2
    }
    const uint32_t r0 = ld(a0);
    const uint32_t r1 = a1 ? ld(a1) : 0u;
    // ---- decide; at most one CAS (op: 0 none, 1 hook ru, 2 splice, 3 compression)
    uint32_t op = 0;
    bool union_end = false, cmp_end = false;
    uint32_t* ca = nullptr;
    uint32_t cexp = 0, cdes = 0;
    switch (st) {
      case OFF: {
        const uint32_t deg = r1 - r0;
        b = r0;
        take = deg < k ? deg : k;
        sampled += take;
        j = 0;
        if (take) st = NBR;
        else if (++vtx >= vend) st = DONE;
        break;
      }
      case NBR:
        u = (uint32_t)vtx;
        v = r0;
        have_next = a1 != nullptr;
        wnext = r1;
        ru = u;
        rv = v;
        st = REM;
        break;
      case REM:
        pru = r0;
        prv = r1;
        if (pru == prv) {
          union_end = true;
        } else {
          if (pru < prv) {
            uint32_t t = ru; ru = rv; rv = t;
            t = pru; pru = prv; prv = t;
          }
          if (ru == pru) {
            op = 1; ca = P + ru; cexp = ru; cdes = prv;
          } else {
            st = SPL;
          }
        }
        break;
      case SPL: {
        const uint32_t w = r0;
        if (w != pru) { op = 2; ca = P + ru; cexp = pru; cdes = w; }
        ru = (S == kSpliceSplitOne) ? pru : w;
        st = REM;
        break;
      }
      case CMP1:
        xp = r0;
        if (xp == x) cmp_end = true;
        else st = CMP2;
        break;
      default: {  // CMP2
        const uint32_t w = r0;
        if (w == xp) cmp_end = true;
        else { op = 3; ca = P + x; cexp = xp; cdes = w; }
        break;
      }
    }
    uint32_t e = cexp;
    bool ok = false;
    if (op) ok = cas(ca, e, cdes);
    // ---- transitions that need the CAS result
    if (op == 1) {                    // hook attempt of root ru
      if (ok) {
        if (lc.fu) { lc.fu[ru] = u; lc.fv[ru] = v; }
        ++hooks;
        if constexpr (F != kFindNaive) { side = 0; x = u; st = CMP1; }
        else union_end = true;
      } else {
        pru = e;                      // ru was linked meanwhile: splice from its fresh parent
        st = SPL;
      }
    } else if (op == 3) {             // compression step done
      x = (F == kFindSplit) ? xp : (ok ? cdes : e);
      st = CMP1;
    }
    if (cmp_end) {
      if (side == 0) { side = 1; x = v; st = CMP1; }
      else union_end = true;
    }
    if (union_end) {
      if (have_next) {
        have_next = 0;
        ++j;
        v = wnext;
        ru = u;
        rv = v;
        st = REM;
      } else if (j + 1 < take) {
        ++j;
        st = NBR;
      } else {
        st = (++vtx < vend) ? OFF : DONE;
      }
    }
  }
  if (stats) {
    sampled = wave_sum(sampled);
    hooks = wave_sum(hooks);
    if (lane() == 0) {
      if (sampled) atomicAdd(&stats->stat_sampled, sampled);
      if (hooks && lc.hooks) atomicAdd(lc.hooks, hooks);
    }
  }
}

// Hook-based sampling, step 1 (Sampling Algorithms, HB): P[v] = min(v, w) for
// the first (smallest) neighbour w; contention-free, one write per vertex.
template <typename OffT>
__global__ void k_hb_step1(const OffT* __restrict__ off, const uint32_t* __restrict__ nbrs,
                           uint32_t* P, uint32_t n, uint32_t* fu, uint32_t* fv, Ctrl* stats) {
  for (uint64_t base = wave_base(); base < n; base += wave_stride()) {
    uint64_t v = base + lane();
    uint32_t took = 0, linked = 0;
    if (v < n) {
      uint64_t b = off[v];
      if ((uint64_t)off[v + 1] > b) {
        took = 1;
        uint32_t w = nbrs[b];
        if (w < v) {
          P[v] = w;
          linked = 1;
          if (fu) {
            fu[v] = (uint32_t)v;
            fv[v] = w;
          }
        }
      }
    }
    if (stats) {
      unsigned long long s = wave_sum(took), l = wave_sum(linked);
      if (lane() == 0 && s) atomicAdd(&stats->stat_sampled, s);
      if (lane() == 0 && l) atomicAdd(&stats->stat_hooks, l);
    }
  }
}

// HB step 2: vertices that stayed roots after step 1 (degree 0, or first
// neighbour not smaller -- decided from the graph, not from P, so concurrent
// links of step 2 cannot change the sampled set) unite with their first N
// neighbours.
template <class R, typename OffT>
__global__ void k_hb_step2(const OffT* __restrict__ off, const uint32_t* __restrict__ nbrs,
                           uint32_t n, uint32_t N, LinkCtx lc, Ctrl* stats) {
  for (uint64_t base = wave_base(); base < n; base += wave_stride()) {
    uint64_t v = base + lane();
    uint32_t take = 0;
    if (v < n) {
      uint64_t b = off[v], deg = (uint64_t)off[v + 1] - b;
      if (deg > 0 && nbrs[b] >= v) {
        take = (uint32_t)(deg < N ? deg : N);
        for (uint32_t j = 0; j < take; ++j) R::unite(lc, (uint32_t)v, nbrs[b + j]);
      }
    }
    if (stats) {
      unsigned long long s = wave_sum(take);
      if (lane() == 0 && s) atomicAdd(&stats->stat_sampled, s);
    }
  }
}

// GetMostFrequentLabel over a seeded sample of vertices: sample j is vertex
// floor(hi32(SplitMix64_j(seed)) * n / 2^32), its label the root of its tree
// (so no full compression has to precede it).  Counts go to an LDS hash
// table; the winner is the largest count, smallest label on ties.
constexpr uint32_t kLmaxTable = 2 * kMaxLmaxSamples;
__global__ void __launch_bounds__(1024) k_lmax(const uint32_t* P, uint32_t n, uint32_t samples,
                                               uint64_t seed, Ctrl* c) {
  __shared__ uint32_t keys[kLmaxTable];
  __shared__ uint32_t cnts[kLmaxTable];
  __shared__ unsigned long long best;
  for (uint32_t i = threadIdx.x; i < kLmaxTable; i += blockDim.x) {
    keys[i] = kEmpty;
    cnts[i] = 0;
  }
  if (threadIdx.x == 0) best = 0;
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < samples; j += blockDim.x) {
    const uint32_t hi = (uint32_t)(splitmix64_at(seed, j) >> 32);
    const uint32_t v = (uint32_t)(((uint64_t)hi * n) >> 32);
    const uint32_t label = root_plain(P, v);
    uint32_t h = (label * 2654435761u) & (kLmaxTable - 1);
    for (;;) {
      const uint32_t prev = atomicCAS(&keys[h], kEmpty, label);
      if (prev == kEmpty || prev == label) {
        atomicAdd(&cnts[h], 1u);
        break;
      }
      h = (h + 1) & (kLmaxTable - 1);
    }
  }
  __syncthreads();
  unsigned long long mine = 0;
  for (uint32_t i = threadIdx.x; i < kLmaxTable; i += blockDim.x)
    if (keys[i] != kEmpty) {
      const unsigned long long key = ((unsigned long long)cnts[i] << 32) | (kEmpty - keys[i]);
      mine = key > mine ? key : mine;
    }
  mine = wave_max(mine);
  if (lane() == 0) atomicMax(&best, mine);
  __syncthreads();
  if (threadIdx.x == 0 && best) c->lmax = kEmpty - (uint32_t)(best & 0xFFFFFFFFu);
}

// Full compression fused with vertex gathering.  mode 0: no sampling (P is the
// identity, every vertex with edges is active); mode 1: P is already flat
// (BFS sampling); mode 2: P[v] = root(v) first (k-out, hook-based).  Active:
// degree > 0 and label != L_max (unless skip_lmax is 0).  Each lane takes four
// consecutive vertices: their offsets and parents are all loaded before any
// is used, and the four root chases advance together, so one wave keeps
// several independent loads in flight instead of one dependent chain.
template <typename OffT>
__global__ void k_compress_gather(const OffT* __restrict__ off, uint32_t* P, uint32_t n, Ctrl* c,
                                  WorkLists wl, int mode, int skip_lmax, int want_stats) {
  const uint32_t lmax = skip_lmax ? c->lmax : kEmpty;
  // L_max is the root of the largest sampled tree (k_lmax found it by walking
  // to roots, and no link runs between sampling and this pass), so a chase
  // that reaches it stops there without reading its slot: that one word
  // would otherwise be read by almost every wave of the launch
  const uint32_t known_root = c->lmax;
  // 16-byte loads of a lane's four offsets and parents when they are aligned
  // (uint32 offsets, 16-byte aligned arrays, four vertices in range).
  const bool vec = sizeof(OffT) == 4 &&
                   ((reinterpret_cast<uintptr_t>(off) | reinterpret_cast<uintptr_t>(P)) % 16) == 0;
  unsigned long long act = 0, edges = 0;
  for (uint64_t base = wave_base() * 4; base < n; base += wave_stride() * 4) {
    const uint64_t v0 = base + 4 * lane();
    uint64_t o[5];
    uint32_t p[4], r[4];
    if (vec && v0 + 4 <= n) {
      const uint4 oo = *reinterpret_cast<const uint4*>(off + v0);
      o[0] = oo.x;
      o[1] = oo.y;
      o[2] = oo.z;
      o[3] = oo.w;
      o[4] = (uint64_t)off[v0 + 4];  // off has n + 1 entries
      if (mode != 0) {
        const uint4 pp = *reinterpret_cast<const uint4*>(P + v0);
        p[0] = pp.x;
        p[1] = pp.y;
        p[2] = pp.z;
        p[3] = pp.w;
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) p[k] = (uint32_t)(v0 + k);
      }
    } else {
#pragma unroll
      for (int k = 0; k < 5; ++k) o[k] = (v0 + k <= n) ? (uint64_t)off[v0 + k] : 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) p[k] = (mode != 0 && v0 + k < n) ? P[v0 + k] : (uint32_t)(v0 + k);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = p[k];
    if (mode == 2) {
      bool more = true;
      while (more) {  // lockstep pointer jumping of the four chases
        more = false;
        uint32_t q[4];
        if (lane() == 0) GCONN_COUNT(kOpChaseRounds);  // diagnostic builds: one per wave round
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const bool walk = r[k] != v0 + k && r[k] != known_root && v0 + k < n;
          if (walk) GCONN_COUNT(kOpChase);
          q[k] = walk ? P[r[k]] : r[k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (q[k] != r[k]) {
            r[k] = q[k];
            more = true;
          }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (v0 + k < n && r[k] != p[k]) P[v0 + k] = r[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool valid = v0 + k < n;
      const uint64_t deg = valid ? o[k + 1] - o[k] : 0;
      const bool active = valid && deg > 0 && r[k] != lmax;
      // group (base / 64) + k: each push call covers at most 64 vertices
      wl_push(wl, c, (base >> 6) + k, (uint32_t)(v0 + k), deg, active);
      act += active ? 1 : 0;
      edges += active ? deg : 0;
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

// Finish phase for the union-find rules (Alg. union-find meta-algorithm):
// every edge (u, v) of every active u is united.  Small vertices one lane
// each, medium vertices one wave each, hub segments one wave each.
template <class R, typename OffT>
__global__ void k_finish(const OffT* __restrict__ off, const uint32_t* __restrict__ nbrs,
                         WorkLists wl, const Ctrl* c, LinkCtx lc) {
  __shared__ uint32_t pre_s[kSubLists + 1], pre_m[kSubLists + 1];
  wl_prefix(c->small_cnt, pre_s);
  wl_prefix(c->medium_cnt, pre_m);
  __syncthreads();
  const uint32_t S = pre_s[kSubLists], M = pre_m[kSubLists], G = c->seg_count;
  for (uint64_t i = gtid(); i < S; i += wave_stride()) {
    const uint32_t u = wl_get(wl.small, wl.cap, pre_s, (uint32_t)i);
    const uint64_t e = off[u + 1];
    for (uint64_t x = off[u]; x < e; ++x) R::unite(lc, u, nbrs[x]);
  }
  for (uint64_t w = wave_index(); w < M; w += wave_count()) {
    const uint32_t u = wl_get(wl.medium, wl.cap, pre_m, (uint32_t)w);
    const uint64_t e = off[u + 1];
    for (uint64_t x = off[u] + lane(); x < e; x += 64) R::unite(lc, u, nbrs[x]);
  }
  for (uint64_t s = wave_index(); s < G; s += wave_count()) {
    const uint2 sg = wl.segs[s];
    const uint64_t b = (uint64_t)off[sg.x] + (uint64_t)sg.y * kSeg;
    uint64_t e = off[sg.x + 1];
    if (e > b + kSeg) e = b + kSeg;
    for (uint64_t x = b + lane(); x < e; x += 64) R::unite(lc, sg.x, nbrs[x]);
  }
}

// Label finalisation: labels[v] = root(v).  When sampling ran and the L_max
// root is still a root, only the active vertices can have a changed root (the
// L_max group points at it, isolated vertices are their own roots), so only
// the work lists are finalised; otherwise every vertex is.
__global__ void k_finalize(uint32_t* P, uint32_t n, const Ctrl* c, WorkLists wl, int sampled) {
  __shared__ uint32_t pre_s[kSubLists + 1], pre_m[kSubLists + 1];
  wl_prefix(c->small_cnt, pre_s);
  wl_prefix(c->medium_cnt, pre_m);
  __syncthreads();
  const uint32_t lmax = c->lmax;
  const bool partial = sampled && lmax != kEmpty && lmax < n && P[lmax] == lmax;
  if (partial) {
    const uint32_t S = pre_s[kSubLists], M = pre_m[kSubLists], G = c->seg_count;
    const uint64_t total = (uint64_t)S + M + G;
    for (uint64_t i = gtid(); i < total; i += wave_stride()) {
      uint32_t a;
      if (i < S) a = wl_get(wl.small, wl.cap, pre_s, (uint32_t)i);
      else if (i < (uint64_t)S + M) a = wl_get(wl.medium, wl.cap, pre_m, (uint32_t)(i - S));
      else {
        const uint2 sg = wl.segs[i - S - M];
        if (sg.y != 0) continue;
        a = sg.x;
      }
      const uint32_t p = P[a];
      const uint32_t r = root_plain(P, p);
      if (r != p) P[a] = r;
    }
  } else {
    for (uint64_t v = gtid(); v < n; v += wave_stride()) {
      const uint32_t p = P[v];
      if (p == v) continue;
      const uint32_t r = root_plain(P, p);
      if (r != p) P[v] = r;
    }
  }
}

// labels_out[v] = root(v) into a separate buffer (incremental labels).
__global__ void k_compress_to(const uint32_t* P, uint32_t* out, uint32_t n) {
  for (uint64_t v = gtid(); v < n; v += wave_stride()) out[v] = root_plain(P, (uint32_t)v);
}

// COO finish (no sampling for COO): one lane per edge.
template <class R>
__global__ void k_unite_pairs(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b,
                              uint64_t m, LinkCtx lc) {
  for (uint64_t e = gtid(); e < m; e += wave_stride()) R::unite(lc, a[e], b[e]);
}

// --------------------------------------------------------------- materialised edges
// SV, LT and LP iterate over the active edges many times; they are laid out
// once as a COO pair list (one entry per CSR entry of an active vertex).
constexpr uint32_t kMatChunks = 16;

template <typename OffT>
__global__ void k_materialize(const OffT* __restrict__ off, const uint32_t* __restrict__ nbrs,
                              WorkLists wl, Ctrl* c, uint32_t* esrc, uint32_t* edst) {
  __shared__ uint32_t pre_s[kSubLists + 1], pre_m[kSubLists + 1];
  wl_prefix(c->small_cnt, pre_s);
  wl_prefix(c->medium_cnt, pre_m);
  __syncthreads();
  const uint32_t S = pre_s[kSubLists], M = pre_m[kSubLists], G = c->seg_count;
  // Small vertices: a wave takes kMatChunks groups of 64 list entries and
  // reserves their edges with one atomic (a reservation per 64 entries put one
  // single-address atomic per wave of the launch in one L2 queue): the first
  // pass adds up the degrees, the second writes the edges.
  // (fewer groups per wave when the list is short, so that every wave has some)
  const uint64_t W = wave_count();
  const uint32_t chunks = (uint32_t)std::min<uint64_t>(
      kMatChunks, std::max<uint64_t>(1, (S + 64 * W - 1) / (64 * W)));
  for (uint64_t base = wave_base() * chunks; base < S; base += wave_stride() * chunks) {
    unsigned long long mine = 0;
    for (uint32_t k = 0; k < chunks; ++k) {
      const uint64_t i = base + (uint64_t)k * 64 + lane();
      if (i < S) {
        const uint32_t u = wl_get(wl.small, wl.cap, pre_s, (uint32_t)i);
        mine += (uint64_t)off[u + 1] - off[u];
      }
    }
    const unsigned long long all = wave_sum(mine);
    unsigned long long pos = 0;
    if (all && lane() == 0) pos = atomicAdd(&c->edge_count, all);
    pos = __shfl(pos, 0);
    for (uint32_t k = 0; k < chunks; ++k) {
      const uint64_t i = base + (uint64_t)k * 64 + lane();
      uint32_t u = 0, deg = 0;
      uint64_t b = 0;
      if (i < S) {
        u = wl_get(wl.small, wl.cap, pre_s, (uint32_t)i);
        b = off[u];
        deg = (uint32_t)((uint64_t)off[u + 1] - b);
      }
      uint32_t total;
      const uint32_t o = wave_exclusive(deg, &total);
      for (uint32_t j = 0; j < deg; ++j) {
        esrc[pos + o + j] = u;
        edst[pos + o + j] = nbrs[b + j];
      }
      pos += total;
    }
  }
  for (uint64_t w = wave_index(); w < (uint64_t)M + G; w += wave_count()) {
    uint32_t u;
    uint64_t b, e;
    if (w < M) {
      u = wl_get(wl.medium, wl.cap, pre_m, (uint32_t)w);
      b = off[u];
      e = off[u + 1];
    } else {
      const uint2 sg = wl.segs[w - M];
      u = sg.x;
      b = (uint64_t)off[u] + (uint64_t)sg.y * kSeg;
      e = off[u + 1];
      if (e > b + kSeg) e = b + kSeg;
    }
    unsigned long long pos = 0;
    if (lane() == 0) pos = atomicAdd(&c->edge_count, (unsigned long long)(e - b));
    pos = __shfl(pos, 0);
    for (uint64_t x = b + lane(); x < e; x += 64) {
      esrc[pos + (x - b)] = u;
      edst[pos + (x - b)] = nbrs[x];
    }
  }
}

__global__ void k_materialize_coo(const uint32_t* a, const uint32_t* b, uint64_t m, Ctrl* c,
                                  uint32_t* esrc, uint32_t* edst) {
  if (gtid() == 0) c->edge_count = m;
  for (uint64_t e = gtid(); e < m; e += wave_stride()) {
    esrc[e] = a[e];
    edst[e] = b[e];
  }
}

// --------------------------------------------------------------- rounds (SV, LT, LP)
// Rounds run K at a time between host checks.  round_begin decides on the
// device whether the previous round changed anything; once a round makes no
// change every later kernel of the batch returns at once.
__global__ void k_round_begin(Ctrl* c, uint32_t r) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (r > 0 && c->changed[(r - 1) % kRoundSlots] == 0) c->done = 1;
    c->changed[r % kRoundSlots] = 0;
  }
}

__device__ __forceinline__ void mark_changed(Ctrl* c, uint32_t slot) {
  __hip_atomic_store(&c->changed[slot], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// One flag store per workgroup (every thread of the block must call it):
// write-throughs of one word from every wave of a launch queue at the L2.
__device__ __forceinline__ void block_mark_changed(Ctrl* c, uint32_t slot, bool any) {
  if (__syncthreads_or(any) && threadIdx.x == 0) mark_changed(c, slot);
}

// Shiloach-Vishkin round (Appendix A.3): for each edge, the larger of the two
// labels, if it was a root at the start of the round, is lowered to the
// smaller with writeMin.  snapshot = 1 reads both labels from the round-start
// copy (used when recording a spanning forest).
__global__ void k_sv_round(const uint32_t* __restrict__ esrc, const uint32_t* __restrict__ edst,
                           Ctrl* c, uint32_t* P, const uint32_t* __restrict__ prev, uint32_t slot,
                           int snapshot) {
  if (c->done) return;
  const uint64_t E = c->edge_count;
  bool any = false;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += wave_stride()) {
    uint32_t u = esrc[e], v = edst[e];
    uint32_t pu = snapshot ? prev[u] : ld(&P[u]);
    uint32_t pv = snapshot ? prev[v] : ld(&P[v]);
    uint32_t l = pu < pv ? pu : pv, h = pu < pv ? pv : pu;
    // the atomic only when it can lower the slot: once a component's root
    // holds its final label, the many edges into it would otherwise all queue
    // on that one word (a read may be stale, but P only decreases, so a
    // stale value is never below the current one)
    if (l != h && prev[h] == h && ld(&P[h]) > l) {
      amin(&P[h], l);
      any = true;
    }
  }
  block_mark_changed(c, slot, any);
}

// Forest edge for SV: an edge whose round-start labels are {l, h} and whose
// larger root h ended the hooking step at exactly l is a valid forest edge for
// slot h; the first such edge claims the slot.
__global__ void k_sv_record(const uint32_t* __restrict__ esrc, const uint32_t* __restrict__ edst,
                            const Ctrl* c, const uint32_t* P, const uint32_t* __restrict__ prev,
                            uint32_t* fu, uint32_t* fv) {
  if (c->done) return;
  const uint64_t E = c->edge_count;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += wave_stride()) {
    uint32_t u = esrc[e], v = edst[e];
    uint32_t pu = prev[u], pv = prev[v];
    uint32_t l = pu < pv ? pu : pv, h = pu < pv ? pv : pu;
    if (l != h && ld(&P[h]) == l) {
      uint32_t x = kEmpty;
      if (cas(&fu[h], x, u)) fv[h] = v;
    }
  }
}

// FullShortcut over every vertex, then prev = P (Shiloach-Vishkin round end;
// Liu-Tarjan FullShortcut).  Changes count as progress for LT.
__global__ void k_shortcut_full(Ctrl* c, uint32_t* P, uint32_t* prev, uint32_t n, uint32_t slot,
                                int count_change) {
  if (c->done) return;
  bool any = false;
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += wave_stride()) {
    uint32_t p = P[v];
    uint32_t r = p;
    if (p != v) r = root_plain(P, p);
    if (r != p) {
      P[v] = r;
      any = true;
    }
    if (prev) prev[v] = r;
  }
  block_mark_changed(c, slot, count_change && any);
}

// Liu-Tarjan Shortcut: one pointer-jumping step, P[v] = P[P[v]].
__global__ void k_shortcut_one(Ctrl* c, uint32_t* P, uint32_t* prev, uint32_t n, uint32_t slot) {
  if (c->done) return;
  bool any = false;
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += wave_stride()) {
    uint32_t p = ld(&P[v]);
    uint32_t g = ld(&P[p]);
    if (g < p) {
      amin(&P[v], g);
      any = true;
    }
    if (prev) prev[v] = ld(&P[v]);
  }
  block_mark_changed(c, slot, any);
}

// Liu-Tarjan connect + update (Appendix A.4) with in-place atomic minimum:
// connect 0 = Connect (endpoints to each other), 1 = ParentConnect (parents to
// each other's parents), 2 = ExtendedConnect (parents to both endpoints and
// both parents).  root_update = 1 applies a message only to a vertex that was a
// root at the start of the round.
__device__ __forceinline__ bool lt_send(uint32_t* P, const uint32_t* prev, uint32_t to,
                                        uint32_t val, int root_update) {
  if (root_update && prev[to] != to) return false;
  if (ld(&P[to]) <= val) return false;  // cannot lower it (P only decreases)
  return amin(&P[to], val) > val;
}

__global__ void k_lt_round(const uint32_t* __restrict__ esrc, const uint32_t* __restrict__ edst,
                           Ctrl* c, uint32_t* P, const uint32_t* __restrict__ prev, uint32_t slot,
                           int connect, int root_update) {
  if (c->done) return;
  const uint64_t E = c->edge_count;
  bool any = false;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += wave_stride()) {
    uint32_t v = esrc[e], w = edst[e];
    if (v == kEmpty) continue;  // removed by Alter
    if (connect == 0) {
      any |= lt_send(P, prev, v, w, root_update);
      any |= lt_send(P, prev, w, v, root_update);
    } else {
      uint32_t pv = ld(&P[v]), pw = ld(&P[w]);
      if (pv == pw) continue;
      any |= lt_send(P, prev, pv, pw, root_update);
      any |= lt_send(P, prev, pw, pv, root_update);
      if (connect == 2) {
        any |= lt_send(P, prev, v, pw, root_update);
        any |= lt_send(P, prev, w, pv, root_update);
      }
    }
  }
  block_mark_changed(c, slot, any);
}

// Liu-Tarjan Alter: replace each edge by the edge between its endpoints'
// parents; an edge whose parents coincide is removed.
__global__ void k_lt_alter(uint32_t* esrc, uint32_t* edst, Ctrl* c, const uint32_t* P,
                           uint32_t slot) {
  if (c->done) return;
  const uint64_t E = c->edge_count;
  bool any = false;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += wave_stride()) {
    uint32_t v = esrc[e];
    if (v == kEmpty) continue;
    uint32_t w = edst[e];
    uint32_t pv = P[v], pw = P[w];
    if (pv == pw) {
      esrc[e] = kEmpty;
    } else if (pv != v || pw != w) {
      esrc[e] = pv;
      edst[e] = pw;
      any = true;
    }
  }
  block_mark_changed(c, slot, any);
}

// Label propagation round: across an edge with different labels the larger
// label is lowered to the smaller.  After sampling, the vertices labelled L_max
// never process their edges, so the edges inside that group are never seen
// and its members must move together: every vertex whose entry holds L_max is
// treated as one node whose current label lives at P[L_max] (lowering it
// lowers the whole group, which finalisation then follows).  Without sampling
// L_max is the empty sentinel and this is plain label propagation.
__device__ __forceinline__ void lp_label(const uint32_t* P, uint32_t x, uint32_t group,
                                         uint32_t* label, uint32_t* slot) {
  uint32_t l = ld(&P[x]);
  uint32_t t = x;
  if (l == group) {
    t = group;
    l = ld(&P[group]);
  }
  *label = l;
  *slot = t;
}

__global__ void k_lp_round(const uint32_t* __restrict__ esrc, const uint32_t* __restrict__ edst,
                           Ctrl* c, uint32_t* P, uint32_t slot) {
  if (c->done) return;
  const uint64_t E = c->edge_count;
  const uint32_t group = c->lmax;
  bool any = false;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += wave_stride()) {
    uint32_t lu, tu, lv, tv;
    lp_label(P, esrc[e], group, &lu, &tu);
    lp_label(P, edst[e], group, &lv, &tv);
    if (lu == lv) continue;
    if (lu > lv) {
      if (amin(&P[tu], lv) > lv) any = true;
    } else {
      if (amin(&P[tv], lu) > lu) any = true;
    }
  }
  block_mark_changed(c, slot, any);
}

// Workgroup partial results of the source choice (argmax of the degree) and
// of the BFS component's minimum id: workgroup b stores its result in slot b
// and one workgroup of kFoldThreads folds the slots, so no workgroup takes an
// atomic on a single address (device atomics there serialise at about 11 ns
// each, which for thousands of workgroups is most of such a kernel's time).
constexpr uint32_t kBfsSlots = 8192;
constexpr uint32_t kFoldThreads = 1024;

// Maximum (kMax) or minimum of slots[0, nslots), nslots <= kBfsSlots, over a
// workgroup of kFoldThreads: each thread issues its eight loads before it
// combines them, so the fold waits about one load latency, not eight.  The
// result is valid in thread 0; `none` is the identity.
template <bool kMax, typename T>
__device__ __forceinline__ T fold_slots(const T* __restrict__ slots, uint32_t nslots, T none) {
  constexpr uint32_t kPer = kBfsSlots / kFoldThreads;
  T v[kPer];
#pragma unroll
  for (uint32_t j = 0; j < kPer; ++j) {
    const uint32_t i = threadIdx.x + j * kFoldThreads;
    v[j] = i < nslots ? slots[i] : none;
  }
  T x = none;
#pragma unroll
  for (uint32_t j = 0; j < kPer; ++j) x = kMax ? (v[j] > x ? v[j] : x) : (v[j] < x ? v[j] : x);
  for (int d = 32; d >= 1; d >>= 1) {
    const T o = __shfl_xor(x, d);
    x = kMax ? (o > x ? o : x) : (o < x ? o : x);
  }
  __shared__ T part[kFoldThreads / 64];
  if (lane() == 0) part[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0)
    for (uint32_t w = 1; w < kFoldThreads / 64; ++w)
      x = kMax ? (part[w] > x ? part[w] : x) : (part[w] < x ? part[w] : x);
  return x;
}

template <typename OffT>
__global__ void k_bfs_argmax(const OffT* __restrict__ off, uint32_t n,
                             unsigned long long* __restrict__ slots) {
  // four consecutive vertices per lane: their five row bounds are loaded
  // together, so a lane's iterations are not one dependent load each
  unsigned long long best = 0;
  for (uint64_t base = wave_base() * 4; base < n; base += wave_stride() * 4) {
    const uint64_t v0 = base + 4 * lane();
    uint64_t o[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) o[j] = v0 + j <= n ? (uint64_t)off[v0 + j] : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (v0 + j >= n) break;
      uint64_t deg = o[j + 1] - o[j];
      if (deg > 0xFFFFFFFEull) deg = 0xFFFFFFFEull;
      const unsigned long long key = ((deg + 1) << 32) | (0xFFFFFFFFull - (v0 + j));
      best = key > best ? key : best;
    }
  }
  // every lane of a wave ran the same iterations, so all are active here;
  // then the workgroup's waves combine in LDS into the workgroup's slot
  __shared__ unsigned long long wmax[16];
  best = wave_max(best);
  if (lane() == 0) wmax[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t w = 1; w < (blockDim.x + 63) / 64; ++w) best = wmax[w] > best ? wmax[w] : best;
    slots[blockIdx.x] = best;
  }
}

// A level's discovered vertices and their row entries are added up by the
// level's workgroups into 64 stripes (one 128-byte line each, workgroup i into
// stripe i mod 64) instead of into one counter: device atomics on a single
// address serialise at about 11 ns each, which for thousands of workgroups is
// most of a level.  The next level's decision kernel folds the stripes of its
// frontier into the counters and clears them.
struct alignas(128) BfsStripe {
  unsigned long long count, edges;
};
constexpr uint32_t kBfsStripes = 64;

__device__ __forceinline__ void bfs_stripe_add(BfsStripe* st, uint32_t level_slot,
                                               unsigned long long count,
                                               unsigned long long edges) {
  // whole workgroup: wave sums, then one atomic pair from thread 0
  __shared__ unsigned long long part[2][16];
  count = wave_sum(count);
  edges = wave_sum(edges);
  if (lane() == 0) {
    part[0][threadIdx.x >> 6] = count;
    part[1][threadIdx.x >> 6] = edges;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t w = 1; w < (blockDim.x + 63) / 64; ++w) {
      count += part[0][w];
      edges += part[1][w];
    }
    BfsStripe* t = st + level_slot * kBfsStripes + (blockIdx.x % kBfsStripes);
    if (count) atomicAdd(&t->count, count);
    if (edges) atomicAdd(&t->edges, edges);
  }
}

// Launched with one workgroup of kFoldThreads: folds the argmax slots of the
// `nslots` workgroups of k_bfs_argmax into the source and seeds the first
// frontier.
template <typename OffT>
__global__ void __launch_bounds__(kFoldThreads)
    k_bfs_start(const OffT* __restrict__ off, Ctrl* c, uint32_t* visited, uint32_t* queue0,
                BfsStripe* st, const unsigned long long* __restrict__ slots, uint32_t nslots) {
  for (uint32_t i = threadIdx.x; i < 2 * kBfsStripes; i += blockDim.x) st[i].count = st[i].edges = 0;
  const unsigned long long key = fold_slots<true>(slots, nslots, 0ull);
  if (threadIdx.x == 0) {
    uint32_t s = (uint32_t)(0xFFFFFFFFull - (key & 0xFFFFFFFFull));
    c->bfs_source = s;
    visited[s >> 5] |= 1u << (s & 31);
    queue0[0] = s;
    c->frontier_count[0] = 1;
    c->frontier_count[1] = 0;
    uint64_t deg = (uint64_t)off[s + 1] - off[s];
    c->frontier_edges[0] = deg;
    c->frontier_edges[1] = 0;
    c->explored_edges = deg;
    c->bfs_as_queue = 1;
    c->bfs_mode = 1;
    c->bfs_levels = 0;
  }
}

// One BFS level's decision, on the device (so that the host enqueues several
// levels between checks): stop when the frontier `cur` is empty; otherwise
// pick the direction with the direction-optimising rule of Beamer, Asanovic
// and Patterson (SC'12) -- switch to bottom-up once the frontier's edges
// exceed 1/alpha of the unexplored edges, back to top-down once the frontier
// holds fewer than n/beta vertices; alpha = 14, beta = 24, compared in
// integers -- note which representation change the level needs first, and
// clear the counters of frontier `nxt`.  Every later kernel of the level
// reads bfs_mode and returns at once when the level is not its kind.
// Fold the stripes of frontier `cur` into its counters (threads 0..63, one
// wave).
__device__ __forceinline__ void bfs_fold(Ctrl* c, BfsStripe* st, uint32_t cur) {
  BfsStripe* t = st + cur * kBfsStripes + threadIdx.x;
  unsigned long long sc = t->count, se = t->edges;
  t->count = t->edges = 0;
  sc = wave_sum(sc);
  se = wave_sum(se);
  if (threadIdx.x == 0 && (sc || se)) {
    c->frontier_count[cur] += (uint32_t)sc;
    c->frontier_edges[cur] += se;
    c->explored_edges += se;
  }
}

// The same fold on its own, so that the host can read the next frontier's
// size at a check (launched with 64 threads).
__global__ void k_bfs_fold(Ctrl* c, BfsStripe* st, uint32_t cur) { bfs_fold(c, st, cur); }

// force_td: the host enqueued only the top-down kernels for this level (a
// batch of levels whose frontier is far below the switch point), so the
// level stays top-down whatever the rule would pick.
__global__ void k_bfs_decide(Ctrl* c, BfsStripe* st, uint32_t cur, uint64_t m, uint32_t n,
                             int force_td) {
  __shared__ uint32_t run;
  if (threadIdx.x < 64) bfs_fold(c, st, cur);
  if (threadIdx.x == 0) {
    const uint32_t count = c->frontier_count[cur];
    run = c->bfs_mode != 0 && count != 0;
    if (!run) {
      c->bfs_mode = 0;
    } else {
      const uint64_t m_f = c->frontier_edges[cur];
      const uint64_t m_u = m > c->explored_edges ? m - c->explored_edges : 0;
      bool bu = c->bfs_mode == 2;
      if (!bu && 14 * m_f > m_u) bu = true;
      else if (bu && 24ull * count < n) bu = false;
      if (force_td) bu = false;
      const bool q = c->bfs_as_queue != 0;
      c->bfs_convert = bu ? (q ? 1u : 0u) : (q ? 0u : 2u);
      c->bfs_mode = bu ? 2u : 1u;
      c->bfs_as_queue = bu ? 0u : 1u;  // after this level
      ++c->bfs_levels;
    }
  }
  __syncthreads();
  if (!run) return;
  const uint32_t nxt = cur ^ 1u;
  for (uint32_t i = threadIdx.x; i < kSubLists; i += blockDim.x) {
    c->small_cnt[i * kCntPad] = 0;
    c->medium_cnt[i * kCntPad] = 0;
  }
  if (threadIdx.x == 0) {
    c->frontier_count[nxt] = 0;
    c->frontier_edges[nxt] = 0;
    c->seg_count = 0;
    c->queue_cursor = 0;
  }
}

// Fill of a frontier bitmap when this level is bottom-up (and, with
// need_convert, only when the frontier is first turned from a queue into bits).
__global__ void k_bfs_clear_bits(uint32_t* bits, uint32_t words, const Ctrl* c, int need_convert) {
  if (c->bfs_mode != 2 || (need_convert && c->bfs_convert != 1)) return;
  for (uint64_t i = gtid(); i < words; i += wave_stride()) bits[i] = 0u;
}

__global__ void k_bfs_level_reset(Ctrl* c, uint32_t nxt) {
  if (blockIdx.x != 0) return;
  for (uint32_t i = threadIdx.x; i < kSubLists; i += blockDim.x) {
    c->small_cnt[i * kCntPad] = 0;
    c->medium_cnt[i * kCntPad] = 0;
  }
  if (threadIdx.x == 0) {
    c->frontier_count[nxt] = 0;
    c->frontier_edges[nxt] = 0;
    c->seg_count = 0;
    c->queue_cursor = 0;
  }
}

// Top-down: sort the frontier queue into the work classes.
template <typename OffT>
__global__ void k_bfs_td_split(const OffT* __restrict__ off, const uint32_t* __restrict__ queue,
                               Ctrl* c, uint32_t cur, WorkLists wl) {
  if (c->bfs_mode != 1) return;
  const uint32_t count = c->frontier_count[cur];
  for (uint64_t base = wave_base(); base < count; base += wave_stride()) {
    const uint64_t i = base + lane();
    uint32_t u = 0;
    uint64_t deg = 0;
    if (i < count) {
      u = queue[i];
      deg = (uint64_t)off[u + 1] - off[u];
    }
    wl_push(wl, c, base >> 6, u, deg, i < count && deg > 0);
  }
}

// Top-down level with the next frontier staged in LDS: a wave claims the
// visited bits of its neighbours, appends the fresh vertices to its
// workgroup's LDS buffer (one LDS atomic per wave), and the workgroup copies
// the buffer to the next queue with one global atomic when it fills up and at
// the end (the queue's counter is a single address, where device atomics
// serialise).  Fresh vertices record their BFS-tree edge.
constexpr uint32_t kBfsStage = 4096;

// Claim w from u (valid lanes); returns whether this lane made w visited.
__device__ __forceinline__ bool bfs_claim(bool valid, uint32_t w, uint32_t* visited) {
  if (!valid) return false;
  const uint32_t bit = 1u << (w & 31);
  if (ld(&visited[w >> 5]) & bit) return false;
  return !(atomicOr(&visited[w >> 5], bit) & bit);
}

template <typename OffT>
__global__ void __launch_bounds__(256) k_bfs_td(const OffT* __restrict__ off,
                                                const uint32_t* __restrict__ nbrs, WorkLists wl,
                                                Ctrl* c, BfsStripe* st, uint32_t nxt,
                                                uint32_t* visited, uint32_t* queue_out,
                                                uint32_t* fu, uint32_t* fv) {
  __shared__ uint32_t pre_s[kSubLists + 1], pre_m[kSubLists + 1];
  __shared__ uint32_t stage[kBfsStage];
  __shared__ uint32_t staged, base_out;
  if (c->bfs_mode != 1) return;
  wl_prefix(c->small_cnt, pre_s);
  wl_prefix(c->medium_cnt, pre_m);
  if (threadIdx.x == 0) staged = 0;
  __syncthreads();
  const uint32_t S = pre_s[kSubLists], M = pre_m[kSubLists], G = c->seg_count;
  unsigned long long edges = 0;
  // Append the lanes' fresh vertices (all 64 lanes active) to the stage, or,
  // when it has no room, straight to the queue.
  auto emit = [&](bool fresh, uint32_t u, uint32_t w) {
    const unsigned long long mask = __ballot(fresh);
    if (!mask) return;
    const uint32_t cnt = (uint32_t)__popcll(mask);
    const uint32_t rank = (uint32_t)__popcll(mask & ((1ull << lane()) - 1));
    const uint32_t leader = __ffsll(mask) - 1;
    // the leader reserves cnt stage slots if they fit, else cnt queue slots
    uint32_t at = 0, in_stage = 0;
    if (lane() == leader) {
      uint32_t old = __hip_atomic_load(&staged, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      while (old + cnt <= kBfsStage) {
        if (__hip_atomic_compare_exchange_strong(&staged, &old, old + cnt, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
          at = old;
          in_stage = 1;
          break;
        }
      }
      if (!in_stage) at = atomicAdd(&c->frontier_count[nxt], cnt);
    }
    at = __shfl(at, leader);
    in_stage = __shfl(in_stage, leader);
    if (fresh) {
      if (in_stage) stage[at + rank] = w;
      else queue_out[at + rank] = w;  // straight to the queue
      edges += (uint64_t)off[w + 1] - off[w];
      if (fu) {
        fu[w] = u;
        fv[w] = w;
      }
    }
  };
  for (uint64_t b0 = wave_base(); b0 < S; b0 += wave_stride()) {
    const uint64_t i = b0 + lane();
    uint32_t u = 0;
    uint64_t b = 0, deg = 0;
    if (i < S) {
      u = wl_get(wl.small, wl.cap, pre_s, (uint32_t)i);
      b = off[u];
      deg = (uint64_t)off[u + 1] - b;
    }
    for (uint32_t j = 0; __ballot(j < deg); ++j) {
      const bool valid = j < deg;
      const uint32_t w = valid ? nbrs[b + j] : 0u;
      emit(bfs_claim(valid, w, visited), u, w);
    }
  }
  for (uint64_t wi = wave_index(); wi < (uint64_t)M + G; wi += wave_count()) {
    uint32_t u;
    uint64_t b, e;
    if (wi < M) {
      u = wl_get(wl.medium, wl.cap, pre_m, (uint32_t)wi);
      b = off[u];
      e = off[u + 1];
    } else {
      const uint2 sg = wl.segs[wi - M];
      u = sg.x;
      b = (uint64_t)off[u] + (uint64_t)sg.y * kSeg;
      e = off[u + 1];
      if (e > b + kSeg) e = b + kSeg;
    }
    for (uint64_t x0 = b; x0 < e; x0 += 64) {
      const uint64_t x = x0 + lane();
      const bool valid = x < e;
      const uint32_t w = valid ? nbrs[x] : 0u;
      emit(bfs_claim(valid, w, visited), u, w);
    }
  }
  __syncthreads();
  const uint32_t kept = staged;
  if (threadIdx.x == 0 && kept) base_out = atomicAdd(&c->frontier_count[nxt], kept);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < kept; i += blockDim.x) queue_out[base_out + i] = stage[i];
  // the vertex count is the queue cursor itself; the row entries go to a stripe
  bfs_stripe_add(st, nxt, 0, edges);
}

__global__ void k_queue_to_bits(const uint32_t* __restrict__ queue, const Ctrl* c, uint32_t cur,
                                uint32_t* bits) {
  if (c->bfs_mode != 2 || c->bfs_convert != 1) return;
  const uint32_t count = c->frontier_count[cur];
  for (uint64_t i = gtid(); i < count; i += wave_stride()) {
    const uint32_t w = queue[i];
    atomicOr(&bits[w >> 5], 1u << (w & 31));
  }
}

// Rebuild a frontier queue from its bitmap (queue_cursor is the append cursor).
__global__ void k_bits_to_queue(const uint32_t* __restrict__ bits, uint32_t words, Ctrl* c,
                                uint32_t* queue) {
  if (c->bfs_mode != 1 || c->bfs_convert != 2) return;
  for (uint64_t base = wave_base(); base < words; base += wave_stride()) {
    const uint64_t i = base + lane();
    uint32_t word = i < words ? bits[i] : 0u;
    uint32_t pos = wave_reserve(&c->queue_cursor, (uint32_t)__popc(word));
    while (word) {
      const uint32_t b = __ffs(word) - 1;
      queue[pos++] = (uint32_t)(i * 32 + b);
      word &= word - 1;
    }
  }
}

// Bottom-up level: every unvisited vertex looks for a neighbour in the
// frontier, and the first one in its row becomes its parent (the choice a
// sequential scan of the row makes).  A lane takes four consecutive vertices,
// so eight lanes share one visited word and write it once, with no atomic:
// only this level's lanes for those vertices change it.  The first kBuHead
// entries of the four rows are tried with their loads in flight together;
// what remains of the rows is then spread over the wave, 64 entries a step,
// so that one long row does not keep 63 lanes waiting, and a row whose parent
// is known is skipped from the next step on.  Entries of one row found in the
// same step are resolved by an LDS minimum over their positions.
#ifndef GCONN_BU_HEAD
#define GCONN_BU_HEAD 2
#endif
constexpr uint32_t kBuHead = GCONN_BU_HEAD;
constexpr uint32_t kBuBlock = 256;
constexpr uint32_t kBuSlots = 256;  // vertices of one wave iteration

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <typename OffT>
__global__ void __launch_bounds__(kBuBlock)
k_bfs_bu(const OffT* __restrict__ off, const uint32_t* __restrict__ nbrs, uint32_t n,
         uint32_t* visited, const uint32_t* __restrict__ fr_in, uint32_t* fr_out, Ctrl* c,
         BfsStripe* st, uint32_t nxt, uint32_t* fu, uint32_t* fv) {
  if (c->bfs_mode != 2) return;
  // per wave: first flattened position of each slot's remaining entries,
  // where they start in nbrs, and the best (position << 32 | neighbour) found
  __shared__ uint64_t s_ex[kBuBlock / 64][kBuSlots + 1];
  __shared__ uint64_t s_start[kBuBlock / 64][kBuSlots];
  __shared__ unsigned long long s_best[kBuBlock / 64][kBuSlots];
  const uint32_t wv = threadIdx.x >> 6, ln = lane();
  constexpr unsigned long long kNone = ~0ull;
  unsigned long long found = 0, found_edges = 0;
  const uint64_t quads = ((uint64_t)n + 3) / 4;
  for (uint64_t base = wave_base(); base < quads; base += wave_stride()) {
    const uint64_t q = base + ln;
    const uint64_t v0 = q * 4;
    const uint32_t sh = (uint32_t)(v0 & 31);
    // the visited word and the five row bounds are loaded together (a
    // visited vertex's row is then ignored), and so are the first kBuHead
    // entries of the four rows and their frontier words: three dependent
    // loads in all
    const bool live = q < quads;
    const uint32_t vis = live ? visited[v0 >> 5] : 0xFFFFFFFFu;
    OffT ob[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) ob[j] = live ? off[v0 + j < n ? v0 + j : n] : (OffT)0;
    OffT cur[4], end[4];
    uint32_t deg[4], par[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool todo = live && v0 + j < n && !((vis >> (sh + j)) & 1u);
      cur[j] = ob[j];
      end[j] = todo ? ob[j + 1] : ob[j];
      deg[j] = (uint32_t)(end[j] - cur[j]);
      par[j] = kEmpty;
    }
    {
      uint32_t w[4][kBuHead], f[4][kBuHead];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (uint32_t h = 0; h < kBuHead; ++h) w[j][h] = h < end[j] - cur[j] ? nbrs[cur[j] + h] : 0u;
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (uint32_t h = 0; h < kBuHead; ++h)
          f[j][h] = h < end[j] - cur[j] ? fr_in[w[j][h] >> 5] >> (w[j][h] & 31) : 0u;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        bool hit = false;
#pragma unroll
        for (uint32_t h = 0; h < kBuHead; ++h) {
          if (!hit && (f[j][h] & 1u)) {
            par[j] = w[j][h];
            hit = true;
          }
        }
        cur[j] = (hit || end[j] - cur[j] <= kBuHead) ? end[j] : cur[j] + kBuHead;
      }
    }
    uint64_t rem[4], lane_rem = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      rem[j] = (uint64_t)(end[j] - cur[j]);
      lane_rem += rem[j];
    }
    // exclusive prefix of the remaining entries over the wave (64-bit: one
    // row may hold more than 2^32 / 256 entries)
    uint64_t incl = lane_rem;
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t y = __shfl_up(incl, d);
      if (ln >= (uint32_t)d) incl += y;
    }
    const uint64_t total = __shfl(incl, 63);
    if (total) {
      uint64_t ex = incl - lane_rem;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        s_ex[wv][ln * 4 + j] = ex;
        s_start[wv][ln * 4 + j] = (uint64_t)cur[j];
        s_best[wv][ln * 4 + j] = kNone;
        ex += rem[j];
      }
      if (ln == 63) s_ex[wv][kBuSlots] = total;
      wave_lds_sync();
      uint64_t i0 = 0;
      for (;;) {
        const uint64_t i = i0 + ln;
        if (i < total) {
          // the slot whose remaining entries hold position i: the last slot
          // starting at or before i (empty slots start where the next does)
          uint32_t sl = 0;
          for (uint32_t step = kBuSlots / 2; step; step >>= 1)
            if (s_ex[wv][sl + step] <= i) sl += step;
          if (s_best[wv][sl] == kNone) {
            const uint64_t k = i - s_ex[wv][sl];
            const uint32_t w = nbrs[s_start[wv][sl] + k];
            if ((fr_in[w >> 5] >> (w & 31)) & 1u)
              atomicMin(&s_best[wv][sl], (k << 32) | w);
          }
        }
        wave_lds_sync();
        i0 += 64;
        if (i0 >= total) break;
        // continue at the first position >= i0 of a slot still without parent
        unsigned long long nx = kNone;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t sl = ln * 4 + j;
          const uint64_t a = s_ex[wv][sl], e = a + rem[j];
          if (rem[j] && e > i0 && s_best[wv][sl] == kNone) {
            const uint64_t at = a > i0 ? a : i0;
            nx = at < nx ? at : nx;
          }
        }
        for (int d = 32; d >= 1; d >>= 1) {
          const unsigned long long y = __shfl_xor(nx, d);
          nx = y < nx ? y : nx;
        }
        if (nx == kNone) break;
        i0 = nx;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const unsigned long long b = s_best[wv][ln * 4 + j];
        if (rem[j] && b != kNone) par[j] = (uint32_t)b;
      }
      wave_lds_sync();  // the next iteration rewrites the slots
    }
    uint32_t mask = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (par[j] != kEmpty) {
        mask |= 1u << (sh + j);
        ++found;
        found_edges += deg[j];
        if (fu) {
          fu[v0 + j] = par[j];
          fv[v0 + j] = (uint32_t)(v0 + j);
        }
      }
    }
    // the eight lanes of one visited word combine their bits; the first
    // writes the word (it is the only writer of those 32 vertices' bits)
    mask |= __shfl_xor(mask, 1);
    mask |= __shfl_xor(mask, 2);
    mask |= __shfl_xor(mask, 4);
    if ((ln & 7) == 0 && mask) {
      visited[v0 >> 5] = vis | mask;
      fr_out[v0 >> 5] = mask;
    }
  }
  bfs_stripe_add(st, nxt, found, found_edges);
}

// Re-root the BFS component at its minimum id (the BFS labels reached vertices
// with the source, which is not the component minimum).
__global__ void k_bfs_min(const uint32_t* __restrict__ visited, uint32_t words,
                          uint32_t* __restrict__ slots) {
  // the first visited id of the lane's words, then of the wave and the
  // workgroup, stored in the workgroup's slot
  uint32_t best = kEmpty;
  for (uint64_t base = wave_base(); base < words; base += wave_stride()) {
    const uint64_t i = base + lane();
    const uint32_t w = i < words ? visited[i] : 0u;
    if (w) {
      const uint32_t id = (uint32_t)(i * 32 + (__ffs(w) - 1));
      best = id < best ? id : best;
    }
  }
  for (int d = 32; d >= 1; d >>= 1) {
    const uint32_t o = __shfl_xor(best, d);
    best = o < best ? o : best;
  }
  __shared__ uint32_t wmin[16];
  if (lane() == 0) wmin[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t w = 1; w < (blockDim.x + 63) / 64; ++w) best = wmin[w] < best ? wmin[w] : best;
    slots[blockIdx.x] = best;
  }
}

// One workgroup of kFoldThreads folds the `nslots` slots of k_bfs_min into
// the component minimum.
__global__ void __launch_bounds__(kFoldThreads)
    k_bfs_min_fold(const uint32_t* __restrict__ slots, uint32_t nslots, Ctrl* c) {
  const uint32_t best = fold_slots<false>(slots, nslots, kEmpty);
  if (threadIdx.x == 0) c->comp_min = best;
}

// Every slot is written, four per lane: a visited vertex gets the component
// minimum, any other keeps its own id (no BFS kernel writes P before this, so
// that is the value it holds); whole lines are written instead of scattered
// words.
__global__ void k_bfs_label(const uint32_t* __restrict__ visited, uint32_t n, const Ctrl* c,
                            uint32_t* P) {
  const uint32_t r = c->comp_min;
  const bool vec = (reinterpret_cast<uintptr_t>(P) % 16) == 0;
  for (uint64_t v0 = 4 * gtid(); v0 < n; v0 += 4 * wave_stride()) {
    const uint32_t word = visited[v0 >> 5] >> (v0 & 31);
    uint32_t q[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) q[j] = (word >> j) & 1u ? r : (uint32_t)(v0 + j);
    if (vec && v0 + 4 <= n) {
      *reinterpret_cast<uint4*>(P + v0) = make_uint4(q[0], q[1], q[2], q[3]);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (v0 + j < n) P[v0 + j] = q[j];
    }
  }
}

// --------------------------------------------------------------- incremental
template <class R>
__global__ void k_query(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b, uint64_t q,
                        uint32_t* P, uint8_t* out, int ac) {
  for (uint64_t i = gtid(); i < q; i += wave_stride()) {
    const uint32_t ra = find<R::kFind>(P, a[i], ac != 0);
    const uint32_t rb = find<R::kFind>(P, b[i], ac != 0);
    out[i] = (uint8_t)(ra == rb);
  }
}

// Mixed batches (the paper's incremental batches mix inserts and queries): all
// inserts of the batch first, then every query, so the answers do not depend
// on how the two interleave on the device.
template <class R>
__global__ void k_unite_kind(const uint8_t* __restrict__ kind, const uint32_t* __restrict__ a,
                             const uint32_t* __restrict__ b, uint64_t m, LinkCtx lc) {
  for (uint64_t e = gtid(); e < m; e += wave_stride())
    if (kind[e] == GCONN_REQ_INSERT) R::unite(lc, a[e], b[e]);
}

template <class R>
__global__ void k_query_kind(const uint8_t* __restrict__ kind, const uint32_t* __restrict__ a,
                             const uint32_t* __restrict__ b, uint64_t q, uint32_t* P,
                             uint8_t* out, int ac) {
  for (uint64_t i = gtid(); i < q; i += wave_stride()) {
    uint8_t r = 0;
    if (kind[i] == GCONN_REQ_QUERY)
      r = (uint8_t)(find<R::kFind>(P, a[i], ac != 0) == find<R::kFind>(P, b[i], ac != 0));
    out[i] = r;
  }
}

__global__ void k_validate_kinds(const uint8_t* kind, uint64_t m, Ctrl* c) {
  for (uint64_t e = gtid(); e < m; e += wave_stride())
    if (kind[e] > GCONN_REQ_QUERY) c->err = 1;
}

// =============================================================== host side
namespace {

constexpr uint32_t kPersistentBlocks = 2048;  // round kernels: 256 CUs x 8 workgroups

// The k-out pre-link covers first-k sampling with k <= 2.
// The slot-array k-out passes (k_kout_local, then k_kout_residual): the LDS
// local-first variant, or the plain two-pass schedule.
bool kout_local_applies(const gconn_options& o) {
  return (o.kout_local || o.schedule == 4) && o.sample == GCONN_SAMPLE_KOUT && !o.kout_random &&
         o.k <= 2;
}
bool kout_flat_applies(const gconn_options& o) {
  return !kout_local_applies(o) && o.schedule == 5 && o.sample == GCONN_SAMPLE_KOUT &&
         !o.kout_random && o.k <= 2;
}
// The automatic k-out schedule (schedule 0, first k <= 2): a locality probe
// on the device chooses between the local-first passes and the one-pass kernel.
bool kout_auto_local_applies(const gconn_options& o) {
  return o.schedule == 0 && o.sample == GCONN_SAMPLE_KOUT && !o.kout_random && o.k <= 2 &&
         !o.kout_local && !o.kout_prelink;
}
// The XCD-bucketed k-out passes (k_kx_stream, k_kx_flatten, k_kx_unite).
bool kout_xcd_applies(const gconn_options& o) {
  return !kout_local_applies(o) && o.schedule == 6 && o.sample == GCONN_SAMPLE_KOUT &&
         !o.kout_random && o.k <= 2;
}
// Id-range width (log2) of the XCD groups: at least 512 ranges per graph.
uint32_t kx_shift(uint32_t n) {
  uint32_t bits = 0;
  while (bits < 32 && (1ull << bits) < n) ++bits;
  return bits > 14 ? bits - 9 : 5;
}
bool kout_prelink_applies(const gconn_options& o) {
  return !kout_local_applies(o) && !kout_xcd_applies(o) && (o.kout_prelink || kout_flat_applies(o)) &&
         o.sample == GCONN_SAMPLE_KOUT && !o.kout_random && o.k <= 2;
}

template <class Fn>
gconn_status with_rule(int link, int find_rule, int splice, Fn&& fn) {
  switch (link) {
    case GCONN_LINK_ECL:
      return fn(Rule<kUnionAsync, kFindHalve, 0>{});
    case GCONN_LINK_AFFOREST:
      return fn(Rule<kUnionAfforest, kFindNaive, 0>{});
    case GCONN_LINK_REM_LOCK:
      if (splice == kSpliceAtomic) {
        switch (find_rule) {
          case kFindNaive: return fn(Rule<kUnionRemLock, kFindNaive, kSpliceAtomic>{});
          case kFindSplit: return fn(Rule<kUnionRemLock, kFindSplit, kSpliceAtomic>{});
          default: return fn(Rule<kUnionRemLock, kFindHalve, kSpliceAtomic>{});
        }
      }
      if (splice == kSpliceSplitOne) {
        switch (find_rule) {
          case kFindNaive: return fn(Rule<kUnionRemLock, kFindNaive, kSpliceSplitOne>{});
          case kFindSplit: return fn(Rule<kUnionRemLock, kFindSplit, kSpliceSplitOne>{});
          default: return fn(Rule<kUnionRemLock, kFindHalve, kSpliceSplitOne>{});
        }
      }
      switch (find_rule) {
        case kFindNaive: return fn(Rule<kUnionRemLock, kFindNaive, kSpliceHalveOne>{});
        case kFindSplit: return fn(Rule<kUnionRemLock, kFindSplit, kSpliceHalveOne>{});
        default: return fn(Rule<kUnionRemLock, kFindHalve, kSpliceHalveOne>{});
      }
    case GCONN_LINK_ASYNC:
      switch (find_rule) {
        case kFindNaive: return fn(Rule<kUnionAsync, kFindNaive, 0>{});
        case kFindSplit: return fn(Rule<kUnionAsync, kFindSplit, 0>{});
        case kFindHalve: return fn(Rule<kUnionAsync, kFindHalve, 0>{});
        default: return fn(Rule<kUnionAsync, kFindCompress, 0>{});
      }
    case GCONN_LINK_HOOKS:
      switch (find_rule) {
        case kFindNaive: return fn(Rule<kUnionHooks, kFindNaive, 0>{});
        case kFindSplit: return fn(Rule<kUnionHooks, kFindSplit, 0>{});
        case kFindHalve: return fn(Rule<kUnionHooks, kFindHalve, 0>{});
        default: return fn(Rule<kUnionHooks, kFindCompress, 0>{});
      }
    case GCONN_LINK_EARLY:
      switch (find_rule) {
        case kFindNaive: return fn(Rule<kUnionEarly, kFindNaive, 0>{});
        case kFindSplit: return fn(Rule<kUnionEarly, kFindSplit, 0>{});
        case kFindHalve: return fn(Rule<kUnionEarly, kFindHalve, 0>{});
        default: return fn(Rule<kUnionEarly, kFindCompress, 0>{});
      }
    case GCONN_LINK_REM_CAS:
      if (splice == kSpliceAtomic) {
        switch (find_rule) {
          case kFindNaive: return fn(Rule<kUnionRemCas, kFindNaive, kSpliceAtomic>{});
          case kFindSplit: return fn(Rule<kUnionRemCas, kFindSplit, kSpliceAtomic>{});
          default: return fn(Rule<kUnionRemCas, kFindHalve, kSpliceAtomic>{});
        }
      }
      if (splice == kSpliceSplitOne) {
        switch (find_rule) {
          case kFindNaive: return fn(Rule<kUnionRemCas, kFindNaive, kSpliceSplitOne>{});
          case kFindSplit: return fn(Rule<kUnionRemCas, kFindSplit, kSpliceSplitOne>{});
          default: return fn(Rule<kUnionRemCas, kFindHalve, kSpliceSplitOne>{});
        }
      } else {
        switch (find_rule) {
          case kFindNaive: return fn(Rule<kUnionRemCas, kFindNaive, kSpliceHalveOne>{});
          case kFindSplit: return fn(Rule<kUnionRemCas, kFindSplit, kSpliceHalveOne>{});
          default: return fn(Rule<kUnionRemCas, kFindHalve, kSpliceHalveOne>{});
        }
      }
    default:
      // SV / LT / LP: the sampling phase still runs union-find.
      return fn(Rule<kUnionAsync, kFindSplit, 0>{});
  }
}

struct Run {
  const gconn_graph& g;
  uint32_t* P;
  uint32_t* fu;
  uint32_t* fv;
  uint8_t* ws;
  const WsLayout& L;
  const gconn_options& o;
  bool want_stats;
  hipStream_t s;
  uint32_t block;
  Ctrl* ctrl;
  WorkLists wl;
  uint32_t* hooks;
  uint32_t* probe_part = nullptr;  // set when k_init ran the automatic schedule's probe
  uint64_t rounds = 0;

  Run(const gconn_graph& g_, uint32_t* P_, uint32_t* fu_, uint32_t* fv_, uint8_t* ws_,
      const WsLayout& L_, const gconn_options& o_, bool st, hipStream_t s_)
      : g(g_), P(P_), fu(fu_), fv(fv_), ws(ws_), L(L_), o(o_), want_stats(st), s(s_) {
    block = (uint32_t)o.block;
    ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
    wl.small = reinterpret_cast<uint32_t*>(ws + L.small);
    wl.medium = reinterpret_cast<uint32_t*>(ws + L.medium);
    wl.segs = reinterpret_cast<uint2*>(ws + L.segs);
    wl.cap = L.sub_cap;
    hooks = needs_claims(o.link) ? reinterpret_cast<uint32_t*>(ws + L.hooks) : nullptr;
  }

  uint32_t gridN(uint64_t items) const { return grid_for(items, block); }

  // Sampling grid: one lane per 6 vertices up to 2^18 vertices, one per 16
  // beyond, never above `full`.  With every vertex of a small graph in flight
  // at once, the unions of all the vertices whose first sampled neighbours are
  // the same few small ids hit those roots together and serialise (measured:
  // ER with 1e5 vertices 3x, with 1e6 vertices 3.6x slower at a full grid);
  // graphs of millions of vertices keep the full grid.
  uint32_t contention_grid(uint32_t full, uint64_t n) const {
    const uint64_t per_lane = n <= (1ull << 18) ? 6 : 16;
    const uint64_t want = (n + per_lane * block - 1) / (per_lane * block);
    return (uint32_t)std::max<uint64_t>(16, std::min<uint64_t>(full, want));
  }

  // Liu-Tarjan variants whose connect rule sends labels to the edge endpoints
  // under Update (CUSA, CUFA, EUSA, EUS, EUFA, EUF) may re-point a vertex of
  // the L_max group away from its group, whose internal edges the finish never
  // sees; they process every vertex instead of skipping the L_max group.
  bool skip_lmax() const {
    if (o.link != GCONN_LINK_LT) return true;
    switch (o.lt_variant) {
      case GCONN_LT_CUSA: case GCONN_LT_CUFA: case GCONN_LT_EUSA: case GCONN_LT_EUS:
      case GCONN_LT_EUFA: case GCONN_LT_EUF:
        return false;
      default:
        return true;
    }
  }

  LinkCtx link_ctx() const {
    LinkCtx c;
    c.P = P;
    c.H = hooks;
    c.fu = fu;
    c.fv = fv;
    c.hooks = want_stats ? &ctrl->stat_hooks : nullptr;
    // Rem's splice moves a node out of its ancestors' paths, so the writes
    // that compress next to it stay CASes.
    c.atomic_compress = (o.splice == GCONN_SPLICE_ATOMIC && o.link == GCONN_LINK_REM_CAS)
                            ? 1u : (uint32_t)o.atomic_compress;
    return c;
  }

  gconn_status read_ctrl(Ctrl* host) {
    GCONN_HIP(hipMemcpyAsync(host, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    GCONN_HIP(hipStreamSynchronize(s));
    return GCONN_OK;
  }

  // Union-Rem-CAS first-k sampling as a step machine (uint32 offsets only).
  bool kout_step_machine() const {
    return o.link == GCONN_LINK_REM_CAS && o.splice != GCONN_SPLICE_ATOMIC && !o.kout_random &&
           !g.offsets_64 && o.schedule == 2;
  }

  // Id range of the local-first k-out: the largest power of two up to
  // kLocalRangeMax whose parents fit the device's LDS per workgroup (the
  // kernel's dynamic LDS limit is raised to match once per process).
  template <typename OffT>
  static gconn_status local_range(uint32_t* out) {
    static std::mutex mu;
    static uint32_t cached = 0;
    std::lock_guard<std::mutex> lock(mu);
    if (!cached) {
      int dev = 0, lds = 65536;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
              hipSuccess) {
        (void)hipGetLastError();
        lds = 65536;
      }
      uint32_t r = kLocalRangeMax;
      while (r > kLocalRangeMin && 4ull * r > (uint64_t)lds) r >>= 1;
      if (4ull * r > 65536) {
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void*>(&k_kout_local<OffT>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)(4 * r));
        if (e != hipSuccess) {
          (void)hipGetLastError();
          r = 16384;  // 64 KB: always allowed
        }
      }
      cached = r;
    }
    *out = cached;
    return GCONN_OK;
  }

  // The pair-union kernel's dynamic LDS limit, raised once per rule
  // instantiation (needed whenever the set is sized above 64 KB).
  template <class R>
  static gconn_status pairs_lds_ok() {
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [] {
      err = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_kout_pairs<R>),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(8 * kPairSlots));
      if (err != hipSuccess) (void)hipGetLastError();
    });
    if (err != hipSuccess) return hip_fail(err, "hipFuncSetAttribute(k_kout_pairs)");
    return GCONN_OK;
  }

  // The slot-array k-out passes: local-first (LDS pass, then pair unions over
  // the leaving edges) or, with local == false,
  // the plain two-pass schedule.  gate (nullable): the automatic schedule's
  // control block; the local passes then run only if its probe chose them.
  template <typename OffT>
  gconn_status local_passes(bool local, KoutGate gate) {
    const OffT* off = static_cast<const OffT*>(g.offsets);
    const uint32_t n = g.n;
    Ctrl* st = want_stats ? ctrl : nullptr;
    uint2* res = reinterpret_cast<uint2*>(ws + L.resid);
    uint32_t* rsrc = reinterpret_cast<uint32_t*>(ws + L.lrec_src);
    uint32_t* rdst = reinterpret_cast<uint32_t*>(ws + L.lrec_dst);
    uint32_t* rcnt = reinterpret_cast<uint32_t*>(ws + L.lrec_hdr);
    uint32_t range = kLocalRangeMin;
    if (local) GCONN_TRY(local_range<OffT>(&range));
    uint32_t shift = 0;
    while ((1u << shift) < range) ++shift;
    const uint32_t ranges = (uint32_t)((n + range - 1) / range);
    k_kout_local<OffT><<<ranges, 1024, 4 * range, s>>>(off, g.nbrs, n, o.k, shift, P, res, rsrc,
                                                       rdst, rcnt, fu, fv, local ? 1 : 0, st,
                                                       gate);
    GCONN_LAUNCHED("k_kout_local");
    GCONN_TRY(with_rule(o.link, o.find, o.splice, [&](auto rule) -> gconn_status {
      using R = decltype(rule);
      if (!local) {
        k_kout_residual<R><<<contention_grid(gridN(n), n), block, 0, s>>>(res, n, link_ctx());
        GCONN_LAUNCHED("k_kout_residual");
        return GCONN_OK;
      }
      GCONN_TRY(pairs_lds_ok<R>());
      k_kout_pairs<R><<<ranges, 1024, 8 * kPairSlots, s>>>(rsrc, rdst, rcnt, shift, link_ctx(),
                                                          gate);
      GCONN_LAUNCHED("k_kout_pairs");
      return GCONN_OK;
    }));
    return GCONN_OK;
  }

  template <typename OffT>
  gconn_status sample_phase() {
    const OffT* off = static_cast<const OffT*>(g.offsets);
    const uint32_t n = g.n;
    Ctrl* st = want_stats ? ctrl : nullptr;
    GCONN_TRY(prof_mark(kPhaseSample, true, s));
    if (o.sample == GCONN_SAMPLE_KOUT) {
      if (kout_local_applies(o)) {
        GCONN_TRY(local_passes<OffT>(o.kout_local != 0, KoutGate{}));
      } else if (kout_xcd_applies(o)) {
        uint32_t* rsrc = reinterpret_cast<uint32_t*>(ws + L.kx_src);
        uint32_t* rdst = reinterpret_cast<uint32_t*>(ws + L.kx_dst);
        uint32_t* rroot = reinterpret_cast<uint32_t*>(ws + L.kx_root);
        uint32_t* hdr = reinterpret_cast<uint32_t*>(ws + L.kx_hdr);
        const uint32_t chunks = (uint32_t)((n + kKxChunk - 1) / kKxChunk);
        const int vec = (((reinterpret_cast<uintptr_t>(P) | reinterpret_cast<uintptr_t>(fu) |
                           reinterpret_cast<uintptr_t>(fv)) % 16) == 0 ? 1 : 0) |
                        ((sizeof(OffT) == 4 && reinterpret_cast<uintptr_t>(off) % 16 == 0) ? 2 : 0);
        k_kx_stream<OffT><<<chunks, 256, 0, s>>>(off, g.nbrs, n, o.k, kx_shift(n), P, fu, fv,
                                                 rsrc, rdst, hdr, vec, st);
        GCONN_LAUNCHED("k_kx_stream");
        k_kx_flatten<<<chunks, 256, 0, s>>>(P, n, rsrc, hdr, rroot);
        GCONN_LAUNCHED("k_kx_flatten");
        GCONN_TRY(with_rule(o.link, o.find, o.splice, [&](auto rule) -> gconn_status {
          using R = decltype(rule);
          const uint32_t grid = persistent_grid(k_kx_unite<R>, 256);
          k_kx_unite<R><<<grid, 256, 0, s>>>(rsrc, rdst, rroot, hdr, chunks, o.kout_prelink, ctrl,
                                              link_ctx());
          GCONN_LAUNCHED("k_kx_unite");
          return GCONN_OK;
        }));
      } else if (kout_flat_applies(o)) {
        uint2* res = reinterpret_cast<uint2*>(ws + L.resid);
        const uint32_t pgrid = std::min<uint32_t>(gridN(n), 8192);
        k_kout_prelink<OffT><<<pgrid, block, 0, s>>>(off, g.nbrs, n, o.k, P, res, fu, fv, st);
        GCONN_LAUNCHED("k_kout_prelink");
        k_flatten<<<std::min<uint32_t>(gridN(n), 8192), block, 0, s>>>(P, n);
        GCONN_LAUNCHED("k_flatten");
        GCONN_TRY(with_rule(o.link, o.find, o.splice, [&](auto rule) -> gconn_status {
          using R = decltype(rule);
          k_kout_residual_flat<R><<<contention_grid(gridN(n), n), block, 0, s>>>(res, n,
                                                                                  link_ctx());
          GCONN_LAUNCHED("k_kout_residual_flat");
          return GCONN_OK;
        }));
      } else if (kout_prelink_applies(o)) {
        uint2* res = reinterpret_cast<uint2*>(ws + L.resid);
        const uint32_t pgrid = std::min<uint32_t>(gridN(n), 8192);
        k_kout_prelink<OffT><<<pgrid, block, 0, s>>>(off, g.nbrs, n, o.k, P, res, fu, fv, st);
        GCONN_LAUNCHED("k_kout_prelink");
        GCONN_TRY(with_rule(o.link, o.find, o.splice, [&](auto rule) -> gconn_status {
          using R = decltype(rule);
          k_kout_residual<R><<<contention_grid(gridN(n), n), block, 0, s>>>(res, n, link_ctx());
          GCONN_LAUNCHED("k_kout_residual");
          return GCONN_OK;
        }));
      } else if (kout_step_machine()) {
        GCONN_TRY(with_rule(o.link, o.find, o.splice, [&](auto rule) -> gconn_status {
          using R = decltype(rule);
          auto kern = k_sample_kout_rem_sm<R::kFind, R::kSplice>;
          const uint32_t grid = persistent_grid(kern, 256);
          kern<<<grid, 256, 0, s>>>(static_cast<const uint32_t*>(g.offsets), g.nbrs, n, o.k,
                                    link_ctx(), st);
          GCONN_LAUNCHED("k_sample_kout_rem_sm");
          return GCONN_OK;
        }));
      } else if (o.schedule == 3 && o.link == GCONN_LINK_REM_CAS &&
                 o.splice != GCONN_SPLICE_ATOMIC && !o.kout_random && o.k <= 2) {
        GCONN_TRY(with_rule(o.link, o.find, o.splice, [&](auto rule) -> gconn_status {
          using R = decltype(rule);
          const uint32_t grid =
              contention_grid(persistent_grid(k_sample_kout_pipe<R, OffT>, block), n);
          k_sample_kout_pipe<R, OffT><<<grid, block, 0, s>>>(off, g.nbrs, n, o.k, link_ctx(), st);
          GCONN_LAUNCHED("k_sample_kout_pipe");
          return GCONN_OK;
        }));
      } else if (o.schedule == 1) {
        GCONN_TRY(with_rule(o.link, o.find, o.splice, [&](auto rule) -> gconn_status {
          using R = decltype(rule);
          k_sample_kout<R, OffT><<<gridN(n), block, 0, s>>>(off, g.nbrs, n, o.k, o.kout_random,
                                                            o.seed ^ 0x6b6f7574ull, link_ctx(), st);
          GCONN_LAUNCHED("k_sample_kout");
          return GCONN_OK;
        }));
      } else {
        // Automatic schedule: the locality probe picks the local-first passes
        // or the one-pass kernel on the device; the other side returns at once.
        KoutGate gate{};
        if (probe_part) {  // k_init probed the graph
          uint32_t range = kLocalRangeMin, shift = 0;
          GCONN_TRY(local_range<OffT>(&range));
          while ((1u << shift) < range) ++shift;
          gate = KoutGate{probe_part, n, shift};
          GCONN_TRY(local_passes<OffT>(true, gate));
        }
        GCONN_TRY(with_rule(o.link, o.find, o.splice, [&](auto rule) -> gconn_status {
          using R = decltype(rule);
          const uint32_t grid = contention_grid(persistent_grid(k_sample_kout_pf<R, OffT>, block), n);
          k_sample_kout_pf<R, OffT><<<grid, block, 0, s>>>(off, g.nbrs, n, o.k, o.kout_random,
                                                           o.seed ^ 0x6b6f7574ull, link_ctx(), st,
                                                           gate);
          GCONN_LAUNCHED("k_sample_kout_pf");
          return GCONN_OK;
        }));
      }
    } else if (o.sample == GCONN_SAMPLE_HB) {
      k_hb_step1<OffT><<<gridN(n), block, 0, s>>>(off, g.nbrs, P, n, fu, fv, st);
      GCONN_LAUNCHED("k_hb_step1");
      GCONN_TRY(with_rule(o.link, o.find, o.splice, [&](auto rule) -> gconn_status {
        using R = decltype(rule);
        k_hb_step2<R, OffT><<<gridN(n), block, 0, s>>>(off, g.nbrs, n, o.hb_n, link_ctx(), st);
        GCONN_LAUNCHED("k_hb_step2");
        return GCONN_OK;
      }));
    } else if (o.sample == GCONN_SAMPLE_BFS) {
      GCONN_TRY(bfs_phase<OffT>());
    }
    GCONN_TRY(prof_mark(kPhaseSample, false, s));
    GCONN_TRY(prof_mark(kPhaseLmax, true, s));
    k_lmax<<<1, 1024, 0, s>>>(P, n, o.lmax_samples, o.seed, ctrl);
    GCONN_LAUNCHED("k_lmax");
    GCONN_TRY(prof_mark(kPhaseLmax, false, s));
    return GCONN_OK;
  }

  template <typename OffT>
  gconn_status bfs_phase() {
    const OffT* off = static_cast<const OffT*>(g.offsets);
    const uint32_t n = g.n;
    const uint32_t words = (n + 31) / 32;
    uint32_t* visited = reinterpret_cast<uint32_t*>(ws + L.visited);
    uint32_t* bits[2] = {reinterpret_cast<uint32_t*>(ws + L.fr_bits0),
                         reinterpret_cast<uint32_t*>(ws + L.fr_bits1)};
    uint32_t* queue[2] = {reinterpret_cast<uint32_t*>(ws + L.queue0),
                          reinterpret_cast<uint32_t*>(ws + L.queue1)};
    k_fill<<<gridN(words), block, 0, s>>>(visited, 0u, words);
    GCONN_LAUNCHED("k_fill(visited)");
    unsigned long long* key_slots = reinterpret_cast<unsigned long long*>(ws + L.bfs_slots);
    const uint32_t argmax_grid = std::min<uint32_t>(gridN((n + 3) / 4), kBfsSlots);
    k_bfs_argmax<OffT><<<argmax_grid, block, 0, s>>>(off, n, key_slots);
    GCONN_LAUNCHED("k_bfs_argmax");
    BfsStripe* stripes = reinterpret_cast<BfsStripe*>(ws + L.bfs_stripes);
    k_bfs_start<OffT><<<1, kFoldThreads, 0, s>>>(off, ctrl, visited, queue[0], stripes,
                                                 key_slots, argmax_grid);
    GCONN_LAUNCHED("k_bfs_start");
    // Levels run kRoundsPerSync at a time between host checks: each level's
    // direction and representation changes are decided on the device
    // (k_bfs_decide), every kernel of the level has a fixed grid and returns
    // at once when the level is not its kind, and once the frontier is empty
    // all of them do.
    const uint32_t td_grid = persistent_grid(k_bfs_td<OffT>, 256);
    const uint32_t fixed = std::min<uint32_t>(gridN(n), kPersistentBlocks);
    const uint32_t wgrid = std::min<uint32_t>(gridN(words), kPersistentBlocks);
    const uint32_t bu_grid = (uint32_t)std::min<uint64_t>(
        ((uint64_t)n / 4 + kBuBlock) / kBuBlock, kPersistentBlocks);
    // A batch whose frontier starts as a top-down queue far below the point
    // where the rule would turn bottom-up (edges x 14 x 64 under the
    // unexplored edges) enqueues only the top-down kernels: a high-diameter
    // graph runs thousands of small top-down levels, where the bottom-up
    // kernels' launches, each returning at once, would be most of the time.
    // Such a batch also sizes the top-down grids to the frontier it starts
    // from (both kernels loop over their work, so any grid is correct): a
    // full grid spends more on starting its workgroups, and on each of them
    // reading the work-list counters, than on a few thousand vertices.
    bool td_only = false;
    uint32_t small_grid = fixed, small_td_grid = td_grid;
    for (uint64_t level = 0;; level += kRoundsPerSync) {
      for (int j = 0; j < kRoundsPerSync; ++j) {
        const uint32_t cur = (uint32_t)((level + j) & 1), nxt = cur ^ 1;
        k_bfs_decide<<<1, 128, 0, s>>>(ctrl, stripes, cur, g.m, n, td_only ? 1 : 0);
        GCONN_LAUNCHED("k_bfs_decide");
        if (!td_only) {
          // bottom-up: the frontier as bits (from the queue if it was one)
          k_bfs_clear_bits<<<wgrid, block, 0, s>>>(bits[cur], words, ctrl, 1);
          GCONN_LAUNCHED("k_bfs_clear_bits");
          k_queue_to_bits<<<fixed, block, 0, s>>>(queue[cur], ctrl, cur, bits[cur]);
          GCONN_LAUNCHED("k_queue_to_bits");
          k_bfs_clear_bits<<<wgrid, block, 0, s>>>(bits[nxt], words, ctrl, 0);
          GCONN_LAUNCHED("k_bfs_clear_bits");
          k_bfs_bu<OffT><<<bu_grid, kBuBlock, 0, s>>>(off, g.nbrs, n, visited, bits[cur],
                                                      bits[nxt], ctrl, stripes, nxt, fu, fv);
          GCONN_LAUNCHED("k_bfs_bu");
          // top-down: the frontier as a queue (from the bits if it was those)
          k_bits_to_queue<<<wgrid, block, 0, s>>>(bits[cur], words, ctrl, queue[cur]);
          GCONN_LAUNCHED("k_bits_to_queue");
        }
        k_bfs_td_split<OffT><<<td_only ? small_grid : fixed, block, 0, s>>>(off, queue[cur], ctrl,
                                                                          cur, wl);
        GCONN_LAUNCHED("k_bfs_td_split");
        k_bfs_td<OffT><<<td_only ? small_td_grid : td_grid, 256, 0, s>>>(
            off, g.nbrs, wl, ctrl, stripes, nxt, visited, queue[nxt], fu, fv);
        GCONN_LAUNCHED("k_bfs_td");
      }
      const uint32_t next = (uint32_t)((level + kRoundsPerSync) & 1);
      k_bfs_fold<<<1, 64, 0, s>>>(ctrl, stripes, next);
      GCONN_LAUNCHED("k_bfs_fold");
      Ctrl h;
      GCONN_HIP(hipMemcpyAsync(&h, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
      GCONN_HIP(hipStreamSynchronize(s));
      const uint32_t mode = h.bfs_mode;
      if (mode == 0) {
        // the copy followed every kernel of the last batch, so the level
        // count in it is final
        rounds = h.bfs_levels;
        break;
      }
      const uint64_t unexplored = g.m > h.explored_edges ? g.m - h.explored_edges : 0;
      td_only = mode == 1 && h.bfs_as_queue != 0 &&
                (unsigned __int128)h.frontier_edges[next] * 14 * 64 <= unexplored;
      if (td_only) {
        // a lane per frontier vertex and four row entries per lane, with
        // room for the frontier to grow 8x over the batch
        const uint64_t cnt = h.frontier_count[next], edges = h.frontier_edges[next];
        const uint64_t lanes = std::max<uint64_t>(cnt, edges / 4) * 8;
        small_grid = (uint32_t)std::min<uint64_t>(fixed, std::max<uint64_t>(8, lanes / block + 1));
        small_td_grid = (uint32_t)std::min<uint64_t>(td_grid, std::max<uint64_t>(8, lanes / 256 + 1));
      }
      if (level + kRoundsPerSync > (uint64_t)n + kRoundsPerSync)
        return fail(GCONN_EDEVICE, "BFS did not finish within n levels");
    }
    // the argmax slots are free again: the minimum's slots reuse them
    uint32_t* min_slots = reinterpret_cast<uint32_t*>(ws + L.bfs_slots);
    const uint32_t min_grid = std::min<uint32_t>(gridN(words), kBfsSlots);
    k_bfs_min<<<min_grid, block, 0, s>>>(visited, words, min_slots);
    GCONN_LAUNCHED("k_bfs_min");
    k_bfs_min_fold<<<1, kFoldThreads, 0, s>>>(min_slots, min_grid, ctrl);
    GCONN_LAUNCHED("k_bfs_min_fold");
    k_bfs_label<<<gridN((n + 3) / 4), block, 0, s>>>(visited, n, ctrl, P);
    GCONN_LAUNCHED("k_bfs_label");
    // the work lists were used as scratch: clear their counters
    k_bfs_level_reset<<<1, 128, 0, s>>>(ctrl, 0);
    GCONN_LAUNCHED("k_bfs_level_reset");
    return GCONN_OK;
  }

  template <typename OffT>
  gconn_status gather() {
    const OffT* off = static_cast<const OffT*>(g.offsets);
    const int mode = o.sample == GCONN_SAMPLE_NONE ? 0 : (o.sample == GCONN_SAMPLE_BFS ? 1 : 2);
    k_compress_gather<OffT><<<gridN((g.n + 3) / 4), block, 0, s>>>(off, P, g.n, ctrl, wl, mode,
                                                         skip_lmax() ? 1 : 0, want_stats ? 1 : 0);
    GCONN_LAUNCHED("k_compress_gather");
    return GCONN_OK;
  }

  template <typename OffT>
  gconn_status finish_union_find() {
    const OffT* off = static_cast<const OffT*>(g.offsets);
    return with_rule(o.link, o.find, o.splice, [&](auto rule) -> gconn_status {
      using R = decltype(rule);
      const uint32_t grid = persistent_grid(k_finish<R, OffT>, block);
      k_finish<R, OffT><<<grid, block, 0, s>>>(off, g.nbrs, wl, ctrl, link_ctx());
      GCONN_LAUNCHED("k_finish");
      return GCONN_OK;
    });
  }

  template <typename OffT>
  gconn_status materialize(uint32_t* esrc, uint32_t* edst) {
    const OffT* off = static_cast<const OffT*>(g.offsets);
    const uint32_t grid = persistent_grid(k_materialize<OffT>, block);
    k_materialize<OffT><<<grid, block, 0, s>>>(off, g.nbrs, wl, ctrl, esrc, edst);
    GCONN_LAUNCHED("k_materialize");
    return GCONN_OK;
  }

  // SV / LT / LP: K early-exit rounds per host check.
  gconn_status iterate(uint32_t* esrc, uint32_t* edst) {
    const uint32_t n = g.n;
    uint32_t* prev = reinterpret_cast<uint32_t*>(ws + L.prev);
    const bool sv = o.link == GCONN_LINK_SV, lt = o.link == GCONN_LINK_LT;
    const int v = o.lt_variant;
    // variant decoding, paper order: CUSA CRSA PUSA PRSA PUS PRS EUSA EUS, then F-forms
    static const int kConnect[16] = {0, 0, 1, 1, 1, 1, 2, 2, 0, 0, 1, 1, 1, 1, 2, 2};
    static const int kRoot[16] = {0, 1, 0, 1, 0, 1, 0, 0, 0, 1, 0, 1, 0, 1, 0, 0};
    static const int kAlter[16] = {1, 1, 1, 1, 0, 0, 1, 0, 1, 1, 1, 1, 0, 0, 1, 0};
    const bool full = v >= 8;
    const bool need_prev = sv || (lt && kRoot[v]);
    if (need_prev) {
      k_copy<<<gridN(n), block, 0, s>>>(prev, P, n);
      GCONN_LAUNCHED("k_copy(prev)");
    }
    const bool sv_snapshot = sv && fu != nullptr;
    for (uint64_t r = 0;; r += kRoundsPerSync) {
      for (int j = 0; j < kRoundsPerSync; ++j) {
        const uint32_t rr = (uint32_t)(r + j);
        const uint32_t slot = rr % kRoundSlots;
        k_round_begin<<<1, 64, 0, s>>>(ctrl, rr);
        GCONN_LAUNCHED("k_round_begin");
        if (sv) {
          k_sv_round<<<kPersistentBlocks, block, 0, s>>>(esrc, edst, ctrl, P, prev, slot,
                                                         sv_snapshot ? 1 : 0);
          GCONN_LAUNCHED("k_sv_round");
          if (fu) {
            k_sv_record<<<kPersistentBlocks, block, 0, s>>>(esrc, edst, ctrl, P, prev, fu, fv);
            GCONN_LAUNCHED("k_sv_record");
          }
          k_shortcut_full<<<gridN(n), block, 0, s>>>(ctrl, P, prev, n, slot, 0);
          GCONN_LAUNCHED("k_shortcut_full");
        } else if (lt) {
          k_lt_round<<<kPersistentBlocks, block, 0, s>>>(esrc, edst, ctrl, P, prev, slot,
                                                         kConnect[v], kRoot[v]);
          GCONN_LAUNCHED("k_lt_round");
          if (full) {
            k_shortcut_full<<<gridN(n), block, 0, s>>>(ctrl, P, kRoot[v] ? prev : nullptr, n,
                                                       slot, 1);
            GCONN_LAUNCHED("k_shortcut_full");
          } else {
            k_shortcut_one<<<gridN(n), block, 0, s>>>(ctrl, P, kRoot[v] ? prev : nullptr, n, slot);
            GCONN_LAUNCHED("k_shortcut_one");
          }
          if (kAlter[v]) {
            k_lt_alter<<<kPersistentBlocks, block, 0, s>>>(esrc, edst, ctrl, P, slot);
            GCONN_LAUNCHED("k_lt_alter");
          }
        } else {
          k_lp_round<<<kPersistentBlocks, block, 0, s>>>(esrc, edst, ctrl, P, slot);
          GCONN_LAUNCHED("k_lp_round");
        }
      }
      uint32_t done = 0;
      GCONN_HIP(hipMemcpyAsync(&done, &ctrl->done, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      GCONN_HIP(hipStreamSynchronize(s));
      if (done) {
        // count the rounds that ran: find the first slot that reported no change
        Ctrl h;
        GCONN_TRY(read_ctrl(&h));
        // the first round (from the last one of the previous batch on) that
        // reported no change is the converged round; count it
        uint64_t ran = r + kRoundsPerSync;
        for (int64_t j = (r > 0 ? -1 : 0); j < kRoundsPerSync; ++j)
          if (h.changed[(r + j) % kRoundSlots] == 0) {
            ran = r + j + 1;
            break;
          }
        rounds = ran;
        break;
      }
      if (r + kRoundsPerSync >= kMaxRounds)
        return fail(GCONN_ETIMEOUT, "iterative finish did not converge within the round cap");
    }
    return GCONN_OK;
  }
};

}  // namespace

gconn_status reset_ctrl_and_parents(Ctrl* ctrl, uint32_t* P, uint32_t n, hipStream_t s) {
  const bool vec = (reinterpret_cast<uintptr_t>(P) % 16) == 0;
  k_init<<<grid_for(std::max<uint64_t>(vec ? n / 4 : n, 1), 256), 256, 0, s>>>(
      ctrl, P, n, nullptr, nullptr, vec ? 1 : 0, KoutProbe{});
  GCONN_LAUNCHED("k_init");
  return GCONN_OK;
}

gconn_status launch_iota(uint32_t* P, uint32_t n, hipStream_t s) {
  if (n == 0) return GCONN_OK;
  k_iota<<<grid_for(n, 256), 256, 0, s>>>(P, n);
  GCONN_LAUNCHED("k_iota");
  return GCONN_OK;
}

gconn_status launch_fill(uint32_t* p, uint32_t value, uint64_t count, hipStream_t s) {
  if (count == 0) return GCONN_OK;
  k_fill<<<grid_for(count, 256), 256, 0, s>>>(p, value, count);
  GCONN_LAUNCHED("k_fill");
  return GCONN_OK;
}

gconn_status launch_finalize(uint32_t* P, uint32_t n, uint32_t* labels, hipStream_t s) {
  if (n == 0) return GCONN_OK;
  k_compress_to<<<grid_for(n, 256), 256, 0, s>>>(P, labels, n);
  GCONN_LAUNCHED("k_compress_to");
  return GCONN_OK;
}

gconn_status launch_insert(const gconn_options& o, uint32_t* P, uint32_t* H, const uint32_t* src,
                           const uint32_t* dst, uint64_t k, hipStream_t s) {
  if (k == 0) return GCONN_OK;
  LinkCtx c;
  c.P = P;
  c.H = H;
  c.fu = c.fv = nullptr;
  c.hooks = nullptr;
  c.atomic_compress = (o.splice == GCONN_SPLICE_ATOMIC && o.link == GCONN_LINK_REM_CAS)
                          ? 1u : (uint32_t)o.atomic_compress;
  const uint32_t block = (uint32_t)o.block;
  return with_rule(o.link, o.find, o.splice, [&](auto rule) -> gconn_status {
    using R = decltype(rule);
    k_unite_pairs<R><<<grid_for(k, block), block, 0, s>>>(src, dst, k, c);
    GCONN_LAUNCHED("k_unite_pairs");
    return GCONN_OK;
  });
}

gconn_status launch_query(const gconn_options& o, uint32_t* P, const uint32_t* a,
                          const uint32_t* b, uint64_t q, uint8_t* out, hipStream_t s) {
  if (q == 0) return GCONN_OK;
  const uint32_t block = (uint32_t)o.block;
  return with_rule(o.link, o.find, o.splice, [&](auto rule) -> gconn_status {
    using R = decltype(rule);
    k_query<R><<<grid_for(q, block), block, 0, s>>>(a, b, q, P, out, o.atomic_compress);
    GCONN_LAUNCHED("k_query");
    return GCONN_OK;
  });
}

// --------------------------------------------------------------- phase profiler
namespace {
struct Profiler {
  bool on = false;
  uint32_t mask = ~0u;  // bit p: bracket phase p
  struct Mark {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Mark> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t open[kPhaseCount] = {};
  double acc[kPhaseCount] = {};
  uint64_t runs = 0;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return e;
  }
};
thread_local Profiler g_prof;
}  // namespace

bool profiling() { return g_prof.on; }

gconn_status prof_mark(int phase, bool begin, hipStream_t s) {
  if (!g_prof.on || !((g_prof.mask >> phase) & 1u)) return GCONN_OK;
  hipEvent_t e = g_prof.get();
  if (!e) return fail(GCONN_EDEVICE, "hipEventCreate failed");
  GCONN_HIP(hipEventRecord(e, s));
  if (begin) {
    g_prof.open[phase] = e;
  } else {
    g_prof.pending.push_back({phase, g_prof.open[phase], e});
    g_prof.open[phase] = nullptr;
  }
  return GCONN_OK;
}

void prof_count_run() {
  if (g_prof.on) ++g_prof.runs;
}

gconn_status profile_enable(int on) {
  if (on < 0) return fail(GCONN_EINVAL, "profile mask must be >= 0");
  g_prof.on = on != 0;
  g_prof.mask = on == 1 ? ~0u : ((uint32_t)on >> 1);
  return GCONN_OK;
}

gconn_status profile_read(gconn_phase_times* out, int reset) {
  for (auto& m : g_prof.pending) {
    GCONN_HIP(hipEventSynchronize(m.b));
    float ms = 0.f;
    if (m.a) {
      GCONN_HIP(hipEventElapsedTime(&ms, m.a, m.b));
      g_prof.pool.push_back(m.a);
    }
    g_prof.acc[m.phase] += ms;
    g_prof.pool.push_back(m.b);
  }
  g_prof.pending.clear();
  if (out) {
    out->init_ms = g_prof.acc[kPhaseInit];
    out->sample_ms = g_prof.acc[kPhaseSample];
    out->compress_ms = g_prof.acc[kPhaseCompress];
    out->lmax_ms = g_prof.acc[kPhaseLmax];
    out->gather_ms = g_prof.acc[kPhaseGather];
    out->finish_ms = g_prof.acc[kPhaseFinish];
    out->finalize_ms = g_prof.acc[kPhaseFinalize];
    out->runs = g_prof.runs;
  }
  if (reset) {
    for (double& a : g_prof.acc) a = 0;
    g_prof.runs = 0;
  }
  return GCONN_OK;
}

gconn_status launch_mixed(const gconn_options& o, uint32_t* P, uint32_t* H, const uint8_t* kind,
                          const uint32_t* a, const uint32_t* b, uint64_t count, uint8_t* out,
                          hipStream_t s) {
  if (count == 0) return GCONN_OK;
  LinkCtx c;
  c.P = P;
  c.H = H;
  c.fu = c.fv = nullptr;
  c.hooks = nullptr;
  c.atomic_compress = (o.splice == GCONN_SPLICE_ATOMIC && o.link == GCONN_LINK_REM_CAS)
                          ? 1u : (uint32_t)o.atomic_compress;
  const uint32_t block = (uint32_t)o.block;
  return with_rule(o.link, o.find, o.splice, [&](auto rule) -> gconn_status {
    using R = decltype(rule);
    k_unite_kind<R><<<grid_for(count, block), block, 0, s>>>(kind, a, b, count, c);
    GCONN_LAUNCHED("k_unite_kind");
    k_query_kind<R><<<grid_for(count, block), block, 0, s>>>(kind, a, b, count, P, out,
                                                            (int)c.atomic_compress);
    GCONN_LAUNCHED("k_query_kind");
    return GCONN_OK;
  });
}

gconn_status validate_kinds(const uint8_t* kind, uint64_t count, Ctrl* ctrl, hipStream_t s) {
  if (count == 0) return GCONN_OK;
  k_ctrl_init<<<1, 256, 0, s>>>(ctrl);
  GCONN_LAUNCHED("k_ctrl_init");
  k_validate_kinds<<<grid_for(count, 256), 256, 0, s>>>(kind, count, ctrl);
  GCONN_LAUNCHED("k_validate_kinds");
  uint32_t err = 0;
  GCONN_HIP(hipMemcpyAsync(&err, &ctrl->err, sizeof(err), hipMemcpyDeviceToHost, s));
  GCONN_HIP(hipStreamSynchronize(s));
  if (err) return fail(GCONN_EINVAL, "mixed batch: a kind other than insert (0) or query (1)");
  return GCONN_OK;
}

gconn_status validate_pairs(const uint32_t* a, const uint32_t* b, uint64_t k, uint32_t n,
                            Ctrl* ctrl, hipStream_t s) {
  if (k == 0) return GCONN_OK;
  k_ctrl_init<<<1, 256, 0, s>>>(ctrl);
  GCONN_LAUNCHED("k_ctrl_init");
  k_validate_ids<<<grid_for(k, 256), 256, 0, s>>>(a, b, k, n, ctrl);
  GCONN_LAUNCHED("k_validate_ids");
  uint32_t err = 0;
  GCONN_HIP(hipMemcpyAsync(&err, &ctrl->err, sizeof(err), hipMemcpyDeviceToHost, s));
  GCONN_HIP(hipStreamSynchronize(s));
  if (err) return fail(GCONN_EINVAL, "vertex id out of range in batch");
  return GCONN_OK;
}

WsLayout plan_workspace(const gconn_graph& g, const gconn_options& o, bool forest, bool labels) {
  if (o.link == GCONN_LINK_JTB) return plan_workspace_jtb(g, o, forest, labels);
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
  const bool csr = g.format == GCONN_CSR;
  if (csr) {
    // push calls cover at most 64 items with group ids below ceil(n/256)*4
    // <= ceil(n/64) + 3, so a sub-list gets at most ceil(ceil(n/64)/64) + 1 calls
    const uint64_t groups = (n + 63) / 64;
    L.sub_cap = (uint32_t)(((groups + kSubLists - 1) / kSubLists + 1) * 64);
    L.small = take(4ull * kSubLists * L.sub_cap);
    L.medium = take(4ull * kSubLists * L.sub_cap);
    // a vertex of degree d > kMedDeg (= kSeg) yields ceil(d / kSeg) <= 2d / kSeg segments
    L.seg_cap = 2 * m / kSeg + 1;
    L.segs = take(8 * L.seg_cap);
  }
  if (needs_claims(o.link)) L.hooks = take(4 * n);
  if (csr && (kout_prelink_applies(o) || (kout_local_applies(o) && !o.kout_local)))
    L.resid = take(8 * n);
  if (csr && kout_auto_local_applies(o)) L.probe = take(8 * kProbeBlocks);
  if (csr && ((kout_local_applies(o) && o.kout_local) || kout_auto_local_applies(o))) {
    // records: at most two per vertex, in per-range blocks of 2 * range
    const uint64_t cap = 2 * (n + kLocalRangeMax);
    L.lrec_src = take(4 * cap);
    L.lrec_dst = take(4 * cap);
    L.lrec_hdr = take(4ull * (n / kLocalRangeMin + 1));  // record counts
  }
  if (csr && kout_xcd_applies(o)) {
    const uint64_t chunks = (n + kKxChunk - 1) / kKxChunk;
    L.kx_src = take(4 * chunks * kKxCap);
    L.kx_dst = take(4 * chunks * kKxCap);
    L.kx_root = take(4 * chunks * kKxCap);
    L.kx_hdr = take(4 * chunks * kKxGroups);
  }
  const bool iterative =
      o.link == GCONN_LINK_SV || o.link == GCONN_LINK_LT || o.link == GCONN_LINK_LP;
  if (iterative) {
    L.prev = take(4 * n);
    L.edge_cap = m;
    L.esrc = take(4 * m);
    L.edst = take(4 * m);
  }
  if (csr && o.sample == GCONN_SAMPLE_BFS) {
    const uint64_t words = (n + 31) / 32;
    L.visited = take(4 * words);
    L.fr_bits0 = take(4 * words);
    L.fr_bits1 = take(4 * words);
    L.queue0 = take(4 * n);
    L.queue1 = take(4 * n);
    L.bfs_stripes = take(2 * kBfsStripes * sizeof(BfsStripe));
    L.bfs_slots = take(kBfsSlots * sizeof(unsigned long long));
  }
  L.total = at;
  return L;
}

gconn_status validate_graph(const gconn_graph& g, Ctrl* ctrl, uint32_t block, hipStream_t s) {
  const uint32_t n = g.n;
  if (g.format == GCONN_CSR) {
    if (g.offsets_64)
      k_validate_csr<uint64_t><<<grid_for(std::max<uint64_t>(g.m, n), block), block, 0, s>>>(
          static_cast<const uint64_t*>(g.offsets), g.nbrs, n, g.m, ctrl);
    else
      k_validate_csr<uint32_t><<<grid_for(std::max<uint64_t>(g.m, n), block), block, 0, s>>>(
          static_cast<const uint32_t*>(g.offsets), g.nbrs, n, g.m, ctrl);
  } else {
    k_validate_ids<<<grid_for(g.m, block), block, 0, s>>>(g.nbrs, g.dst, g.m, n, ctrl);
  }
  GCONN_LAUNCHED("k_validate");
  uint32_t err = 0;
  GCONN_HIP(hipMemcpyAsync(&err, &ctrl->err, sizeof(err), hipMemcpyDeviceToHost, s));
  GCONN_HIP(hipStreamSynchronize(s));
  if (err) return fail(GCONN_EINVAL, "graph validation failed (offsets or vertex id out of range)");
  return GCONN_OK;
}

gconn_status run_static(const gconn_graph& g, uint32_t* P, uint32_t* fu, uint32_t* fv,
                        bool finalize, uint8_t* ws, const WsLayout& L, const gconn_options& o,
                        gconn_stats* stats, hipStream_t s) {
  if (o.link == GCONN_LINK_JTB)
    return run_static_jtb(g, P, fu, fv, finalize, ws, L, o, stats, s, nullptr);
  Run run(g, P, fu, fv, ws, L, o, stats != nullptr, s);
  const uint32_t n = g.n;
  const uint32_t block = run.block;
  prof_count_run();
  GCONN_TRY(prof_mark(kPhaseInit, true, s));
  const bool vec = (reinterpret_cast<uintptr_t>(P) % 16) == 0 &&
                   (!fu || ((reinterpret_cast<uintptr_t>(fu) | reinterpret_cast<uintptr_t>(fv)) % 16) == 0);
  // The XCD-bucketed k-out writes every parent and forest slot itself.
  const bool kx_writes_all = g.format == GCONN_CSR && n > 0 && g.m > 0 && kout_xcd_applies(o);
  if (kx_writes_all) {
    k_ctrl_init<<<1, 256, 0, s>>>(run.ctrl);
    GCONN_LAUNCHED("k_ctrl_init");
  } else {
    // the automatic k-out schedule's locality probe rides in blocks 1-16
    KoutProbe probe{};
    const uint32_t init_grid = grid_for(std::max<uint64_t>(vec ? n / 4 : n, 1), block);
    if (g.format == GCONN_CSR && n > 0 && g.m > 0 && kout_auto_local_applies(o) &&
        init_grid > kProbeBlocks) {
      uint32_t range = kLocalRangeMin;
      GCONN_TRY(g.offsets_64 ? Run::local_range<uint64_t>(&range)
                             : Run::local_range<uint32_t>(&range));
      uint32_t shift = 0;
      while ((1u << shift) < range) ++shift;
      probe.off32 = g.offsets_64 ? nullptr : static_cast<const uint32_t*>(g.offsets);
      probe.off64 = g.offsets_64 ? static_cast<const uint64_t*>(g.offsets) : nullptr;
      probe.nbrs = g.nbrs;
      probe.part = reinterpret_cast<uint32_t*>(ws + L.probe);
      probe.k = o.k;
      probe.shift = shift;
      probe.seed = o.seed ^ 0x70726f6265ull;
      run.probe_part = probe.part;
    }
    k_init<<<init_grid, block, 0, s>>>(run.ctrl, P, n, fu, fv, vec ? 1 : 0, probe);
    GCONN_LAUNCHED("k_init");
  }
  if (run.hooks) GCONN_TRY(launch_fill(run.hooks, kEmpty, n, s));
  GCONN_TRY(prof_mark(kPhaseInit, false, s));

  const bool csr = g.format == GCONN_CSR;
  const bool o64 = g.offsets_64 != 0;
  if (o.validate && (g.m > 0 || csr)) GCONN_TRY(validate_graph(g, run.ctrl, block, s));

  const bool iterative =
      o.link == GCONN_LINK_SV || o.link == GCONN_LINK_LT || o.link == GCONN_LINK_LP;
  const bool sampled = csr && o.sample != GCONN_SAMPLE_NONE;
  if (n > 0 && g.m > 0) {
    if (csr) {
      if (sampled) GCONN_TRY(o64 ? run.sample_phase<uint64_t>() : run.sample_phase<uint32_t>());
      GCONN_TRY(prof_mark(kPhaseGather, true, s));
      GCONN_TRY(o64 ? run.gather<uint64_t>() : run.gather<uint32_t>());
      GCONN_TRY(prof_mark(kPhaseGather, false, s));
    }
    GCONN_TRY(prof_mark(kPhaseFinish, true, s));
    if (!iterative) {
      if (csr) {
        GCONN_TRY(o64 ? run.finish_union_find<uint64_t>() : run.finish_union_find<uint32_t>());
      } else {
        GCONN_TRY(with_rule(o.link, o.find, o.splice, [&](auto rule) -> gconn_status {
          using R = decltype(rule);
          k_unite_pairs<R><<<grid_for(g.m, block), block, 0, s>>>(g.nbrs, g.dst, g.m,
                                                                  run.link_ctx());
          GCONN_LAUNCHED("k_unite_pairs");
          return GCONN_OK;
        }));
      }
    } else {
      uint32_t* esrc = reinterpret_cast<uint32_t*>(ws + L.esrc);
      uint32_t* edst = reinterpret_cast<uint32_t*>(ws + L.edst);
      if (csr) {
        GCONN_TRY(o64 ? run.materialize<uint64_t>(esrc, edst)
                      : run.materialize<uint32_t>(esrc, edst));
      } else {
        k_materialize_coo<<<grid_for(g.m, block), block, 0, s>>>(g.nbrs, g.dst, g.m, run.ctrl,
                                                                esrc, edst);
        GCONN_LAUNCHED("k_materialize_coo");
      }
      GCONN_TRY(run.iterate(esrc, edst));
    }
    GCONN_TRY(prof_mark(kPhaseFinish, false, s));
    if (finalize || o.link == GCONN_LINK_ECL || o.link == GCONN_LINK_AFFOREST) {
      // ECL-CC's and Afforest's separate full-compress pass doubles as finalisation.
      GCONN_TRY(prof_mark(kPhaseFinalize, true, s));
      const uint32_t grid = persistent_grid(k_finalize, block);
      k_finalize<<<grid, block, 0, s>>>(P, n, run.ctrl, run.wl, (sampled && csr) ? 1 : 0);
      GCONN_LAUNCHED("k_finalize");
      GCONN_TRY(prof_mark(kPhaseFinalize, false, s));
    }
  }
  if (stats) {
    Ctrl h;
    GCONN_TRY(run.read_ctrl(&h));
    // BFS sampling reads whole rows: the entries of the visited vertices
    stats->sampled_edges =
        (sampled && o.sample == GCONN_SAMPLE_BFS) ? h.explored_edges : h.stat_sampled;
    stats->active_vertices = h.stat_active;
    stats->finish_edges = h.stat_finish_edges;
    stats->hooks = h.stat_hooks;
    stats->rounds = run.rounds;
    stats->lmax = h.lmax;
    stats->bfs_source = h.bfs_source;
  }
  return GCONN_OK;
}

}  // namespace gconn

#if GCONN_COUNT_OPS
// The rules' operation counters of this translation unit (diagnostic builds
// only; see gconn_rules.hpp): out[kind] summed over the slots.
extern "C" gconn_status gconn_diag_op_counts(uint64_t* out, int reset) {
  using namespace gconn;
  static unsigned long long h[1024 * kOpKinds];
  GCONN_HIP(hipDeviceSynchronize());
  GCONN_HIP(hipMemcpyFromSymbol(h, HIP_SYMBOL(g_op_count), sizeof(h)));
  for (int k = 0; k < kOpKinds; ++k) {
    unsigned long long t = 0;
    for (int i = 0; i < 1024; ++i) t += h[i * kOpKinds + k];
    out[k] = t;
  }
  if (reset) {
    std::memset(h, 0, sizeof(h));
    GCONN_HIP(hipMemcpyToSymbol(HIP_SYMBOL(g_op_count), h, sizeof(h)));
  }
  return GCONN_OK;
}
#endif
