// gconn_rules.hpp -- device-side find, splice and union rules on the parent
// array P (gfx950, wave64).
//
// P[x] == x marks a root; every other P[x] points to a smaller id in the same
// tree (Notation and Preliminaries: elements point to themselves or to a parent
// with a smaller ID).  Every write stores a smaller id than the slot's owner
// (and than the value it replaces), so no cycle can form.  All rules but Rem's
// SpliceAtomic are root-based: a link only ever turns a root into a child.
//
// Memory model.  The eight XCDs of an MI355X each have a private L2 that is
// not kept coherent with the others inside a kernel.  Links (a root becoming a
// child) are agent-scope CAS.  Reads of P inside find / union loops are relaxed
// atomic loads whose scope is GCONN_P_LOAD_SCOPE; at wavefront or workgroup
// scope they are ordinary cached loads (L2 hits for the hot entries near the
// roots of large trees) and may return stale values.  Two invariants make
// that safe, and they differ between the rule families:
//   * Root-based rules (every union rule below except Rem's SpliceAtomic):
//     only roots are re-pointed by links, and compression only moves a
//     non-root's pointer to one of its ancestors.  So any value P[x] has ever
//     held is an ancestor of x in the current forest, and a walk may start
//     from any of them, stale or not.
//   * Rem's SpliceAtomic re-hangs a non-root (with its subtree) under the
//     other side's parent, moving it out of its ancestors' tree; an old value
//     of P[x] is then no longer an ancestor of x.  What still holds is weaker:
//     P[x] only ever decreases (every write stores a smaller id), and every
//     value it has held belongs to the set x ends up in once the unions of
//     the phase are done (a splice is part of a union that goes on to join
//     the two sides).  The ancestry argument does not cover this rule, so it
//     reads both parents device-coherently on every iteration, and its
//     trailing compressing finds rely on the CAS instead: a split CAS on P[x]
//     succeeds only if P[x] still holds the value the walk read, so the value
//     written is the current parent's parent, whatever an earlier read saw.
// Progress: every loop iteration below either moves to a strictly smaller
// id, or continues from the value a failed CAS returned (which is fresh), so
// no loop can spin on a stale line.  Coherent reads are needed only where a
// stale value could send a lane back to a CAS that is bound to fail again
// (Union-Hooks' root test, the splice and lock rules).
//
// Compression writes of the root-based rules (the splitting / halving steps of
// the finds and the SplitAtomicOne / HalveAtomicOne steps) only ever touch a
// non-root x and set P[x] to an ancestor of x.
// A non-root never becomes a root again and no link targets it, so such a
// write needs no CAS: whatever order concurrent compression writes land in,
// P[x] ends as some ancestor of x, which is all the forest needs.  With
// LinkCtx::atomic_compress == 0 they are relaxed agent-scope stores, which
// write through to memory like the atomics do; with 1 they are the CASes of
// the atomic rules as written (always so next to SpliceAtomic, whose moves
// break the ancestor argument).  They must not be ordinary cached stores: an
// XCD's L2 writes a dirty line back later, and on MI355X that write-back has
// been measured to undo links that other XCDs made meanwhile on other words
// of the same line (wrong labels at RMAT-24 scale).
//
// Readings of the appendix pseudocode (Appendix A.2, find / splice / union
// algorithms) where it is garbled:
//   * FindSplit / FindHalve re-read v = P[u], w = P[v] on every iteration and
//     return v once v == w (as printed the loop never reloads them).
//   * The union rules CAS the parent of the larger *root* p_u (not of the
//     endpoint u), which is what "only performs links on roots" requires.
//   * SplitAtomicOne / HalveAtomicOne act on r_u: v = P[r_u], w = P[v]; if
//     v != w, CAS P[r_u] from v to w; return v (split) or w (halve).
//   * FindCompress lowers each path entry with an atomic min, which keeps
//     P[x] <= x and is safe against concurrent lowering.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// The rules are host-callable too, so that a CPU harness can run the very same
// code from many threads (the atomic builtins below compile for both sides).
#define GCONN_HD __host__ __device__ __forceinline__

namespace gconn {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;

enum FindRule : int { kFindNaive = 0, kFindSplit = 1, kFindHalve = 2, kFindCompress = 3 };
enum SpliceRule : int { kSpliceSplitOne = 0, kSpliceHalveOne = 1, kSpliceAtomic = 2 };
enum UnionRule : int {
  kUnionAsync = 0, kUnionHooks = 1, kUnionEarly = 2, kUnionRemCas = 3, kUnionAfforest = 4,
  kUnionRemLock = 5
};

// Wavefront scope compiles to an ordinary cached global load (measured fastest
// for the union-find kernels on MI355X; see the memory-model note above).
#ifndef GCONN_P_LOAD_SCOPE
#define GCONN_P_LOAD_SCOPE __HIP_MEMORY_SCOPE_WAVEFRONT
#endif
#ifndef GCONN_ROOT_RECHECK
#define GCONN_ROOT_RECHECK 0
#endif

// Operation counters of a diagnostic build (GCONN_COUNT_OPS=1): every parent
// read, CAS and failed CAS of the rules below adds to one of 1024 slots per
// kind (spread by workgroup so the counting itself does not serialise).
// Timing of such a build is meaningless; the counts are exact.  Off in
// every normal build.
#ifndef GCONN_COUNT_OPS
#define GCONN_COUNT_OPS 0
#endif
#if GCONN_COUNT_OPS
enum OpKind : int { kOpLoad = 0, kOpLoadAgent = 1, kOpCas = 2, kOpCasFail = 3, kOpStore = 4,
                    kOpChase = 5, kOpChaseRounds = 6, kOpKinds = 8 };
// one array per translation unit (no relocatable device code)
static __device__ unsigned long long g_op_count[1024 * kOpKinds];
__device__ __forceinline__ void count_op(int kind) {
  atomicAdd(&g_op_count[(blockIdx.x & 1023u) * kOpKinds + kind], 1ull);
}
#endif
#if GCONN_COUNT_OPS && defined(__HIP_DEVICE_COMPILE__)
#define GCONN_COUNT(kind) count_op(kind)
#else
#define GCONN_COUNT(kind) ((void)0)
#endif

// Read of P inside a find / union loop (see the memory-model note above).  A
// host build may route it through GCONN_HOST_STALE_LOAD(p), a function that
// is free to return any value *p held earlier: the CPU test harness uses it
// to model an XCD's incoherent L2 (device code never defines it).
GCONN_HD uint32_t ld(const uint32_t* p) {
#if defined(GCONN_HOST_STALE_LOAD) && !defined(__HIP_DEVICE_COMPILE__)
  return GCONN_HOST_STALE_LOAD(p);
#else
  GCONN_COUNT(kOpLoad);
  return __hip_atomic_load(p, __ATOMIC_RELAXED, GCONN_P_LOAD_SCOPE);
#endif
}
// Device-coherent read (flags and counters polled across XCDs).
GCONN_HD uint32_t ld_agent(const uint32_t* p) {
  GCONN_COUNT(kOpLoadAgent);
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
GCONN_HD void st(uint32_t* p, uint32_t v) {
  GCONN_COUNT(kOpStore);
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// CAS *p: expected -> desired.  On failure `expected` receives the current value.
GCONN_HD bool cas(uint32_t* p, uint32_t& expected, uint32_t desired) {
  GCONN_COUNT(kOpCas);
  const bool ok = __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!ok) GCONN_COUNT(kOpCasFail);
  return ok;
}
GCONN_HD uint32_t amin(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Compression write at non-root x: P[x] from `expected` to the ancestor
// `desired`.  Returns whether P[x] now holds `desired`; a failed CAS leaves the
// current value in `expected`.
GCONN_HD bool shortcut(uint32_t* p, uint32_t& expected, uint32_t desired, bool atomic) {
  if (atomic) return cas(p, expected, desired);
  st(p, desired);
  return true;
}

// Per-launch state shared by the rules.
struct LinkCtx {
  uint32_t* P;         // parent array
  uint32_t* H;         // hooks array (Union-Hooks only), kEmpty = unclaimed
  uint32_t* fu;        // spanning-forest slots (nullable)
  uint32_t* fv;
  unsigned long long* hooks;  // successful-link counter (nullable)
  uint32_t atomic_compress;   // 1: compression writes are CAS; 0: relaxed stores
};

GCONN_HD void record_link(const LinkCtx& c, uint32_t root, uint32_t u,
                                            uint32_t v) {
  // A root is linked at most once (it never becomes a root again), so the slot
  // write is uncontended.
  if (c.fu) {
    c.fu[root] = u;
    c.fv[root] = v;
  }
  if (c.hooks) __hip_atomic_fetch_add(c.hooks, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ finds
// pu: a value P[u] is known to have held (kEmpty: read it).  Any such value is
// an ancestor of u, so the walk may start from it.
template <int F>
GCONN_HD uint32_t find(uint32_t* P, uint32_t u, bool ac, uint32_t pu = kEmpty) {
  if constexpr (F == kFindNaive) {
    uint32_t x = u;
    for (;;) {
      uint32_t p = ld(&P[x]);
      if (p == x) return x;
      x = p;
    }
  } else if constexpr (F == kFindSplit) {
    // After the split step u moves to v, whose parent w was just read: it is
    // carried into the next step instead of being read again.
    uint32_t v = pu != kEmpty ? pu : ld(&P[u]);
    for (;;) {
      if (v == u) return u;
      const uint32_t w = ld(&P[v]);
      if (v == w) return v;
      uint32_t e = v;
      shortcut(&P[u], e, w, ac);
      u = v;  // v < u
      v = w;
    }
  } else if constexpr (F == kFindHalve) {
    for (;;) {
      uint32_t v = pu != kEmpty ? pu : ld(&P[u]);
      pu = kEmpty;
      if (v == u) return u;
      uint32_t w = ld(&P[v]);
      if (v == w) return v;
      uint32_t e = v;
      u = shortcut(&P[u], e, w, ac) ? w : e;  // the new P[u], smaller than u either way
    }
  } else {  // kFindCompress
    uint32_t r = u, first = kEmpty;
    for (;;) {
      uint32_t p = ld(&P[r]);
      if (first == kEmpty) first = p;
      if (p == r) break;
      r = p;
    }
    // u is the root or points at it already: no atomic on its slot (a hub's
    // slot would take one from every find that starts there)
    if (first == r) return r;
    uint32_t x = u;
    while (x != r) {
      uint32_t old = amin(&P[x], r);
      if (old <= r) break;
      x = old;
    }
    return r;
  }
}

// ------------------------------------------------------------------ unions
// Union-Async (Appendix A.2): find both roots; CAS the larger root onto the
// smaller; on failure the CAS result is the new parent of the former root and
// the search resumes from there.
template <int F>
GCONN_HD bool union_async(const LinkCtx& c, uint32_t u, uint32_t v) {
  uint32_t pu = find<F>(c.P, u, c.atomic_compress), pv = find<F>(c.P, v, c.atomic_compress);
  while (pu != pv) {
    if (pu < pv) {
      uint32_t t = pu;
      pu = pv;
      pv = t;
    }
    uint32_t e = pu;
    if (cas(&c.P[pu], e, pv)) {
      record_link(c, pu, u, v);
      return true;
    }
    pu = find<F>(c.P, e, c.atomic_compress);
    pv = find<F>(c.P, pv, c.atomic_compress);
  }
  return false;
}

// Union-Hooks (Appendix A.2): the race is decided by a CAS on H[p_u]; the
// winner then writes P[p_u] without contention.  A loser follows the claimed
// hook target instead of waiting for the winner's write (a lane of the same
// wave may be that winner, and lanes of one wave make no independent progress).
template <int F>
GCONN_HD bool union_hooks(const LinkCtx& c, uint32_t u, uint32_t v) {
  uint32_t pu = find<F>(c.P, u, c.atomic_compress), pv = find<F>(c.P, v, c.atomic_compress);
  while (pu != pv) {
    if (pu < pv) {
      uint32_t t = pu;
      pu = pv;
      pv = t;
    }
    // A stale "still a root" read here would send the lane to a hook CAS that
    // is bound to fail, so this test reads the parent coherently.
    uint32_t next = ld_agent(&c.P[pu]);
    if (next == pu) {
      uint32_t h = kEmpty;
      if (cas(&c.H[pu], h, pv)) {
        st(&c.P[pu], pv);
        record_link(c, pu, u, v);
        return true;
      }
      next = h;  // pu is being linked under h
    }
    pu = find<F>(c.P, next, c.atomic_compress);
    pv = find<F>(c.P, pv, c.atomic_compress);
  }
  return false;
}

// Union-Early (Appendix A.2): walk the two paths together, always advancing the
// larger endpoint with a splitting step, and link it the moment it is a root.
// Optional trailing finds compress both paths.
template <int F>
GCONN_HD bool union_early(const LinkCtx& c, uint32_t u, uint32_t v) {
  uint32_t pu = u, pv = v;
  bool linked = false;
  while (pu != pv) {
    if (pu < pv) {
      uint32_t t = pu;
      pu = pv;
      pv = t;
    }
    uint32_t z = ld(&c.P[pu]);
    if (z == pu) {
      uint32_t e = pu;
      if (cas(&c.P[pu], e, pv)) {
        record_link(c, pu, u, v);
        linked = true;
        break;
      }
      z = e;
    }
    uint32_t w = ld(&c.P[z]);
    if (w != z) {
      uint32_t e = z;
      shortcut(&c.P[pu], e, w, c.atomic_compress);
    }
    pu = w;
  }
  if constexpr (F != kFindNaive) {
    find<F>(c.P, u, c.atomic_compress);
    find<F>(c.P, v, c.atomic_compress);
  }
  return linked;
}

// Union-Rem-CAS (Appendix A.2): compare the parents of the two current nodes;
// the side with the larger parent either is a root (CAS it onto the other
// side's parent) or takes one splice step towards its root.
// The parents compared in each iteration are carried from the previous one:
// after a split step the new r_u's parent is the value the step just read,
// and r_v's side did not move.  A carried value can be older than a fresh
// read, which the argument above already allows for; the hook itself is a CAS
// that validates r_u is still a root.
template <int F, int S>
GCONN_HD bool union_rem_cas(const LinkCtx& c, uint32_t u, uint32_t v, uint32_t pu = kEmpty,
                            uint32_t pv = kEmpty, uint32_t eu = kEmpty, uint32_t ev = kEmpty) {
  // pu, pv: values P[u], P[v] are known to have held (a caller that loaded
  // them ahead of time); kEmpty reads them here.  eu, ev: the input edge a
  // spanning forest records for a link (kEmpty: (u, v) itself) -- a caller
  // may unite an ancestor u of eu instead of eu, which joins the same sets.
  uint32_t ru = u, rv = v;
  uint32_t pru = pu != kEmpty ? pu : ld(&c.P[ru]), prv = pv != kEmpty ? pv : ld(&c.P[rv]);
  for (;;) {
    if (pru == prv) return false;
    if (pru < prv) {
      uint32_t t = ru;
      ru = rv;
      rv = t;
      t = pru;
      pru = prv;
      prv = t;
    }
    if (ru == pru) {
#if GCONN_ROOT_RECHECK
      {
        const uint32_t fresh = ld_agent(&c.P[ru]);
        if (fresh != ru) {
          pru = fresh;
          continue;
        }
      }
#endif
      uint32_t e = ru;
      if (cas(&c.P[ru], e, prv)) {
        record_link(c, ru, eu != kEmpty ? eu : u, ev != kEmpty ? ev : v);
        if constexpr (F != kFindNaive) {
          // P[ru] is now prv, and prv was read as P[rv]: an endpoint that is
          // ru or rv starts its compressing find from prv.
          find<F>(c.P, u, c.atomic_compress, (u == ru || u == rv) ? prv : kEmpty);
          find<F>(c.P, v, c.atomic_compress, (v == ru || v == rv) ? prv : kEmpty);
        }
        return true;
      }
      pru = e;  // ru was linked meanwhile: continue from its fresh parent
    }
    const uint32_t w = ld(&c.P[pru]);
    if (w != pru) {
      uint32_t e = pru;
      shortcut(&c.P[ru], e, w, c.atomic_compress);
    }
    if constexpr (S == kSpliceSplitOne) {
      ru = pru;  // P[pru] = w was just read
      pru = w;
    } else {
      ru = w;
      pru = ld(&c.P[w]);
    }
  }
}

// Union-Rem-CAS with Rem's own splice (SpliceAtomic, Appendix A.2): while the
// two current nodes have different parents, the one with the larger parent is
// either a root (CAS it under the other parent) or is re-hung under the other
// node's parent by a CAS, and the walk moves on to its old parent, whose side
// of the union is still pending.  A splice moves a node out of its ancestors'
// path, so the carried-value shortcuts of union_rem_cas do not apply: both
// parents are re-read, device-coherently, on every iteration, and a failed
// CAS only means the next iteration sees the new parent.
// pu, pv (kEmpty: none): values P[u], P[v] held at some time, read without
// coherence (an L2 copy may be stale); the first iteration compares them
// instead of fresh reads.  Every value P[x] ever holds lies in the set x
// belongs to once the phase's unions are done (each write stores an id of
// the union's other side, and that union goes on to join the two sides), so
// comparing a stale value unites sets that end up joined anyway, and a stale
// "root" only costs one CAS that fails, after which the reads are coherent.
template <int F>
GCONN_HD bool union_rem_splice(const LinkCtx& c, uint32_t u, uint32_t v, uint32_t pu = kEmpty,
                               uint32_t pv = kEmpty) {
  uint32_t ru = u, rv = v;
  for (;;) {
    uint32_t pru = pu != kEmpty ? pu : ld_agent(&c.P[ru]);
    uint32_t prv = pv != kEmpty ? pv : ld_agent(&c.P[rv]);
    pu = pv = kEmpty;
    if (pru == prv) return false;
    if (pru < prv) {
      uint32_t t = ru;
      ru = rv;
      rv = t;
      t = pru;
      pru = prv;
      prv = t;
    }
    uint32_t e = pru;
    if (ru == pru) {
      if (cas(&c.P[ru], e, prv)) {
        record_link(c, ru, u, v);
        if constexpr (F != kFindNaive) {
          // P[ru] is now prv, and prv was read as P[rv]: an endpoint that is
          // ru or rv starts its compressing find from prv (a value its slot
          // has held) instead of reading it again
          find<F>(c.P, u, true, (u == ru || u == rv) ? prv : kEmpty);
          find<F>(c.P, v, true, (v == ru || v == rv) ? prv : kEmpty);
        }
        return true;
      }
      continue;
    }
    cas(&c.P[ru], e, prv);  // splice; on failure P[ru] moved and is re-read next time
    ru = pru;
  }
}

// G_Afforest's link (the finish of Afforest, Sutton et al. 2018, brought into
// the framework; Related Work and the state-of-the-art comparison): compare
// the parents of the two endpoints; when they differ, the higher one either
// already points at the lower (done), or is a root and is CASed under the
// lower, or both sides move up (the higher side by two levels).  No path
// compression happens here: a separate full compress pass follows.  Every
// iteration lowers the larger of the two values compared, so it terminates.
GCONN_HD bool union_afforest(const LinkCtx& c, uint32_t u, uint32_t v) {
  uint32_t p1 = ld(&c.P[u]), p2 = ld(&c.P[v]);
  while (p1 != p2) {
    const uint32_t high = p1 > p2 ? p1 : p2, low = p1 > p2 ? p2 : p1;
    const uint32_t ph = ld(&c.P[high]);
    if (ph == low) return false;
    if (ph == high) {
      uint32_t e = high;
      if (cas(&c.P[high], e, low)) {
        record_link(c, high, u, v);
        return true;
      }
    }
    p1 = ld(&c.P[ld(&c.P[high])]);
    p2 = ld(&c.P[low]);
  }
  return false;
}

// Union-Rem-Lock (Appendix A.2, after Patwary et al.): Rem's walk, the link of
// a root made under a lock on that root.  GPU lanes of one wave run in
// lockstep, so a lane spinning on a lock held by another lane of its wave
// would never let the holder run: the lock is only ever tried, and a lane that
// gets it does the guarded check-and-link and releases it in the same step;
// a lane that does not get it re-reads and tries again.  The lock array is
// LinkCtx::H (kEmpty = free).  As printed the procedure returns after the
// critical section whether or not the link happened; a failed check (the root
// was linked meanwhile) continues the walk instead.  Compression runs when the
// walk ends without a link, as in the listing.
template <int F, int S>
GCONN_HD bool union_rem_lock(const LinkCtx& c, uint32_t u, uint32_t v) {
  uint32_t ru = u, rv = v;
  for (;;) {
    uint32_t pru = ld_agent(&c.P[ru]), prv = ld_agent(&c.P[rv]);
    if (pru == prv) break;
    if (pru < prv) {
      uint32_t t = ru;
      ru = rv;
      rv = t;
      t = pru;
      pru = prv;
      prv = t;
    }
    if (ru == pru) {
      uint32_t lk = kEmpty;
      if (__hip_atomic_compare_exchange_strong(&c.H[ru], &lk, 0u, __ATOMIC_ACQUIRE,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        const uint32_t pv = ld_agent(&c.P[rv]);
        const bool ok = ld_agent(&c.P[ru]) == ru && ru > pv;
        if (ok) st(&c.P[ru], pv);
        __hip_atomic_store(&c.H[ru], kEmpty, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (ok) {
          record_link(c, ru, u, v);
          return true;
        }
      }
      continue;
    }
    if constexpr (S == kSpliceAtomic) {
      uint32_t e = pru;
      cas(&c.P[ru], e, prv);
      ru = pru;
    } else {
      const uint32_t w = ld_agent(&c.P[pru]);
      if (w != pru) {
        uint32_t e = pru;
        cas(&c.P[ru], e, w);
      }
      ru = (S == kSpliceSplitOne) ? pru : w;
    }
  }
  if constexpr (F != kFindNaive) {
    find<F>(c.P, u, true);
    find<F>(c.P, v, true);
  }
  return false;
}

// Compile-time rule bundle.
template <int U, int F, int S>
struct Rule {
  static constexpr int kUnion = U, kFind = F, kSplice = S;
  GCONN_HD static bool unite(const LinkCtx& c, uint32_t u, uint32_t v) {
    if constexpr (U == kUnionAsync) return union_async<F>(c, u, v);
    else if constexpr (U == kUnionHooks) return union_hooks<F>(c, u, v);
    else if constexpr (U == kUnionEarly) return union_early<F>(c, u, v);
    else if constexpr (U == kUnionAfforest) return union_afforest(c, u, v);
    else if constexpr (U == kUnionRemLock) return union_rem_lock<F, S>(c, u, v);
    else if constexpr (S == kSpliceAtomic) return union_rem_splice<F>(c, u, v);
    else return union_rem_cas<F, S>(c, u, v);
  }
  // The same union, given parent values of u and v loaded ahead of time (any
  // value a slot has held is an ancestor, so a stale one is a valid start).
  // Only Union-Rem-CAS (SplitAtomicOne / HalveAtomicOne) uses them.
  GCONN_HD static bool unite_from(const LinkCtx& c, uint32_t u, uint32_t v, uint32_t pu,
                                  uint32_t pv) {
    if constexpr (U == kUnionRemCas && S != kSpliceAtomic) return union_rem_cas<F, S>(c, u, v, pu, pv);
    else if constexpr (U == kUnionRemCas) return union_rem_splice<F>(c, u, v, pu, pv);
    else return unite(c, u, v);
  }
  // The union of the input edge (eu, v), started from u, an ancestor of eu
  // (same set), with parent values pu, pv loaded ahead of time as above.  A
  // spanning forest records (eu, v).  Union-Rem-CAS with SplitAtomicOne /
  // HalveAtomicOne starts from u; the other rules unite (u, v) when no forest
  // is recorded and (eu, v) when one is.
  // The union of the input edge (eu, ev) started from a and b, members of
  // eu's and ev's sets: Union-Rem-CAS with SplitAtomicOne / HalveAtomicOne
  // unites (a, b) and records (eu, ev) in a spanning forest; the other rules
  // unite (a, b) when no forest is recorded and (eu, ev) when one is.
  GCONN_HD static bool unite_pair(const LinkCtx& c, uint32_t a, uint32_t b, uint32_t eu,
                                  uint32_t ev) {
    if constexpr (U == kUnionRemCas && S != kSpliceAtomic)
      return union_rem_cas<F, S>(c, a, b, kEmpty, kEmpty, eu, ev);
    else if (c.fu) return unite(c, eu, ev);
    else return unite(c, a, b);
  }
  GCONN_HD static bool unite_edge(const LinkCtx& c, uint32_t u, uint32_t v, uint32_t pu,
                                  uint32_t pv, uint32_t eu) {
    if constexpr (U == kUnionRemCas && S != kSpliceAtomic)
      return union_rem_cas<F, S>(c, u, v, pu, pv, eu, v);
    else return unite(c, c.fu ? eu : u, v);
  }
};

}  // namespace gconn
