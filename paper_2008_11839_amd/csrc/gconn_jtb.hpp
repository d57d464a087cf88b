// gconn_jtb.hpp -- Union-JTB: randomized linking by rank with FindSimple or
// FindTwoTrySplit (Finish Algorithms, union-find; the paper takes the
// algorithm from Jayanti, Tarjan and Boix-Adsera, PODC 2019, and defers to
// that paper for its pseudocode).
//
// Reading adopted here.  Every vertex x owns one 64-bit word W[x] holding its
// parent (low 32 bits) and its rank (high 32 bits); x is a root iff its parent
// is x.  Roots are ordered by (rank, key), key a seeded random bijection of
// the id, so the order is total and ties in rank are broken at random.  A
// union finds both roots and hangs the lower one under the higher one with a
// single 64-bit CAS that expects the lower root's word exactly as read:
// parent == itself *and* the same rank, which is why the rule needs 64-bit
// CAS (the paper attributes its extra cost to them).  When the two ranks were
// equal the new parent's rank is then raised by one with a second CAS that
// expects it unchanged and still a root; if that fails the parent has moved
// on, and the link stands.  Only roots are ever linked or have their rank
// changed, so a non-root's (rank, key) is frozen and every parent is above its
// children in the order: the forest stays acyclic and every walk ends.
//
// FindTwoTrySplit: at each vertex u of the walk (parent v, grandparent w),
// try the splitting CAS of u's parent from v to w; then re-read u's parent v'
// and its parent w' and try the CAS from v' to w' once more; then move to v'.
// FindSimple walks without writing.  Compression CASes keep the rank field,
// so they never disturb the rank order.
//
// Unlike the min-linking rules, the surviving root of a component is not its
// minimum vertex; canonical labels (component minima) are computed after the
// unions by a separate reduction.
//
// Memory model as for the 32-bit rules: reads inside the walks are relaxed
// loads that may be stale (any value W[x] has held names an ancestor of x),
// links and splits are agent-scope CASes, and after a failed CAS the walk
// continues from the fresh value the CAS returned.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gconn_rules.hpp"

namespace gconn {

enum JtbFind : int { kJtbFindSimple = 0, kJtbFindTwoTrySplit = 1 };

constexpr uint64_t kNoWord = ~0ull;  // "read the word" (no vertex has rank 2^32 - 1)

GCONN_HD uint64_t jtb_word(uint32_t parent, uint32_t rank) {
  return ((uint64_t)rank << 32) | parent;
}
GCONN_HD uint32_t jtb_parent(uint64_t w) { return (uint32_t)w; }
GCONN_HD uint32_t jtb_rank(uint64_t w) { return (uint32_t)(w >> 32); }

GCONN_HD uint64_t jtb_ld(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, GCONN_P_LOAD_SCOPE);
}
GCONN_HD bool jtb_cas(uint64_t* p, uint64_t& expected, uint64_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Random priority of a root: MurmurHash3's 32-bit finaliser of (id ^ salt),
// a bijection, so distinct ids never tie.
GCONN_HD uint32_t jtb_key(uint32_t x, uint32_t salt) {
  uint32_t h = x ^ salt;
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// Is root a (word wa) below root b (word wb) in the (rank, key) order?
GCONN_HD bool jtb_below(uint64_t wa, uint32_t a, uint64_t wb, uint32_t b, uint32_t salt) {
  const uint32_t ra = jtb_rank(wa), rb = jtb_rank(wb);
  if (ra != rb) return ra < rb;
  return jtb_key(a, salt) < jtb_key(b, salt);
}

struct JtbCtx {
  uint64_t* W;                // (rank, parent) words
  uint32_t* fu;               // spanning-forest slots (nullable)
  uint32_t* fv;
  unsigned long long* hooks;  // successful-link counter (nullable)
  uint32_t salt;              // seeds the tie-breaking keys
};

// Root of u's tree; *wr receives the word the root was seen with.  wu: a word
// W[u] is known to have held, or kNoWord to read it.
template <int F>
GCONN_HD uint32_t jtb_find(uint64_t* W, uint32_t u, uint64_t wu, uint64_t* wr) {
  if (wu == kNoWord) wu = jtb_ld(&W[u]);
  for (;;) {
    uint32_t v = jtb_parent(wu);
    if (v == u) {
      *wr = wu;
      return u;
    }
    uint64_t wv = jtb_ld(&W[v]);
    uint32_t w = jtb_parent(wv);
    if (w == v) {
      *wr = wv;
      return v;
    }
    if constexpr (F == kJtbFindTwoTrySplit) {
      // First try at u.  Either way e ends as a value W[u] has held.
      uint64_t e = wu;
      const uint64_t first = jtb_word(w, jtb_rank(wu));
      if (jtb_cas(&W[u], e, first)) e = first;
      // Second try at u, from u's current parent.
      v = jtb_parent(e);
      wv = jtb_ld(&W[v]);
      w = jtb_parent(wv);
      if (w == v) {
        *wr = wv;
        return v;
      }
      uint64_t e2 = e;
      jtb_cas(&W[u], e2, jtb_word(w, jtb_rank(e)));
    }
    u = v;
    wu = wv;
  }
}

template <int F>
GCONN_HD void jtb_unite(const JtbCtx& c, uint32_t x, uint32_t y) {
  uint32_t u = x, v = y;
  uint64_t wu = kNoWord, wv = kNoWord;
  for (;;) {
    uint64_t ru, rv;
    u = jtb_find<F>(c.W, u, wu, &ru);
    v = jtb_find<F>(c.W, v, wv, &rv);
    if (u == v) return;
    if (!jtb_below(ru, u, rv, v, c.salt)) {
      const uint32_t t = u;
      u = v;
      v = t;
      const uint64_t tw = ru;
      ru = rv;
      rv = tw;
    }
    // u is the lower root: hang it under v, keeping its rank.
    uint64_t e = ru;
    if (jtb_cas(&c.W[u], e, jtb_word(v, jtb_rank(ru)))) {
      if (c.fu) {  // u is linked once and never becomes a root again
        c.fu[u] = x;
        c.fv[u] = y;
      }
      if (c.hooks)
        __hip_atomic_fetch_add(c.hooks, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (jtb_rank(ru) == jtb_rank(rv)) {
        uint64_t ev = rv;
        jtb_cas(&c.W[v], ev, jtb_word(v, jtb_rank(rv) + 1));  // fails only if v moved on
      }
      return;
    }
    // e is u's fresh word (u was linked, or its rank rose): continue from it.
    wu = e;
    wv = rv;
  }
}

}  // namespace gconn
