/*
 * oracle.c -- plain sequential CPU reference for graph connectivity.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test-suite, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header or table with the GPU library.
 *
 * What it computes (Hong, Dhulipala, Shun, "Exploring the Design Space of
 * Static and Incremental Graph Connectivity Algorithms on GPUs", PACT 2020):
 *
 *  - Connected-component labels (Notation and Preliminaries: two vertices share
 *    a label iff they are connected).  The canonical label is the minimum
 *    vertex id of the component, which is what every min-based method of the
 *    paper converges to (Finish Algorithms: min-based algorithms keep the
 *    minimum label received; union operations link larger id to smaller id).
 *    Computed by the textbook sequential union-find of the Preliminaries:
 *    MakeSet for every vertex, Union on the endpoints of every edge, Find at the
 *    end; parents always point to a smaller id (root of a set = its minimum),
 *    with full path compression in Find.
 *  - Spanning forest (Static Spanning Forest paragraph, Alg. "GConn for
 *    Spanning Forest"): each successful union records its edge in the slot of
 *    the root that stopped being a root.
 *  - Incremental connectivity (Incremental Connectivity Support, Alg.
 *    "GConn for Incremental Connectivity"): the same union-find kept across
 *    batches; a query (a,b) is Find(a) == Find(b).
 *  - Sampling-phase partitions (Sampling Algorithms; Appendix A.1): the
 *    components of the edge subset each sampler inspects, and the most
 *    frequent label over a seeded vertex sample (GetMostFrequentLabel).
 *
 * Style: deliberately simple loops, no blocking or concurrency.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------ union-find */

/* Find with full path compression (two passes). */
static uint32_t uf_find(uint32_t* P, uint32_t x) {
  uint32_t r = x;
  while (P[r] != r) r = P[r];
  while (P[x] != r) {
    uint32_t next = P[x];
    P[x] = r;
    x = next;
  }
  return r;
}

/* Union of the sets of u and v: the root with the larger id is made a child of
 * the root with the smaller id.  Returns the root that was linked, or
 * UINT32_MAX when u and v were already in the same set. */
static uint32_t uf_union(uint32_t* P, uint32_t u, uint32_t v) {
  uint32_t ru = uf_find(P, u), rv = uf_find(P, v);
  if (ru == rv) return UINT32_MAX;
  if (ru < rv) {
    uint32_t t = ru;
    ru = rv;
    rv = t;
  }
  P[ru] = rv;
  return ru;
}

void oracle_uf_init(uint32_t* P, uint32_t n) {
  for (uint32_t v = 0; v < n; ++v) P[v] = v;
}

/* Insert k edges (src[i], dst[i]) in order.  If fu/fv are non-NULL, the edge
 * that links root r is written to fu[r], fv[r].  Returns the number of links.
 * Ids must be < n (checked: returns -1 before touching P otherwise). */
int64_t oracle_uf_insert(uint32_t* P, uint32_t n, uint64_t k, const uint32_t* src,
                         const uint32_t* dst, uint32_t* fu, uint32_t* fv) {
  for (uint64_t i = 0; i < k; ++i)
    if (src[i] >= n || dst[i] >= n) return -1;
  int64_t links = 0;
  for (uint64_t i = 0; i < k; ++i) {
    uint32_t r = uf_union(P, src[i], dst[i]);
    if (r != UINT32_MAX) {
      ++links;
      if (fu) fu[r] = src[i];
      if (fv) fv[r] = dst[i];
    }
  }
  return links;
}

/* out[i] = 1 iff a[i] and b[i] are in the same set. */
int oracle_uf_query(uint32_t* P, uint32_t n, uint64_t q, const uint32_t* a, const uint32_t* b,
                    uint8_t* out) {
  for (uint64_t i = 0; i < q; ++i)
    if (a[i] >= n || b[i] >= n) return -1;
  for (uint64_t i = 0; i < q; ++i) out[i] = (uint8_t)(uf_find(P, a[i]) == uf_find(P, b[i]));
  return 0;
}

/* labels[v] = Find(v): the minimum id of v's set. */
void oracle_uf_labels(uint32_t* P, uint32_t n, uint32_t* labels) {
  for (uint32_t v = 0; v < n; ++v) labels[v] = uf_find(P, v);
}

/* ------------------------------------------------------------ static CC */

static int csr_check(uint32_t n, const uint64_t* off, const uint32_t* nbrs) {
  if (n > 0 && off[0] != 0) return -1;
  for (uint32_t v = 0; v < n; ++v)
    if (off[v + 1] < off[v]) return -1;
  uint64_t m = n ? off[n] : 0;
  for (uint64_t e = 0; e < m; ++e)
    if (nbrs[e] >= n) return -1;
  return 0;
}

/* Static connectivity over a CSR graph (every stored entry is an edge). */
int oracle_cc_csr(uint32_t n, const uint64_t* off, const uint32_t* nbrs, uint32_t* labels) {
  if (csr_check(n, off, nbrs)) return -1;
  uint32_t* P = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
  if (!P) return -2;
  oracle_uf_init(P, n);
  for (uint32_t u = 0; u < n; ++u)
    for (uint64_t e = off[u]; e < off[u + 1]; ++e) uf_union(P, u, nbrs[e]);
  oracle_uf_labels(P, n, labels);
  free(P);
  return 0;
}

/* Static connectivity over a COO edge list. */
int oracle_cc_coo(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                  uint32_t* labels) {
  uint32_t* P = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
  if (!P) return -2;
  oracle_uf_init(P, n);
  if (oracle_uf_insert(P, n, m, src, dst, NULL, NULL) < 0) {
    free(P);
    return -1;
  }
  oracle_uf_labels(P, n, labels);
  free(P);
  return 0;
}

/* Spanning forest over CSR: fu[r], fv[r] = edge that linked root r, or
 * 0xFFFFFFFF when r was never linked.  Returns the number of forest edges. */
int64_t oracle_sf_csr(uint32_t n, const uint64_t* off, const uint32_t* nbrs, uint32_t* fu,
                      uint32_t* fv) {
  if (csr_check(n, off, nbrs)) return -1;
  uint32_t* P = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
  if (!P) return -2;
  oracle_uf_init(P, n);
  for (uint32_t v = 0; v < n; ++v) fu[v] = fv[v] = 0xFFFFFFFFu;
  int64_t links = 0;
  for (uint32_t u = 0; u < n; ++u)
    for (uint64_t e = off[u]; e < off[u + 1]; ++e) {
      uint32_t r = uf_union(P, u, nbrs[e]);
      if (r != UINT32_MAX) {
        fu[r] = u;
        fv[r] = nbrs[e];
        ++links;
      }
    }
  free(P);
  return links;
}

/* ------------------------------------------------------------ sampling */

/* k-out sampling with the first k edges of every vertex (Sampling Algorithms,
 * k-out paragraph; Appendix A.1, k-out pseudocode with the "first k" choice
 * the paper found fastest).  labels[v] = minimum id of v's component in the
 * sampled subgraph.  Returns the number of sampled edge entries. */
int64_t oracle_sample_kout(uint32_t n, const uint64_t* off, const uint32_t* nbrs, uint32_t k,
                           uint32_t* labels) {
  if (csr_check(n, off, nbrs)) return -1;
  uint32_t* P = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
  if (!P) return -2;
  oracle_uf_init(P, n);
  int64_t inspected = 0;
  for (uint32_t v = 0; v < n; ++v) {
    uint64_t deg = off[v + 1] - off[v];
    uint64_t take = deg < k ? deg : k;
    for (uint64_t j = 0; j < take; ++j) uf_union(P, v, nbrs[off[v] + j]);
    inspected += (int64_t)take;
  }
  oracle_uf_labels(P, n, labels);
  free(P);
  return inspected;
}

/* Hook-based (HB) sampling (Sampling Algorithms, HB paragraph; Appendix A.1).
 * Step 1: every vertex v with a first (smallest) neighbour w < v takes w as its
 * parent.  Step 2: every vertex still a root after step 1 unions with its first
 * N neighbours.  labels[v] = minimum id of v's component in the union of the
 * edges used by both steps.  Returns the number of edge entries inspected
 * (one per vertex with degree >= 1 in step 1, plus step 2's). */
int64_t oracle_sample_hb(uint32_t n, const uint64_t* off, const uint32_t* nbrs, uint32_t N,
                         uint32_t* labels) {
  if (csr_check(n, off, nbrs)) return -1;
  uint32_t* P = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
  uint8_t* root_after_step1 = (uint8_t*)malloc(n ? n : 1);
  if (!P || !root_after_step1) {
    free(P);
    free(root_after_step1);
    return -2;
  }
  oracle_uf_init(P, n);
  int64_t inspected = 0;
  for (uint32_t v = 0; v < n; ++v) {
    uint64_t deg = off[v + 1] - off[v];
    root_after_step1[v] = 1;
    if (deg >= 1) {
      ++inspected;
      if (nbrs[off[v]] < v) root_after_step1[v] = 0;
    }
  }
  for (uint32_t v = 0; v < n; ++v)
    if (!root_after_step1[v]) uf_union(P, v, nbrs[off[v]]);
  for (uint32_t v = 0; v < n; ++v) {
    if (!root_after_step1[v]) continue;
    uint64_t deg = off[v + 1] - off[v];
    uint64_t take = deg < N ? deg : N;
    for (uint64_t j = 0; j < take; ++j) uf_union(P, v, nbrs[off[v] + j]);
    inspected += (int64_t)take;
  }
  oracle_uf_labels(P, n, labels);
  free(P);
  free(root_after_step1);
  return inspected;
}

/* BFS sampling (Sampling Algorithms, BFS paragraph; Appendix A.1): the source
 * is the vertex of largest degree (smallest id among ties); every vertex the
 * BFS reaches takes the minimum id of the reached set, every other vertex keeps
 * its own id.  Returns the source, or -1 on bad input / n == 0. */
int64_t oracle_sample_bfs(uint32_t n, const uint64_t* off, const uint32_t* nbrs,
                          uint32_t* labels) {
  if (n == 0 || csr_check(n, off, nbrs)) return -1;
  uint32_t s = 0;
  for (uint32_t v = 1; v < n; ++v)
    if (off[v + 1] - off[v] > off[s + 1] - off[s]) s = v;
  uint32_t* queue = (uint32_t*)malloc(sizeof(uint32_t) * n);
  uint8_t* seen = (uint8_t*)calloc(n, 1);
  if (!queue || !seen) {
    free(queue);
    free(seen);
    return -2;
  }
  uint64_t head = 0, tail = 0;
  queue[tail++] = s;
  seen[s] = 1;
  uint32_t minv = s;
  while (head < tail) {
    uint32_t u = queue[head++];
    if (u < minv) minv = u;
    for (uint64_t e = off[u]; e < off[u + 1]; ++e) {
      uint32_t w = nbrs[e];
      if (!seen[w]) {
        seen[w] = 1;
        queue[tail++] = w;
      }
    }
  }
  for (uint32_t v = 0; v < n; ++v) labels[v] = seen[v] ? minv : v;
  free(queue);
  free(seen);
  return (int64_t)s;
}

/* ------------------------------------------------------------ L_max */

/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): state += golden gamma, then
 * the variant-13 finaliser. */
static uint64_t splitmix64_at(uint64_t state0, uint64_t i) {
  uint64_t z = state0 + (i + 1) * 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

uint64_t oracle_splitmix64(uint64_t state0, uint64_t i) { return splitmix64_at(state0, i); }

static int cmp_u32(const void* a, const void* b) {
  uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return (x > y) - (x < y);
}

/* GetMostFrequentLabel over a seeded sample: sample j is vertex
 * floor(hi32(SplitMix64_j(seed)) * n / 2^32), j < s.  Returns the label that
 * occurs most often among the sampled vertices, smallest label on ties. */
int64_t oracle_lmax(const uint32_t* labels, uint32_t n, uint32_t s, uint64_t seed) {
  if (n == 0 || s == 0) return -1;
  uint32_t* got = (uint32_t*)malloc(sizeof(uint32_t) * s);
  if (!got) return -2;
  for (uint32_t j = 0; j < s; ++j) {
    uint32_t hi = (uint32_t)(splitmix64_at(seed, j) >> 32);
    uint32_t v = (uint32_t)(((uint64_t)hi * n) >> 32);
    got[j] = labels[v];
  }
  qsort(got, s, sizeof(uint32_t), cmp_u32);
  uint32_t best = got[0], best_count = 0, run = 0;
  for (uint32_t j = 0; j < s; ++j) {
    run = (j > 0 && got[j] == got[j - 1]) ? run + 1 : 1;
    if (run > best_count) {
      best_count = run;
      best = got[j];
    }
  }
  free(got);
  return (int64_t)best;
}

/* Vertices that process edges in the finish phase (vertex gathering): label
 * differs from L_max and degree > 0. */
int64_t oracle_active_count(uint32_t n, const uint64_t* off, const uint32_t* labels,
                            uint32_t lmax) {
  int64_t a = 0;
  for (uint32_t v = 0; v < n; ++v)
    if (labels[v] != lmax && off[v + 1] > off[v]) ++a;
  return a;
}

/* Sum of the degrees of the active vertices (edge entries the finish reads). */
int64_t oracle_active_edges(uint32_t n, const uint64_t* off, const uint32_t* labels,
                            uint32_t lmax) {
  int64_t e = 0;
  for (uint32_t v = 0; v < n; ++v)
    if (labels[v] != lmax) e += (int64_t)(off[v + 1] - off[v]);
  return e;
}
