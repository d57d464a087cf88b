// CPU stress harness for the union-find rules of the HIP library: the same
// header (gconn_rules.hpp) compiled for the host, run from many std::threads
// on one shared parent array.  Test infrastructure only.
//
//   rules_stress <edges.bin> <n> <rule> <threads> <labels.out> [atomic_compress]
//                [stale_percent]
// edges.bin: uint32 pairs; rule: 0-3 Async (naive/split/halve/compress),
// 4-7 Hooks, 8-11 Early, 12-17 Rem-CAS (naive/split/halve x split_one/halve_one),
// 18-20 Rem-CAS with Rem's splice (naive/split/halve), 21 G_Afforest's link,
// 22-25 Rem-Lock (naive/split_one, split/split_one, halve/halve_one, split/splice),
// 26-27 Union-JTB (FindSimple, FindTwoTrySplit) on 64-bit (rank, parent) words.
// Writes labels (the minimum vertex of every vertex's tree, uint32) and prints
// the hook count.
//
// stale_percent > 0 models the incoherent L2 of an XCD for the rules' cached
// reads (ld): every thread keeps a private direct-mapped copy of the parent
// entries it has read (4096 slots, tagged by address); a read returns the
// copy, however old, with probability stale_percent / 100 when the slot holds
// that address, and otherwise reads memory and refreshes the copy.  The
// thread's own CAS and stores do not update its copy, so it can even read back
// a value older than one it wrote.  Device-coherent reads (ld_agent) and the
// atomics always see memory.  Every other union then starts from parent values
// read through this model (Rule::unite_from), as the prefetching kernels do.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

namespace stale {
struct Line {
  const uint32_t* tag;
  uint32_t value;
};
static int g_percent = 0;
thread_local Line t_cache[4096];
thread_local uint64_t t_rng = 0;
inline uint32_t next_u32() {
  if (t_rng == 0) t_rng = 0x9E3779B97F4A7C15ull ^ (uint64_t)(uintptr_t)&t_rng;
  t_rng ^= t_rng << 13;
  t_rng ^= t_rng >> 7;
  t_rng ^= t_rng << 17;
  return (uint32_t)(t_rng >> 32);
}
inline uint32_t load(const uint32_t* p) {
  Line& l = t_cache[((uintptr_t)p >> 2) & 4095];
  if (g_percent > 0 && l.tag == p && next_u32() % 100 < (uint32_t)g_percent) return l.value;
  const uint32_t v = __atomic_load_n(p, __ATOMIC_RELAXED);
  l.tag = p;
  l.value = v;
  return v;
}
}  // namespace stale
#define GCONN_HOST_STALE_LOAD(p) ::stale::load(p)

#include "../../paper_2008_11839_amd/csrc/gconn_jtb.hpp"
#include "../../paper_2008_11839_amd/csrc/gconn_rules.hpp"

using namespace gconn;

template <class R>
void run(const std::vector<uint32_t>& e, LinkCtx c, int threads) {
  const size_t m = e.size() / 2;
  std::vector<std::thread> ts;
  for (int t = 0; t < threads; ++t)
    ts.emplace_back([&, t] {
      // interleaved slices so that threads race on the same regions; with
      // stale reads modelled, every other union starts from parent values
      // read through the stale model (unite_from: the starting points the
      // prefetching kernels hand over)
      for (size_t i = t; i < m; i += threads) {
        const uint32_t u = e[2 * i], v = e[2 * i + 1];
        if (stale::g_percent > 0 && (i & 1))
          R::unite_from(c, u, v, ld(&c.P[u]), ld(&c.P[v]));
        else
          R::unite(c, u, v);
      }
    });
  for (auto& th : ts) th.join();
}

template <int F>
void run_jtb(const std::vector<uint32_t>& e, JtbCtx c, int threads) {
  const size_t m = e.size() / 2;
  std::vector<std::thread> ts;
  for (int t = 0; t < threads; ++t)
    ts.emplace_back([&, t] {
      for (size_t i = t; i < m; i += threads) jtb_unite<F>(c, e[2 * i], e[2 * i + 1]);
    });
  for (auto& th : ts) th.join();
}

// Union-JTB: every parent must lie above its child in the (rank, key) order
// and hold a rank no lower; labels are the minimum vertex of each tree.
int jtb_main(const std::vector<uint32_t>& e, uint32_t n, int rule, int threads, const char* out) {
  std::vector<uint64_t> W(n);
  for (uint32_t v = 0; v < n; ++v) W[v] = jtb_word(v, 0);
  unsigned long long hooks = 0;
  const uint32_t salt = 0x9e3779b9u;
  JtbCtx c{W.data(), nullptr, nullptr, &hooks, salt};
  if (rule == 26) run_jtb<kJtbFindSimple>(e, c, threads);
  else run_jtb<kJtbFindTwoTrySplit>(e, c, threads);
  std::vector<uint32_t> root(n), lab(n);
  for (uint32_t v = 0; v < n; ++v) {
    uint32_t r = v;
    for (;;) {
      const uint32_t p = jtb_parent(W[r]);
      if (p == r) break;
      if (jtb_rank(W[p]) < jtb_rank(W[r])) return 6;
      if (!jtb_below(W[r], r, W[p], p, salt)) return 6;
      r = p;
    }
    root[v] = r;
  }
  for (uint32_t v = 0; v < n; ++v) lab[v] = kEmpty;
  for (uint32_t v = 0; v < n; ++v)
    if (v < lab[root[v]]) lab[root[v]] = v;
  for (uint32_t v = 0; v < n; ++v) lab[v] = lab[root[v]];
  FILE* o = fopen(out, "wb");
  if (!o) return 7;
  fwrite(lab.data(), 4, n, o);
  fclose(o);
  printf("%llu\n", hooks);
  return 0;
}

int main(int argc, char** argv) {
  if (argc < 6 || argc > 8) return 2;
  if (argc == 8) stale::g_percent = atoi(argv[7]);
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 3;
  std::vector<uint32_t> e;
  uint32_t buf[4096];
  size_t got;
  while ((got = fread(buf, 4, 4096, f)) > 0) e.insert(e.end(), buf, buf + got);
  fclose(f);
  const uint32_t n = (uint32_t)atoi(argv[2]);
  const int rule = atoi(argv[3]), threads = atoi(argv[4]);
  for (uint32_t x : e)
    if (x >= n) return 4;
  if (rule == 26 || rule == 27) return jtb_main(e, n, rule, threads, argv[5]);
  std::vector<uint32_t> P(n), H(n, kEmpty);
  for (uint32_t v = 0; v < n; ++v) P[v] = v;
  unsigned long long hooks = 0;
  const uint32_t ac = argc >= 7 ? (uint32_t)atoi(argv[6]) : 1u;
  LinkCtx c{P.data(), H.data(), nullptr, nullptr, &hooks, ac};
  switch (rule) {
    case 0: run<Rule<kUnionAsync, kFindNaive, 0>>(e, c, threads); break;
    case 1: run<Rule<kUnionAsync, kFindSplit, 0>>(e, c, threads); break;
    case 2: run<Rule<kUnionAsync, kFindHalve, 0>>(e, c, threads); break;
    case 3: run<Rule<kUnionAsync, kFindCompress, 0>>(e, c, threads); break;
    case 4: run<Rule<kUnionHooks, kFindNaive, 0>>(e, c, threads); break;
    case 5: run<Rule<kUnionHooks, kFindSplit, 0>>(e, c, threads); break;
    case 6: run<Rule<kUnionHooks, kFindHalve, 0>>(e, c, threads); break;
    case 7: run<Rule<kUnionHooks, kFindCompress, 0>>(e, c, threads); break;
    case 8: run<Rule<kUnionEarly, kFindNaive, 0>>(e, c, threads); break;
    case 9: run<Rule<kUnionEarly, kFindSplit, 0>>(e, c, threads); break;
    case 10: run<Rule<kUnionEarly, kFindHalve, 0>>(e, c, threads); break;
    case 11: run<Rule<kUnionEarly, kFindCompress, 0>>(e, c, threads); break;
    case 12: run<Rule<kUnionRemCas, kFindNaive, kSpliceSplitOne>>(e, c, threads); break;
    case 13: run<Rule<kUnionRemCas, kFindSplit, kSpliceSplitOne>>(e, c, threads); break;
    case 14: run<Rule<kUnionRemCas, kFindHalve, kSpliceSplitOne>>(e, c, threads); break;
    case 15: run<Rule<kUnionRemCas, kFindNaive, kSpliceHalveOne>>(e, c, threads); break;
    case 16: run<Rule<kUnionRemCas, kFindSplit, kSpliceHalveOne>>(e, c, threads); break;
    case 17: run<Rule<kUnionRemCas, kFindHalve, kSpliceHalveOne>>(e, c, threads); break;
    case 18: c.atomic_compress = 1; run<Rule<kUnionRemCas, kFindNaive, kSpliceAtomic>>(e, c, threads); break;
    case 19: c.atomic_compress = 1; run<Rule<kUnionRemCas, kFindSplit, kSpliceAtomic>>(e, c, threads); break;
    case 20: c.atomic_compress = 1; run<Rule<kUnionRemCas, kFindHalve, kSpliceAtomic>>(e, c, threads); break;
    case 21: run<Rule<kUnionAfforest, kFindNaive, 0>>(e, c, threads); break;
    case 22: run<Rule<kUnionRemLock, kFindNaive, kSpliceSplitOne>>(e, c, threads); break;
    case 23: run<Rule<kUnionRemLock, kFindSplit, kSpliceSplitOne>>(e, c, threads); break;
    case 24: run<Rule<kUnionRemLock, kFindHalve, kSpliceHalveOne>>(e, c, threads); break;
    case 25: run<Rule<kUnionRemLock, kFindSplit, kSpliceAtomic>>(e, c, threads); break;
    default: return 5;
  }
  std::vector<uint32_t> lab(n);
  for (uint32_t v = 0; v < n; ++v) {
    uint32_t r = v;
    while (P[r] != r) {
      if (P[r] > r) return 6;  // a parent must have a smaller id
      r = P[r];
    }
    lab[v] = r;
  }
  FILE* o = fopen(argv[5], "wb");
  if (!o) return 7;
  fwrite(lab.data(), 4, n, o);
  fclose(o);
  printf("%llu\n", hooks);
  return 0;
}
