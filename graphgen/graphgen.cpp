// Seeded synthetic graph generators (input side only).
//
// This module produces the inputs that both the CPU oracle and the GPU path
// consume: edge lists (COO) and symmetrised CSR with sorted rows.  It holds no
// connectivity arithmetic of any kind (no union-find, no labels); it only draws
// random graphs and lays them out.
//
// Randomness: every draw is the i-th output of SplitMix64 (Steele, Lea and
// Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014) started
// from a per-(seed, stream) key, so any index can be generated independently
// and in parallel, and a Python mirror can reproduce single values.
//
// Families (the paper's graph classes, Table of inputs; synthetic stand-ins):
//   * Erdos-Renyi: m uniform endpoint pairs, self-loops dropped, duplicates kept.
//   * RMAT (Chakrabarti, Zhan, Faloutsos 2004): quadrant probabilities (a,b,c,d)
//     per level, optional seeded bijective id scramble (Graph500 style),
//     rejection of ids >= n when n is not a power of two.
//   * 2D / 3D bond-percolation grids: each lattice edge kept i.i.d. with prob p.
//   * Barabasi-Albert preferential attachment, drawn with the Batagelj-Brandes
//     edge-copy method (Phys. Rev. E 71, 036113, 2005): edge slot j of vertex v
//     attaches v to the endpoint in a uniform earlier slot of the endpoint list,
//     which picks targets in proportion to degree.
// Build: g++ -O2 -fopenmp -shared -fPIC (no -march=native: the library travels).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ULL;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// i-th output (0-based) of SplitMix64 whose state starts at `key`.
inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * kGamma); }

// Uniform integer in [0, n) from 32 random bits (multiply-shift).
inline uint32_t below(uint32_t r32, uint32_t n) {
  return (uint32_t)(((uint64_t)r32 * (uint64_t)n) >> 32);
}

inline uint32_t threshold32(double p) {
  if (p <= 0.0) return 0;
  if (p >= 1.0) return 0xFFFFFFFFu;
  return (uint32_t)std::floor(p * 4294967296.0);
}

// Chunked parallel "generate then compact" driver: gen(i, &u, &v) -> keep?
template <class Gen>
int64_t generate_compact(uint64_t count, uint32_t* src, uint32_t* dst, Gen gen) {
  int T = omp_get_max_threads();
  if (T < 1) T = 1;
  uint64_t chunk = (count + T - 1) / T;
  std::vector<uint64_t> kept(T + 1, 0);
#pragma omp parallel num_threads(T)
  {
    int t = omp_get_thread_num();
    uint64_t lo = std::min<uint64_t>(count, (uint64_t)t * chunk);
    uint64_t hi = std::min<uint64_t>(count, lo + chunk);
    uint64_t c = 0;
    uint32_t u, v;
    for (uint64_t i = lo; i < hi; ++i)
      if (gen(i, &u, &v)) ++c;
    kept[t + 1] = c;
#pragma omp barrier
#pragma omp single
    for (int j = 0; j < T; ++j) kept[j + 1] += kept[j];
    uint64_t w = kept[t];
    for (uint64_t i = lo; i < hi; ++i)
      if (gen(i, &u, &v)) {
        src[w] = u;
        dst[w] = v;
        ++w;
      }
  }
  return (int64_t)kept[T];
}

// Seeded bijection on [0, 2^scale): odd-multiply / add / xorshift rounds.
struct Scramble {
  uint64_t mask, m1, a1, m2, a2;
  uint32_t s1, s2;
  bool on;
  Scramble(uint32_t scale, uint64_t key, bool enable) {
    on = enable && scale > 0;
    mask = (scale >= 64) ? ~0ULL : ((1ULL << scale) - 1);
    m1 = draw(key, 0) | 1ULL;
    a1 = draw(key, 1);
    m2 = draw(key, 2) | 1ULL;
    a2 = draw(key, 3);
    s1 = scale / 2 + 1;
    s2 = scale / 3 + 1;
  }
  uint32_t operator()(uint32_t x) const {
    if (!on) return x;
    uint64_t y = x;
    y = (y * m1 + a1) & mask;
    y ^= (y >> s1);
    y = (y * m2 + a2) & mask;
    y ^= (y >> s2);
    return (uint32_t)(y & mask);
  }
};

}  // namespace

extern "C" {

uint64_t gg_key(uint64_t seed, uint64_t stream) {
  return mix64(mix64(seed ^ 0x5851f42d4c957f2dULL) + (stream + 1) * kGamma);
}

uint64_t gg_draw(uint64_t key, uint64_t i) { return draw(key, i); }

uint64_t gg_splitmix64_next(uint64_t* state) {
  *state += kGamma;
  return mix64(*state);
}

// Erdos-Renyi: m_draws uniform pairs over [0,n); self-loops dropped.
// Writes at most m_draws undirected edges; returns the number kept.
int64_t gg_er_edges(uint32_t n, uint64_t m_draws, uint64_t seed, uint32_t* src, uint32_t* dst) {
  if (n == 0) return 0;
  const uint64_t key = gg_key(seed, 1);
  return generate_compact(m_draws, src, dst, [&](uint64_t i, uint32_t* u, uint32_t* v) {
    uint64_t r = draw(key, i);
    *u = below((uint32_t)r, n);
    *v = below((uint32_t)(r >> 32), n);
    return *u != *v;
  });
}

// RMAT at `scale` levels, ids restricted to [0,n) by redrawing the whole edge
// (attempt t uses stream 16+t).  Probabilities a,b,c (d = 1-a-b-c).
int64_t gg_rmat_edges(uint32_t scale, uint32_t n, uint64_t m_draws, double a, double b,
                      double c, uint64_t seed, int scramble, uint32_t* src, uint32_t* dst) {
  if (n == 0 || scale == 0 || scale > 32) return 0;
  if (scale < 32 && (uint64_t)n > (1ULL << scale)) return -1;
  const uint32_t ta = threshold32(a), tab = threshold32(a + b), tabc = threshold32(a + b + c);
  const Scramble perm(scale, gg_key(seed, 2), scramble != 0);
  const uint32_t words = (scale + 1) / 2;  // two 32-bit level draws per 64-bit output
  std::vector<uint64_t> keys(64);
  for (int t = 0; t < 64; ++t) keys[t] = gg_key(seed, 16 + t);
  return generate_compact(m_draws, src, dst, [&](uint64_t i, uint32_t* pu, uint32_t* pv) {
    for (int t = 0; t < 64; ++t) {
      uint32_t u = 0, v = 0;
      for (uint32_t w = 0; w < words; ++w) {
        uint64_t r = draw(keys[t], i * words + w);
        for (int h = 0; h < 2; ++h) {
          uint32_t lvl = 2 * w + h;
          if (lvl >= scale) break;
          uint32_t x = h ? (uint32_t)(r >> 32) : (uint32_t)r;
          // quadrant: [0,ta) -> (0,0), [ta,tab) -> (0,1), [tab,tabc) -> (1,0), else (1,1)
          uint32_t bu = (uint32_t)(x >= tab);
          uint32_t bv = (uint32_t)((x >= ta) & (x < tab)) | (uint32_t)(x >= tabc);
          u = (u << 1) | bu;
          v = (v << 1) | bv;
        }
      }
      u = perm(u);
      v = perm(v);
      if (u < n && v < n) {
        *pu = u;
        *pv = v;
        return u != v;
      }
    }
    return false;  // 64 consecutive rejections: drop the draw (probability negligible)
  });
}

// 2D grid W x H, id = y*W + x; horizontal edges first, then vertical.
int64_t gg_grid2d_edges(uint32_t W, uint32_t H, double p, uint64_t seed, uint32_t* src,
                        uint32_t* dst) {
  if (W == 0 || H == 0) return 0;
  const uint64_t key = gg_key(seed, 3);
  const uint32_t th = threshold32(p);
  const bool all = p >= 1.0;
  const uint64_t nh = (uint64_t)(W - 1) * H, nv = (uint64_t)W * (H - 1);
  return generate_compact(nh + nv, src, dst, [&](uint64_t i, uint32_t* u, uint32_t* v) {
    if (i < nh) {
      uint64_t y = i / (W - 1), x = i % (W - 1);
      *u = (uint32_t)(y * W + x);
      *v = *u + 1;
    } else {
      uint64_t j = i - nh;
      *u = (uint32_t)j;
      *v = (uint32_t)(j + W);
    }
    return all || (uint32_t)draw(key, i) < th;
  });
}

// 3D grid X x Y x Z, id = (z*Y + y)*X + x; x-edges, then y-edges, then z-edges.
int64_t gg_grid3d_edges(uint32_t X, uint32_t Y, uint32_t Z, double p, uint64_t seed,
                        uint32_t* src, uint32_t* dst) {
  if (X == 0 || Y == 0 || Z == 0) return 0;
  const uint64_t key = gg_key(seed, 4);
  const uint32_t th = threshold32(p);
  const bool all = p >= 1.0;
  const uint64_t nx = (uint64_t)(X - 1) * Y * Z, ny = (uint64_t)X * (Y - 1) * Z,
                 nz = (uint64_t)X * Y * (Z - 1);
  const uint64_t plane = (uint64_t)X * Y;
  return generate_compact(nx + ny + nz, src, dst, [&](uint64_t i, uint32_t* u, uint32_t* v) {
    if (i < nx) {
      uint64_t row = i / (X - 1), x = i % (X - 1);
      *u = (uint32_t)(row * X + x);
      *v = *u + 1;
    } else if (i < nx + ny) {
      uint64_t j = i - nx;
      uint64_t z = j / ((uint64_t)X * (Y - 1)), r = j % ((uint64_t)X * (Y - 1));
      *u = (uint32_t)(z * plane + r);
      *v = *u + X;
    } else {
      uint64_t j = i - nx - ny;
      *u = (uint32_t)j;
      *v = (uint32_t)(j + plane);
    }
    return all || (uint32_t)draw(key, i) < th;
  });
}

// CSR from k edges over [0,n).  With `symmetrize`, each edge (u,v) contributes
// u->v and v->u (so nbrs must hold 2k entries); otherwise only u->v.  Rows are
// sorted ascending; duplicates and self-loops are kept as given.
// offsets: n+1 entries.  Returns the number of CSR entries, or -1 on a bad id.
int64_t gg_csr_from_edges(uint32_t n, uint64_t k, const uint32_t* src, const uint32_t* dst,
                          int symmetrize, uint64_t* offsets, uint32_t* nbrs) {
  for (uint64_t i = 0; i < k; ++i)
    if (src[i] >= n || dst[i] >= n) return -1;
  std::memset(offsets, 0, sizeof(uint64_t) * ((size_t)n + 1));
  uint64_t* deg = offsets + 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)k; ++i) {
    __atomic_fetch_add(&deg[src[i]], 1, __ATOMIC_RELAXED);
    if (symmetrize) __atomic_fetch_add(&deg[dst[i]], 1, __ATOMIC_RELAXED);
  }
  for (uint32_t v = 0; v < n; ++v) offsets[v + 1] += offsets[v];
  std::vector<uint64_t> cur(offsets, offsets + n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)k; ++i) {
    uint64_t p = __atomic_fetch_add(&cur[src[i]], 1, __ATOMIC_RELAXED);
    nbrs[p] = dst[i];
    if (symmetrize) {
      uint64_t q = __atomic_fetch_add(&cur[dst[i]], 1, __ATOMIC_RELAXED);
      nbrs[q] = src[i];
    }
  }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < (int64_t)n; ++v) std::sort(nbrs + offsets[v], nbrs + offsets[v + 1]);
  return (int64_t)offsets[n];
}

// Random permutation of [0,k) applied to an edge list in place (Fisher-Yates
// driven by the counter generator; sequential, for stream ordering).
void gg_shuffle_edges(uint64_t k, uint64_t seed, uint32_t* src, uint32_t* dst) {
  const uint64_t key = gg_key(seed, 5);
  for (uint64_t i = k; i > 1; --i) {
    uint64_t r = draw(key, k - i);
    uint64_t j = (uint64_t)(((unsigned __int128)r * i) >> 64);
    std::swap(src[i - 1], src[j]);
    std::swap(dst[i - 1], dst[j]);
  }
}

// Barabasi-Albert stream: vertex v = 0..n-1 arrives with k edges, in order.
// The endpoint list holds 2 entries per edge slot (v, target); slot e of the
// list draws r uniform in [0, 2e] and copies the endpoint stored at r (the
// first slot copies itself, a self-loop).  Self-loops are dropped, duplicates
// kept; edges come out in arrival order (sequential by construction).
int64_t gg_ba_edges(uint32_t n, uint32_t k, uint64_t seed, uint32_t* src, uint32_t* dst) {
  if (n == 0 || k == 0) return 0;
  const uint64_t key = gg_key(seed, 6);
  const uint64_t slots = (uint64_t)n * k;
  std::vector<uint32_t> target(slots);
  for (uint64_t e = 0; e < slots; ++e) {
    const uint64_t r = (uint64_t)(((unsigned __int128)draw(key, e) * (2 * e + 1)) >> 64);
    // even entry 2s: the vertex arriving with slot s; odd entry 2s+1: its target
    target[e] = (r & 1) ? target[r / 2] : (uint32_t)((r / 2) / k);
  }
  uint64_t w = 0;
  for (uint64_t e = 0; e < slots; ++e) {
    const uint32_t v = (uint32_t)(e / k);
    if (target[e] != v) {
      src[w] = v;
      dst[w] = target[e];
      ++w;
    }
  }
  return (int64_t)w;
}

// Uniform vertex pairs (query batches).
void gg_uniform_pairs(uint32_t n, uint64_t q, uint64_t seed, uint64_t stream, uint32_t* a,
                      uint32_t* b) {
  const uint64_t key = gg_key(seed, 1000 + stream);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)q; ++i) {
    uint64_t r = draw(key, (uint64_t)i);
    a[i] = below((uint32_t)r, n);
    b[i] = below((uint32_t)(r >> 32), n);
  }
}

}  // extern "C"
