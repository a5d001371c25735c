// Seeded synthetic graph generators: Erdos-Renyi G(n,p), Barabasi-Albert,
// R-MAT, Watts-Strogatz and the erased configuration model.
//
// This module only produces inputs. It holds none of the Expected Force
// arithmetic, and both the CPU oracle's tests and the GPU library's tests and
// benchmark draw their graphs from it. Every generator is deterministic for a
// given seed, independent of the number of OpenMP threads.
//
// Output is always a simple undirected graph as int32 CSR: self-loops and
// duplicate edges removed, every edge stored in both directions, every row
// sorted ascending. Isolated nodes are kept.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// splitmix64: Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators" (OOPSLA 2014). Used both as a stream generator and as a
// counter-based hash (value = mix(seed, counter)).
inline uint64_t splitmix64_step(uint64_t &x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
inline uint64_t hash2(uint64_t seed, uint64_t ctr) {
  uint64_t x = seed * 0xD1B54A32D192ED03ull ^ (ctr + 0x632BE59BD9B4E019ull);
  uint64_t a = splitmix64_step(x);
  return a ^ splitmix64_step(x);
}
inline double u01(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

struct Rng {
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed * 0x9E3779B97F4A7C15ull + 0x1234567ull) {}
  uint64_t next() { return splitmix64_step(s); }
  double uniform() { return u01(next()); }
  // unbiased integer in [0, m) by rejection
  uint64_t below(uint64_t m) {
    uint64_t lim = UINT64_MAX - UINT64_MAX % m;
    uint64_t r;
    do { r = next(); } while (r >= lim);
    return r % m;
  }
};

struct Csr {
  int32_t n = 0;
  int64_t nnz = 0;
  std::vector<int32_t> row_ptr;
  std::vector<int32_t> col_idx;
};

// Build a simple undirected CSR from an undirected edge list (either
// orientation, duplicates and self-loops allowed in the input).
bool build_csr(int32_t n, const std::vector<int32_t> &src, const std::vector<int32_t> &dst,
               Csr &out) {
  const int64_t m = (int64_t)src.size();
  std::vector<int64_t> cnt((size_t)n + 1, 0);
  for (int64_t e = 0; e < m; ++e) {
    int32_t u = src[e], v = dst[e];
    if (u == v) continue;
    cnt[u + 1]++;
    cnt[v + 1]++;
  }
  for (int32_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  const int64_t arcs = cnt[n];
  std::vector<int32_t> tmp((size_t)arcs);
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  for (int64_t e = 0; e < m; ++e) {
    int32_t u = src[e], v = dst[e];
    if (u == v) continue;
    tmp[pos[u]++] = v;
    tmp[pos[v]++] = u;
  }
  std::vector<int64_t> keep((size_t)n + 1, 0);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t i = 0; i < n; ++i) {
    int32_t *b = tmp.data() + cnt[i], *e = tmp.data() + cnt[i + 1];
    std::sort(b, e);
    keep[i + 1] = std::unique(b, e) - b;
  }
  for (int32_t i = 0; i < n; ++i) keep[i + 1] += keep[i];
  if (keep[n] >= INT32_MAX) return false;
  out.n = n;
  out.nnz = keep[n];
  out.row_ptr.assign((size_t)n + 1, 0);
  out.col_idx.assign((size_t)keep[n], 0);
  for (int32_t i = 0; i <= n; ++i) out.row_ptr[i] = (int32_t)keep[i];
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t i = 0; i < n; ++i) {
    std::memcpy(out.col_idx.data() + keep[i], tmp.data() + cnt[i],
                sizeof(int32_t) * (size_t)(keep[i + 1] - keep[i]));
  }
  return true;
}

}  // namespace

extern "C" {

typedef struct efgen_csr {
  int32_t n;
  int64_t nnz;
  int32_t *row_ptr;
  int32_t *col_idx;
} efgen_csr;

static efgen_csr *export_csr(Csr &c) {
  efgen_csr *o = (efgen_csr *)std::malloc(sizeof(efgen_csr));
  if (!o) return nullptr;
  o->n = c.n;
  o->nnz = c.nnz;
  o->row_ptr = (int32_t *)std::malloc(sizeof(int32_t) * ((size_t)c.n + 1));
  o->col_idx = (int32_t *)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(c.nnz, 1));
  if (!o->row_ptr || !o->col_idx) {
    std::free(o->row_ptr);
    std::free(o->col_idx);
    std::free(o);
    return nullptr;
  }
  std::memcpy(o->row_ptr, c.row_ptr.data(), sizeof(int32_t) * ((size_t)c.n + 1));
  if (c.nnz) std::memcpy(o->col_idx, c.col_idx.data(), sizeof(int32_t) * (size_t)c.nnz);
  return o;
}

void efgen_free(efgen_csr *g) {
  if (!g) return;
  std::free(g->row_ptr);
  std::free(g->col_idx);
  std::free(g);
}

// CSR from an arbitrary edge list (symmetrised, deduplicated, self-loops dropped).
efgen_csr *efgen_from_edges(int32_t n, int64_t m, const int32_t *src, const int32_t *dst) {
  if (n < 0 || m < 0) return nullptr;
  std::vector<int32_t> s(src, src + m), d(dst, dst + m);
  for (int64_t e = 0; e < m; ++e)
    if (s[e] < 0 || s[e] >= n || d[e] < 0 || d[e] >= n) return nullptr;
  Csr c;
  if (!build_csr(n, s, d, c)) return nullptr;
  return export_csr(c);
}

// Erdos-Renyi G(n, p): every unordered pair independently with probability p.
// Geometric skipping over the pair sequence (Batagelj and Brandes, "Efficient
// generation of large random networks", Phys. Rev. E 71, 2005).
efgen_csr *efgen_er(int32_t n, double p, uint64_t seed) {
  if (n < 0 || !(p >= 0.0) || p > 1.0) return nullptr;
  std::vector<int32_t> s, d;
  if (n >= 2 && p > 0.0) {
    Rng rng(seed);
    if (p >= 1.0) {
      for (int32_t v = 1; v < n; ++v)
        for (int32_t w = 0; w < v; ++w) { s.push_back(v); d.push_back(w); }
    } else {
      const double lq = std::log(1.0 - p);
      int64_t v = 1, w = -1;
      while (v < n) {
        double r = rng.uniform();
        w = w + 1 + (int64_t)std::floor(std::log(1.0 - r) / lq);
        while (w >= v && v < n) { w -= v; v++; }
        if (v < n) { s.push_back((int32_t)v); d.push_back((int32_t)w); }
      }
    }
  }
  Csr c;
  if (!build_csr(n, s, d, c)) return nullptr;
  return export_csr(c);
}

// Barabasi-Albert: a star on m+1 nodes, then each new node attaches to m
// distinct earlier nodes chosen with probability proportional to degree
// (the repeated-endpoint list holds every node once per incident edge).
efgen_csr *efgen_ba(int32_t n, int32_t m, uint64_t seed) {
  if (m < 1 || n < m + 1) return nullptr;
  Rng rng(seed);
  std::vector<int32_t> s, d, rep;
  s.reserve((size_t)n * m);
  d.reserve((size_t)n * m);
  rep.reserve((size_t)2 * n * m);
  for (int32_t i = 1; i <= m; ++i) {
    s.push_back(0); d.push_back(i);
    rep.push_back(0); rep.push_back(i);
  }
  std::vector<int32_t> pick;
  for (int32_t t = m + 1; t < n; ++t) {
    pick.clear();
    while ((int32_t)pick.size() < m) {
      int32_t c = rep[rng.below(rep.size())];
      if (std::find(pick.begin(), pick.end(), c) == pick.end()) pick.push_back(c);
    }
    for (int32_t c : pick) {
      s.push_back(t); d.push_back(c);
      rep.push_back(t); rep.push_back(c);
    }
  }
  Csr c;
  if (!build_csr(n, s, d, c)) return nullptr;
  return export_csr(c);
}

// R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004): edge_factor * 2^scale
// draws; at each of the `scale` levels a quadrant is picked with probabilities
// a, b, c, d = 1-a-b-c (no noise). The result is symmetrised, self-loops and
// duplicates are dropped, and node ids are shuffled by a seeded random
// permutation (perm_seed = 0 keeps the raw ids). Every draw takes its random
// numbers from a counter-based hash, so the output does not depend on threads.
efgen_csr *efgen_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c,
                      uint64_t seed, uint64_t perm_seed) {
  if (scale < 1 || scale > 30 || edge_factor < 1) return nullptr;
  const double dsum = a + b + c;
  if (!(a >= 0 && b >= 0 && c >= 0) || dsum > 1.0 + 1e-12) return nullptr;
  const int64_t n = (int64_t)1 << scale;
  const int64_t m = (int64_t)edge_factor * n;
  std::vector<int32_t> s((size_t)m), d((size_t)m);
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    int64_t u = 0, v = 0;
    for (int32_t l = 0; l < scale; ++l) {
      double r = u01(hash2(seed, (uint64_t)e * 64u + (uint64_t)l));
      int bu, bv;
      if (r < a) { bu = 0; bv = 0; }
      else if (r < ab) { bu = 0; bv = 1; }
      else if (r < abc) { bu = 1; bv = 0; }
      else { bu = 1; bv = 1; }
      u = (u << 1) | bu;
      v = (v << 1) | bv;
    }
    s[e] = (int32_t)u;
    d[e] = (int32_t)v;
  }
  if (perm_seed != 0) {
    std::vector<int32_t> perm((size_t)n);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    Rng rng(perm_seed);
    for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[rng.below((uint64_t)i + 1)]);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) { s[e] = perm[s[e]]; d[e] = perm[d[e]]; }
  }
  Csr g;
  if (!build_csr((int32_t)n, s, d, g)) return nullptr;
  return export_csr(g);
}

// Watts-Strogatz: ring lattice where every node links to its k/2 nearest
// neighbours on each side; then each lattice edge (i, i+j) has its far end
// rewired with probability p to a uniform node, avoiding self-loops and
// duplicate edges (the edge is left in place when no valid target is found
// after n tries).
efgen_csr *efgen_ws(int32_t n, int32_t k, double p, uint64_t seed) {
  if (n < 3 || k < 2 || (k & 1) || k >= n || !(p >= 0.0) || p > 1.0) return nullptr;
  Rng rng(seed);
  // adjacency as small per-node lists (degrees stay near k)
  std::vector<std::vector<int32_t>> adj((size_t)n);
  for (int32_t i = 0; i < n; ++i) adj[i].reserve((size_t)k + 4);
  auto has = [&](int32_t u, int32_t w) {
    const auto &a = adj[u];
    return std::find(a.begin(), a.end(), w) != a.end();
  };
  auto drop = [&](int32_t u, int32_t w) {
    auto &a = adj[u];
    a.erase(std::find(a.begin(), a.end(), w));
  };
  std::vector<std::pair<int32_t, int32_t>> edges;
  edges.reserve((size_t)n * k / 2);
  for (int32_t j = 1; j <= k / 2; ++j)
    for (int32_t i = 0; i < n; ++i) {
      int32_t w = (int32_t)(((int64_t)i + j) % n);
      edges.emplace_back(i, w);
      adj[i].push_back(w);
      adj[w].push_back(i);
    }
  for (auto &ed : edges) {
    if (rng.uniform() < p) {
      const int32_t u = ed.first;
      for (int32_t tries = 0; tries < n; ++tries) {
        const int32_t w = (int32_t)rng.below((uint64_t)n);
        if (w == u || has(u, w)) continue;
        drop(u, ed.second);
        drop(ed.second, u);
        adj[u].push_back(w);
        adj[w].push_back(u);
        ed.second = w;
        break;
      }
    }
  }
  std::vector<int32_t> s, d;
  s.reserve(edges.size());
  d.reserve(edges.size());
  for (auto &ed : edges) { s.push_back(ed.first); d.push_back(ed.second); }
  Csr c;
  if (!build_csr(n, s, d, c)) return nullptr;
  return export_csr(c);
}

// Erased configuration model: i.i.d. degrees with P(k) proportional to
// k^-gamma on [kmin, kmax], kmax = min(n-1, floor(n^(1/(gamma-1)))); one
// degree is bumped if the stub total is odd; stubs are matched uniformly at
// random and the self-loops and multi-edges of the matching are erased.
efgen_csr *efgen_cm(int32_t n, double gamma, int32_t kmin, uint64_t seed) {
  if (n < 3 || !(gamma > 1.0) || kmin < 1) return nullptr;
  Rng rng(seed);
  int64_t kmax = (int64_t)std::floor(std::pow((double)n, 1.0 / (gamma - 1.0)));
  kmax = std::min<int64_t>(kmax, (int64_t)n - 1);
  if (kmax < kmin) kmax = kmin;
  std::vector<double> cdf((size_t)(kmax - kmin + 1));
  double acc = 0.0;
  for (int64_t k = kmin; k <= kmax; ++k) {
    acc += std::pow((double)k, -gamma);
    cdf[(size_t)(k - kmin)] = acc;
  }
  for (auto &x : cdf) x /= acc;
  std::vector<int32_t> deg((size_t)n);
  int64_t tot = 0;
  for (int32_t i = 0; i < n; ++i) {
    double r = rng.uniform();
    size_t j = (size_t)(std::lower_bound(cdf.begin(), cdf.end(), r) - cdf.begin());
    if (j >= cdf.size()) j = cdf.size() - 1;
    deg[i] = (int32_t)(kmin + (int64_t)j);
    tot += deg[i];
  }
  if (tot & 1) {
    deg[rng.below((uint64_t)n)] += 1;
    tot += 1;
  }
  std::vector<int32_t> stubs;
  stubs.reserve((size_t)tot);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t t = 0; t < deg[i]; ++t) stubs.push_back(i);
  for (int64_t i = (int64_t)stubs.size() - 1; i > 0; --i)
    std::swap(stubs[i], stubs[rng.below((uint64_t)i + 1)]);
  std::vector<int32_t> s, d;
  s.reserve((size_t)tot / 2);
  d.reserve((size_t)tot / 2);
  for (int64_t i = 0; i + 1 < (int64_t)stubs.size(); i += 2) {
    s.push_back(stubs[i]);
    d.push_back(stubs[i + 1]);
  }
  Csr c;
  if (!build_csr(n, s, d, c)) return nullptr;  // erases self-loops and multi-edges
  return export_csr(c);
}

}  // extern "C"
