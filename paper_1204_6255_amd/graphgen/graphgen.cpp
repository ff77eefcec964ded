// Seeded synthetic web-like digraphs, and the graph statistics of the paper's
// Table 1 (L, D, E, O, max_in, max_out; definitions in Section 2.4).
//
// This module only produces inputs. It holds none of the D-iteration
// arithmetic and is shared by the CPU oracle tests and the GPU library tests.
//
// Generator recipe (web-graph stand-in; the paper's uk-2007-05 and
// gr0.California datasets are not available):
//   * node i is dangling (out-degree 0) with probability p_dangling;
//   * otherwise it draws k ~ P(k) proportional to k^-alpha on [1, kmax]
//     (inverse CDF on the exact pmf);
//   * each of the k links goes, with probability p_local, to i + o with o
//     uniform in [-radius, radius] \ {0} (redrawn until the target lies in
//     [0, n)), else to pi(r) where r ~ Zipf(1) on {1..n} and pi is a random
//     permutation of the ids drawn once per graph;
//   * with p_forward > 0, a local link points forward (o > 0) with
//     probability p_forward (dropped for the last node): mostly-forward
//     graphs where most nodes lie on no cycle, like the paper's Dataset 2
//     (E/N 0.91). p_forward = 0 draws no extra number, so such graphs are
//     the same as without the option;
//   * self-loops and duplicate links are dropped; links come out sorted by
//     (origin, destination), the input format of Section 2.1.
//
// Random numbers: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) seeds
// xoshiro256** (Blackman and Vigna, 2018). Every node has its own stream
// derived from (seed, node id), so the output does not depend on the number
// of threads.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

namespace {

inline uint64_t splitmix64_next(uint64_t& x) {
  uint64_t z = (x += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

struct Xoshiro256ss {
  uint64_t s[4];
  explicit Xoshiro256ss(uint64_t seed) {
    uint64_t sm = seed;
    for (int i = 0; i < 4; ++i) s[i] = splitmix64_next(sm);
  }
  uint64_t next() {
    const uint64_t result = rotl(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return result;
  }
  // uniform in [0, 1) with 53 random bits
  double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }
  // uniform integer in [0, k) by multiply-shift (Lemire); bias < k / 2^64
  uint64_t below(uint64_t k) {
    return (uint64_t)(((unsigned __int128)next() * k) >> 64);
  }
};

// Per-node stream: mix the graph seed and the node id through SplitMix64.
inline uint64_t node_stream_seed(uint64_t seed, int64_t node) {
  uint64_t x = seed ^ 0x5851f42d4c957f2dULL;
  uint64_t a = splitmix64_next(x);
  uint64_t y = a ^ ((uint64_t)node * 0xd1342543de82ef95ULL);
  return splitmix64_next(y);
}

constexpr double kEulerGamma = 0.57721566490153286060651209;

// Harmonic numbers H(r) = sum_{q=1..r} 1/q: exact table below 256, the
// asymptotic expansion ln r + gamma + 1/(2r) - 1/(12 r^2) + 1/(120 r^4)
// above (truncation error below 1/(252 r^6) < 1e-16 there).
struct Harmonic {
  double table[256];
  Harmonic() {
    table[0] = 0.0;
    for (int r = 1; r < 256; ++r) table[r] = table[r - 1] + 1.0 / r;
  }
  double operator()(int64_t r) const {
    if (r < 256) return table[r];
    const double x = (double)r;
    const double x2 = x * x;
    return std::log(x) + kEulerGamma + 0.5 / x - 1.0 / (12.0 * x2) +
           1.0 / (120.0 * x2 * x2);
  }
};

// Smallest r in [1, n] with H(r) >= target (inverse CDF of Zipf(1) on 1..n).
int64_t zipf1_inverse(const Harmonic& H, int64_t n, double target) {
  int64_t r;
  if (target <= H.table[255 < n ? 255 : n]) {
    r = 1;
    const int64_t hi = n < 255 ? n : 255;
    while (r < hi && H.table[r] < target) ++r;
    return r;
  }
  double guess = std::exp(target - kEulerGamma);
  if (!(guess >= 1.0)) guess = 1.0;
  if (guess > (double)n) guess = (double)n;
  r = (int64_t)guess;
  if (r < 1) r = 1;
  while (r < n && H(r) < target) ++r;
  while (r > 1 && H(r - 1) >= target) --r;
  return r;
}

}  // namespace

extern "C" {

typedef struct dg_params {
  int64_t n;          // number of nodes
  uint64_t seed;      // graph seed
  double alpha;       // out-degree power-law exponent
  int32_t kmax;       // out-degree upper bound (lower bound is 1)
  int32_t radius;     // local-link half width
  double p_dangling;  // probability that a node has no out-links
  double p_local;     // probability that a link is local
  double p_forward;   // probability that a local link points forward
} dg_params;

typedef struct dg_result {
  int64_t n;
  std::vector<int32_t> src;
  std::vector<int32_t> dst;
} dg_result;

typedef struct dg_stats {
  int64_t n;        // N
  int64_t L;        // links (non-null entries of P)
  int64_t D;        // dangling nodes (out-degree 0)
  int64_t zero_in;  // nodes with in-degree 0
  int64_t E;        // recursive zero in-degree nodes (Section 2.4)
  int64_t O;        // nodes with a self-loop
  int64_t max_in;   // maximum in-degree
  int64_t max_out;  // maximum out-degree
} dg_stats;

// Returns 0 on success, -1 on invalid parameters, -5 on allocation failure.
int dg_generate(const dg_params* p, dg_result** out) {
  if (!p || !out) return -1;
  *out = nullptr;
  const int64_t n = p->n;
  if (n < 0 || n > 2147483647LL || p->kmax < 1 || p->radius < 1 ||
      !(p->alpha > 0.0) || !(p->p_dangling >= 0.0 && p->p_dangling <= 1.0) ||
      !(p->p_local >= 0.0 && p->p_local <= 1.0) ||
      !(p->p_forward >= 0.0 && p->p_forward <= 1.0))
    return -1;
  dg_result* res = new (std::nothrow) dg_result;
  if (!res) return -5;
  res->n = n;
  if (n < 2) {  // a single node can only link to itself: no links survive
    *out = res;
    return 0;
  }
  try {
    // out-degree CDF on the exact pmf
    std::vector<double> cdf((size_t)p->kmax + 1, 0.0);
    for (int k = 1; k <= p->kmax; ++k)
      cdf[k] = cdf[k - 1] + std::pow((double)k, -p->alpha);
    const double cdf_total = cdf[p->kmax];

    // random permutation of ids for the Zipf ranks (Fisher-Yates)
    std::vector<int32_t> perm((size_t)n);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    {
      Xoshiro256ss g(node_stream_seed(p->seed, -1));
      for (int64_t i = n - 1; i > 0; --i) {
        const int64_t j = (int64_t)g.below((uint64_t)(i + 1));
        std::swap(perm[i], perm[j]);
      }
    }
    const Harmonic H;
    const double Hn = H(n);

    const int64_t chunk = 1 << 16;
    const int64_t nchunks = (n + chunk - 1) / chunk;
    std::vector<std::vector<int32_t>> cdst((size_t)nchunks);
    std::vector<int32_t> deg((size_t)n, 0);

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < nchunks; ++c) {
      std::vector<int32_t>& buf = cdst[c];
      std::vector<int32_t> tmp;
      const int64_t i0 = c * chunk, i1 = std::min(n, i0 + chunk);
      for (int64_t i = i0; i < i1; ++i) {
        Xoshiro256ss g(node_stream_seed(p->seed, i));
        if (g.uniform() < p->p_dangling) continue;
        const double u = g.uniform() * cdf_total;
        int k = (int)(std::lower_bound(cdf.begin() + 1, cdf.end(), u) - cdf.begin());
        if (k > p->kmax) k = p->kmax;
        tmp.clear();
        for (int q = 0; q < k; ++q) {
          int64_t j;
          if (g.uniform() < p->p_local) {
            do {
              const int64_t o = (int64_t)g.below(2 * (uint64_t)p->radius);
              int64_t off = o < p->radius ? o - p->radius : o - p->radius + 1;
              // a forward link from the last node has no target: it is
              // dropped (as a self-loop would be)
              if (p->p_forward > 0.0 && g.uniform() < p->p_forward)
                off = i + 1 < n ? (off < 0 ? -off : off) : 0;
              j = i + off;
            } while (j < 0 || j >= n);
          } else {
            const int64_t r = zipf1_inverse(H, n, g.uniform() * Hn);
            j = perm[r - 1];
          }
          if (j != i) tmp.push_back((int32_t)j);
        }
        std::sort(tmp.begin(), tmp.end());
        tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
        deg[i] = (int32_t)tmp.size();
        buf.insert(buf.end(), tmp.begin(), tmp.end());
      }
    }
    int64_t m = 0;
    std::vector<int64_t> coff((size_t)nchunks + 1, 0);
    for (int64_t c = 0; c < nchunks; ++c) coff[c + 1] = coff[c] + (int64_t)cdst[c].size();
    m = coff[nchunks];
    res->src.resize((size_t)m);
    res->dst.resize((size_t)m);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < nchunks; ++c) {
      int64_t pos = coff[c];
      std::memcpy(res->dst.data() + pos, cdst[c].data(), cdst[c].size() * sizeof(int32_t));
      const int64_t i0 = c * chunk, i1 = std::min(n, i0 + chunk);
      for (int64_t i = i0; i < i1; ++i)
        for (int32_t q = 0; q < deg[i]; ++q) res->src[pos++] = (int32_t)i;
      std::vector<int32_t>().swap(cdst[c]);
    }
  } catch (const std::bad_alloc&) {
    delete res;
    return -5;
  }
  *out = res;
  return 0;
}

int64_t dg_num_edges(const dg_result* r) { return r ? (int64_t)r->src.size() : -1; }

void dg_copy_edges(const dg_result* r, int32_t* src, int32_t* dst) {
  if (!r) return;
  if (src) std::memcpy(src, r->src.data(), r->src.size() * sizeof(int32_t));
  if (dst) std::memcpy(dst, r->dst.data(), r->dst.size() * sizeof(int32_t));
}

void dg_free(dg_result* r) { delete r; }

// Table-1 statistics of an arbitrary link list (ids in [0, n); no ordering
// or uniqueness is assumed, every listed link counts). Returns 0, or -1 on
// out-of-range ids, -5 on allocation failure.
int dg_graph_stats(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                   dg_stats* st) {
  if (!st || n < 0 || m < 0 || (m > 0 && (!src || !dst))) return -1;
  try {
    std::vector<int64_t> outd((size_t)n, 0), ind((size_t)n, 0);
    std::vector<uint8_t> loop((size_t)n, 0);
    for (int64_t e = 0; e < m; ++e) {
      const int64_t a = src[e], b = dst[e];
      if (a < 0 || a >= n || b < 0 || b >= n) return -1;
      ++outd[a];
      ++ind[b];
      if (a == b) loop[a] = 1;
    }
    dg_stats s{};
    s.n = n;
    s.L = m;
    for (int64_t i = 0; i < n; ++i) {
      s.D += outd[i] == 0;
      s.zero_in += ind[i] == 0;
      s.O += loop[i];
      s.max_in = std::max(s.max_in, ind[i]);
      s.max_out = std::max(s.max_out, outd[i]);
    }
    // E: least set closed under "every in-link comes from the set", found by
    // peeling nodes whose remaining in-degree reaches zero.
    std::vector<int64_t> ptr((size_t)n + 1, 0);
    for (int64_t i = 0; i < n; ++i) ptr[i + 1] = ptr[i] + outd[i];
    std::vector<int32_t> adj((size_t)m);
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t e = 0; e < m; ++e) adj[fill[src[e]]++] = dst[e];
    std::vector<int64_t> rem(ind);
    std::vector<int32_t> queue;
    queue.reserve((size_t)n);
    for (int64_t i = 0; i < n; ++i)
      if (rem[i] == 0) queue.push_back((int32_t)i);
    for (size_t h = 0; h < queue.size(); ++h) {
      const int32_t u = queue[h];
      for (int64_t q = ptr[u]; q < ptr[u + 1]; ++q) {
        const int32_t v = adj[q];
        if (--rem[v] == 0) queue.push_back(v);
      }
    }
    s.E = (int64_t)queue.size();
    *st = s;
  } catch (const std::bad_alloc&) {
    return -5;
  }
  return 0;
}

}  // extern "C"
