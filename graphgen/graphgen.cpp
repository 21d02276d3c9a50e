// Seeded synthetic graph generators and the CSR builder they share.
//
// This module produces the inputs that both the GPU path and the oracle
// consume. It holds none of the matching method's arithmetic: it only draws
// edges, symmetrises them, drops self-loops, sorts and deduplicates each
// neighbour list, and lays the result out as CSR (Section II-A of the paper:
// an offsets array of |V|+1 entries and a neighbors array of |E| entries).
//
// Random numbers come from one counter-based generator: the SplitMix64 output
// function (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014) applied to a keyed counter, so every draw is a pure
// function of (seed, stream, counter), whatever the thread count.
//
// Models:
//   * Erdos-Renyi G(n, p) over unordered pairs, by geometric skipping over
//     each row (Batagelj and Brandes, "Efficient generation of large random
//     networks", Phys. Rev. E 71, 2005).
//   * R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004): each sample descends
//     `scale` levels of the adjacency matrix, picking a quadrant with
//     probabilities (a, b, c, 1-a-b-c), resolved to 1/65536; no per-level
//     noise. Vertex ids are then relabelled by a keyed bijection (a Feistel
//     network on the id bits with cycle walking), a seeded pseudo-random
//     permutation.
//   * The 4-neighbour 2D grid, row-major ids, neighbour lists in ascending id
//     order (up, left, right, down).
//   * Mixtures of the three, concatenated into one CSR with global int64
//     offsets, local int32 neighbour ids and a per-graph vertex offset table.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>
#include <omp.h>

namespace {

inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// Counter-based draw: a keyed SplitMix64 state advanced `ctr` steps.
inline uint64_t draw(uint64_t key, uint64_t ctr) {
  return sm64_mix(key + (ctr + 1) * 0x9e3779b97f4a7c15ULL);
}

inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return sm64_mix(sm64_mix(seed ^ 0x5851f42d4c957f2dULL) + stream * 0xd1342543de82ef95ULL);
}

// Uniform double in (0, 1].
inline double unit_open0(uint64_t r) {
  return ((r >> 11) + 1) * (1.0 / 9007199254740992.0);
}

// Keyed bijection on [0, 2^bits): a 4-round balanced Feistel network on
// 2*ceil(bits/2) bits, cycle-walked back into the domain when bits is odd.
// Round function: a keyed multiply-xorshift of the right half.
struct Relabel {
  int half;
  uint64_t hmask, dom;
  uint64_t key[4];
  Relabel(int bits, uint64_t seed) {
    half = (bits + 1) / 2;
    hmask = (half >= 64) ? ~0ULL : ((1ULL << half) - 1);
    dom = 1ULL << bits;
    for (int r = 0; r < 4; ++r) key[r] = stream_key(seed, 0x7e1abe1ULL + r) | 1ULL;
  }
  uint64_t once(uint64_t x) const {
    uint64_t l = x >> half, r = x & hmask;
    for (int k = 0; k < 4; ++k) {
      uint64_t f = (r ^ key[k]) * 0x9e3779b97f4a7c15ULL;
      f = ((f ^ (f >> 29)) * key[k]) >> 23;
      const uint64_t nl = r, nr = (l ^ f) & hmask;
      l = nl;
      r = nr;
    }
    return (l << half) | r;
  }
  uint64_t operator()(uint64_t x) const {
    uint64_t y = once(x);
    while (y >= dom) y = once(y);
    return y;
  }
};

int nthreads_or_default(int nt) {
  if (nt > 0) return nt;
  return omp_get_max_threads();
}

}  // namespace

struct gg_csr {
  int64_t n = 0;
  int64_t m = 0;
  int64_t* off = nullptr;   // n + 1
  int32_t* nbr = nullptr;   // m
  int32_t num_graphs = 0;   // mixtures only
  int64_t* vtx_off = nullptr;   // num_graphs + 1 (mixtures only)
  int32_t* kind = nullptr;      // per graph: 0 ER, 1 grid, 2 RMAT
};

namespace {

// Builds a symmetric CSR from a sampler of undirected pairs.
// `Sampler::for_each(i, emit)` calls emit(u, v) for every pair of chunk i.
// Self-loops are dropped, both orientations inserted, lists sorted and
// deduplicated. The result depends only on the multiset of pairs.
//
// One pass, no atomics: each thread takes a contiguous range of chunks and
// appends its (source, target) pairs to per-bucket chains of fixed-size
// blocks (a bucket is a range of consecutive sources; at most 1024 buckets, so
// every thread writes to few streams). Each bucket is then turned into CSR
// lists by a local counting sort over its chains, and every list is sorted and
// deduplicated.
namespace {
constexpr int64_t kBlockPairs = 4096;
struct PairBlock {
  uint64_t p[kBlockPairs];
  PairBlock* next;
  int64_t used;
};
}  // namespace

template <class Sampler>
gg_csr* build_symmetric(int64_t n, const Sampler& s, int64_t nchunks, int nt) {
  int shift = 0;
  while (((n - 1) >> shift) >= 1024) ++shift;  // at most 1024 buckets
  const int64_t nb = n > 0 ? ((n - 1) >> shift) + 1 : 1;
  // chains[t][b]: head of thread t's block chain for bucket b
  std::vector<PairBlock*> heads((size_t)nt * nb, nullptr);
  std::vector<int64_t> counts((size_t)nt * nb, 0);
  bool oom = false;
  auto chunk_lo = [&](int t) { return nchunks * t / nt; };
#pragma omp parallel num_threads(nt)
  {
    const int t = omp_get_thread_num();
    PairBlock** h = heads.data() + (size_t)t * nb;
    int64_t* c = counts.data() + (size_t)t * nb;
    auto push = [&](int64_t a, int64_t b) {
      const int64_t k = a >> shift;
      PairBlock* blk = h[k];
      if (!blk || blk->used == kBlockPairs) {
        PairBlock* nbk = static_cast<PairBlock*>(std::malloc(sizeof(PairBlock)));
        if (!nbk) {
          oom = true;
          return;
        }
        nbk->next = blk;
        nbk->used = 0;
        h[k] = blk = nbk;
      }
      blk->p[blk->used++] = ((uint64_t)a << 32) | (uint64_t)b;
      ++c[k];
    };
    for (int64_t i = chunk_lo(t); i < chunk_lo(t + 1); ++i)
      s.for_each(i, [&](int64_t u, int64_t v) {
        if (u == v) return;
        push(u, v);
        push(v, u);
      });
  }
  auto free_chains = [&]() {
    for (PairBlock* b : heads)
      while (b) {
        PairBlock* nx = b->next;
        std::free(b);
        b = nx;
      }
  };
  if (oom) {
    free_chains();
    throw std::bad_alloc();
  }
  std::vector<int64_t> bstart(nb + 1, 0);
  for (int64_t b = 0; b < nb; ++b) {
    int64_t tot = 0;
    for (int t = 0; t < nt; ++t) tot += counts[(size_t)t * nb + b];
    bstart[b + 1] = bstart[b] + tot;
  }
  const int64_t total = bstart[nb];
  int64_t* raw_off = static_cast<int64_t*>(std::malloc(sizeof(int64_t) * (n + 1)));
  int32_t* raw = static_cast<int32_t*>(std::malloc(sizeof(int32_t) * (total > 0 ? total : 1)));
  std::vector<uint32_t> deg(n > 0 ? n : 1, 0);
  if (!raw_off || !raw) {
    free_chains();
    throw std::bad_alloc();
  }
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t v0 = b << shift, v1 = std::min(n, (b + 1) << shift);
    for (int t = 0; t < nt; ++t)
      for (const PairBlock* blk = heads[(size_t)t * nb + b]; blk; blk = blk->next)
        for (int64_t q = 0; q < blk->used; ++q) ++deg[blk->p[q] >> 32];
    std::vector<int64_t> fill(v1 - v0);
    int64_t pos = bstart[b];
    for (int64_t v = v0; v < v1; ++v) {
      raw_off[v] = pos;
      fill[v - v0] = pos;
      pos += deg[v];
    }
    for (int t = 0; t < nt; ++t) {
      PairBlock* blk = heads[(size_t)t * nb + b];
      while (blk) {
        for (int64_t q = 0; q < blk->used; ++q) {
          const uint64_t pr = blk->p[q];
          raw[fill[(int64_t)(pr >> 32) - v0]++] = (int32_t)(uint32_t)pr;
        }
        PairBlock* nx = blk->next;
        std::free(blk);
        blk = nx;
      }
      heads[(size_t)t * nb + b] = nullptr;
    }
    for (int64_t v = v0; v < v1; ++v) {
      int32_t* lb = raw + raw_off[v];
      int32_t* le = lb + deg[v];
      std::sort(lb, le);
      deg[v] = (uint32_t)(std::unique(lb, le) - lb);
    }
  }
  gg_csr* g = new gg_csr();
  g->n = n;
  g->off = static_cast<int64_t*>(std::malloc(sizeof(int64_t) * (n + 1)));
  if (!g->off) throw std::bad_alloc();
  g->off[0] = 0;
  for (int64_t v = 0; v < n; ++v) g->off[v + 1] = g->off[v] + deg[v];
  g->m = g->off[n];
  g->nbr = static_cast<int32_t*>(std::malloc(sizeof(int32_t) * (g->m > 0 ? g->m : 1)));
  if (!g->nbr) throw std::bad_alloc();
#pragma omp parallel for schedule(dynamic, 4096) num_threads(nt)
  for (int64_t v = 0; v < n; ++v)
    std::memcpy(g->nbr + g->off[v], raw + raw_off[v], sizeof(int32_t) * deg[v]);
  std::free(raw);
  std::free(raw_off);
  return g;
}

// R-MAT sample k draws 16 bits per level from the counter-based generator
// (four levels per 64-bit draw), so quadrant probabilities are resolved to
// 1/65536.
struct RmatSampler {
  int scale;
  int64_t samples;
  int64_t chunk;
  uint32_t ta, tab, tabc;  // cumulative quadrant thresholds on 16-bit draws
  uint64_t key;
  bool permute;
  Relabel rel;
  RmatSampler(int scale_, int64_t samples_, double a, double b, double c, uint64_t seed, bool perm)
      : scale(scale_), samples(samples_), chunk(1 << 16), key(stream_key(seed, 0x12a7ULL)),
        permute(perm), rel(scale_, seed) {
    auto th = [](double p) {
      double x = std::floor(p * 65536.0 + 0.5);
      if (x < 0) x = 0;
      if (x > 65536.0) x = 65536.0;
      return static_cast<uint32_t>(x);
    };
    ta = th(a);
    tab = th(a + b);
    tabc = th(a + b + c);
  }
  int64_t nchunks() const { return (samples + chunk - 1) / chunk; }
  template <class F>
  void for_each(int64_t ci, F&& emit) const {
    int64_t lo = ci * chunk, hi = std::min(samples, lo + chunk);
    for (int64_t k = lo; k < hi; ++k) {
      uint64_t u = 0, v = 0;
      uint64_t ctr = static_cast<uint64_t>(k) * 8;
      uint64_t r = 0;
      for (int lvl = 0; lvl < scale; ++lvl) {
        if ((lvl & 3) == 0) r = draw(key, ctr++);
        const uint32_t q = static_cast<uint32_t>(r & 0xffffu);
        r >>= 16;
        // quadrant (0,0) below a, (0,1) below a+b, (1,0) below a+b+c, else (1,1)
        const uint64_t bu = q >= tab;
        const uint64_t bv = (q >= ta) & ((q < tab) | (q >= tabc));
        u = (u << 1) | bu;
        v = (v << 1) | bv;
      }
      if (permute) {
        u = rel(u);
        v = rel(v);
      }
      emit(static_cast<int64_t>(u), static_cast<int64_t>(v));
    }
  }
};

struct ErSampler {
  int64_t n;
  double p;
  uint64_t key;
  int64_t rows_per_chunk;
  ErSampler(int64_t n_, double p_, uint64_t seed) : n(n_), p(p_), key(stream_key(seed, 0xe7ULL)) {
    rows_per_chunk = 256;
  }
  int64_t nchunks() const { return (n + rows_per_chunk - 1) / rows_per_chunk; }
  template <class F>
  void for_each(int64_t ci, F&& emit) const {
    if (p <= 0.0) return;
    int64_t lo = ci * rows_per_chunk, hi = std::min(n, lo + rows_per_chunk);
    const double lq = std::log1p(-p);
    for (int64_t i = lo; i < hi; ++i) {
      uint64_t rk = sm64_mix(key ^ (static_cast<uint64_t>(i) * 0x9e3779b97f4a7c15ULL));
      uint64_t ctr = 0;
      int64_t j = i;
      while (true) {
        if (p >= 1.0) {
          j += 1;
        } else {
          double r = unit_open0(draw(rk, ctr++));
          double skip = std::floor(std::log(r) / lq);
          if (skip > static_cast<double>(n)) break;
          j += 1 + static_cast<int64_t>(skip);
        }
        if (j >= n) break;
        emit(i, j);
      }
    }
  }
};

gg_csr* make_grid(int64_t H, int64_t W, int nt) {
  gg_csr* g = new gg_csr();
  const int64_t n = H * W;
  g->n = n;
  g->off = static_cast<int64_t*>(std::malloc(sizeof(int64_t) * (n + 1)));
  if (!g->off) throw std::bad_alloc();
  g->off[0] = 0;
  for (int64_t id = 0; id < n; ++id) {
    int64_t r = id / W, c = id % W;
    int d = (r > 0) + (c > 0) + (c + 1 < W) + (r + 1 < H);
    g->off[id + 1] = g->off[id] + d;
  }
  g->m = g->off[n];
  g->nbr = static_cast<int32_t*>(std::malloc(sizeof(int32_t) * (g->m > 0 ? g->m : 1)));
  if (!g->nbr) throw std::bad_alloc();
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int64_t id = 0; id < n; ++id) {
    int64_t r = id / W, c = id % W;
    int32_t* o = g->nbr + g->off[id];
    if (r > 0) *o++ = static_cast<int32_t>(id - W);
    if (c > 0) *o++ = static_cast<int32_t>(id - 1);
    if (c + 1 < W) *o++ = static_cast<int32_t>(id + 1);
    if (r + 1 < H) *o++ = static_cast<int32_t>(id + W);
  }
  return g;
}

gg_csr* make_rmat(int scale, double ef, double a, double b, double c, uint64_t seed, int permute,
                  int nt) {
  const int64_t n = int64_t(1) << scale;
  const int64_t samples = static_cast<int64_t>(std::llround(ef * static_cast<double>(n)));
  RmatSampler s(scale, samples, a, b, c, seed, permute != 0);
  return build_symmetric(n, s, s.nchunks(), nt);
}

gg_csr* make_er(int64_t n, double avg_deg, uint64_t seed, int nt) {
  double p = (n > 1) ? avg_deg / static_cast<double>(n - 1) : 0.0;
  if (p > 1.0) p = 1.0;
  ErSampler s(n, p, seed);
  return build_symmetric(n, s, s.nchunks(), nt);
}

void free_csr(gg_csr* g) {
  if (!g) return;
  std::free(g->off);
  std::free(g->nbr);
  std::free(g->vtx_off);
  std::free(g->kind);
  delete g;
}

// One graph of the mixture family: kind 0 = ER with average degree `param`,
// kind 1 = grid with floor(sqrt(n)) rows and ceil(n/rows) columns,
// kind 2 = permuted R-MAT with scale `param` and edge factor 8.
gg_csr* make_member(int kind, int64_t n, double param, uint64_t seed, int nt) {
  if (kind == 0) return make_er(n, param, seed, nt);
  if (kind == 1) {
    int64_t r = static_cast<int64_t>(std::floor(std::sqrt(static_cast<double>(n))));
    if (r < 1) r = 1;
    while ((r + 1) * (r + 1) <= n) ++r;
    while (r * r > n) --r;
    int64_t cc = (n + r - 1) / r;
    return make_grid(r, cc, nt);
  }
  return make_rmat(static_cast<int>(param), 8.0, 0.57, 0.19, 0.19, seed, 1, nt);
}

}  // namespace

extern "C" {

gg_csr* gg_rmat(int32_t scale, double edge_factor, double a, double b, double c, uint64_t seed,
                int32_t permute, int32_t nthreads) {
  if (scale < 1 || scale > 30 || edge_factor < 0 || a < 0 || b < 0 || c < 0 || a + b + c > 1.0)
    return nullptr;
  try {
    return make_rmat(scale, edge_factor, a, b, c, seed, permute, nthreads_or_default(nthreads));
  } catch (...) {
    return nullptr;
  }
}

gg_csr* gg_er(int64_t n, double avg_deg, uint64_t seed, int32_t nthreads) {
  if (n < 0 || n > 2147483647LL || avg_deg < 0) return nullptr;
  try {
    return make_er(n, avg_deg, seed, nthreads_or_default(nthreads));
  } catch (...) {
    return nullptr;
  }
}

gg_csr* gg_grid(int64_t H, int64_t W, int32_t nthreads) {
  if (H < 0 || W < 0 || H * W > 2147483647LL) return nullptr;
  try {
    return make_grid(H, W, nthreads_or_default(nthreads));
  } catch (...) {
    return nullptr;
  }
}

gg_csr* gg_member(int32_t kind, int64_t n, double param, uint64_t seed, int32_t nthreads) {
  if (kind < 0 || kind > 2 || n < 1 || n > 2147483647LL) return nullptr;
  try {
    return make_member(kind, n, param, seed, nthreads_or_default(nthreads));
  } catch (...) {
    return nullptr;
  }
}

// Concatenates `num_graphs` members. kinds/ns/params/seeds describe each
// member (chosen by the caller). Offsets are global positions into the
// concatenated neighbour array; neighbour ids stay local to their graph.
gg_csr* gg_concat(int32_t num_graphs, const int32_t* kinds, const int64_t* ns, const double* params,
                  const uint64_t* seeds, int32_t nthreads) {
  if (num_graphs < 0) return nullptr;
  const int nt = nthreads_or_default(nthreads);
  std::vector<gg_csr*> parts(num_graphs, nullptr);
  bool fail = false;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int32_t gi = 0; gi < num_graphs; ++gi) {
    try {
      parts[gi] = make_member(kinds[gi], ns[gi], params[gi], seeds[gi], 1);
    } catch (...) {
      fail = true;
    }
  }
  if (fail) {
    for (auto* p : parts) free_csr(p);
    return nullptr;
  }
  gg_csr* g = new gg_csr();
  g->num_graphs = num_graphs;
  g->vtx_off = static_cast<int64_t*>(std::malloc(sizeof(int64_t) * (num_graphs + 1)));
  g->kind = static_cast<int32_t*>(std::malloc(sizeof(int32_t) * (num_graphs > 0 ? num_graphs : 1)));
  std::vector<int64_t> eoff(num_graphs + 1, 0);
  g->vtx_off[0] = 0;
  for (int32_t gi = 0; gi < num_graphs; ++gi) {
    g->vtx_off[gi + 1] = g->vtx_off[gi] + parts[gi]->n;
    eoff[gi + 1] = eoff[gi] + parts[gi]->m;
    g->kind[gi] = kinds[gi];
  }
  g->n = g->vtx_off[num_graphs];
  g->m = eoff[num_graphs];
  g->off = static_cast<int64_t*>(std::malloc(sizeof(int64_t) * (g->n + 1)));
  g->nbr = static_cast<int32_t*>(std::malloc(sizeof(int32_t) * (g->m > 0 ? g->m : 1)));
  if (!g->off || !g->nbr || !g->vtx_off || !g->kind) {
    for (auto* p : parts) free_csr(p);
    free_csr(g);
    return nullptr;
  }
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int32_t gi = 0; gi < num_graphs; ++gi) {
    const gg_csr* p = parts[gi];
    int64_t vb = g->vtx_off[gi];
    for (int64_t v = 0; v < p->n; ++v) g->off[vb + v] = eoff[gi] + p->off[v];
    std::memcpy(g->nbr + eoff[gi], p->nbr, sizeof(int32_t) * p->m);
  }
  g->off[g->n] = g->m;
  for (auto* p : parts) free_csr(p);
  return g;
}

int64_t gg_n(const gg_csr* g) { return g->n; }
int64_t gg_m(const gg_csr* g) { return g->m; }
int64_t* gg_offsets(gg_csr* g) { return g->off; }
int32_t* gg_neighbors(gg_csr* g) { return g->nbr; }
int32_t gg_num_graphs(const gg_csr* g) { return g->num_graphs; }
int64_t* gg_vtx_off(gg_csr* g) { return g->vtx_off; }
int32_t* gg_kinds(gg_csr* g) { return g->kind; }
void gg_free(gg_csr* g) { free_csr(g); }

// Exposes the counter-based generator so that the Python side draws mixture
// parameters from the same published definition.
uint64_t gg_draw(uint64_t seed, uint64_t stream, uint64_t ctr) {
  return draw(stream_key(seed, stream), ctr);
}

}  // extern "C"
