/*
 * Oracle for maximal matching (MM): test infrastructure only.
 *
 * Only the test suite, the smoke entry point and the benchmark's CPU-baseline
 * leg may load this library. The GPU product path never links, imports or
 * calls it; the two share no code, header or table.
 *
 * Everything here is plain, single-threaded C written from the paper's
 * definitions, except that the checker spreads its O(n + m) counting loops
 * over OpenMP threads with sum reductions (each element is still checked by
 * the same obvious test).
 *
 *   oracle_sgmm     Sequential Greedy MM (Section II-B): visit vertices in
 *                   id order, skip a vertex that is already marked, scan its
 *                   neighbours in stored order and pair it with the first
 *                   unmarked one, then stop scanning that vertex. Self-loops
 *                   are never selected (Algorithm 1 skips them; Section II-B
 *                   is silent, and a loop cannot be a matching edge).
 *   oracle_check    The MM validity test of Section II-B, applied to a mate
 *                   array: (a) every edge has an endpoint covered by the
 *                   output, (b) no two output edges share an endpoint; plus
 *                   the well-formedness conditions a mate array must meet.
 *                   Violations are counted, never short-circuited.
 *   oracle_enumerate  Brute force over all matchings of a graph with at most
 *                   20 vertices, optionally keeping only the maximal ones.
 *   oracle_greedy_weighted  The matching that iterated Endpoints Mutual
 *                   Selection (Section II-C) reaches when every vertex selects
 *                   its heaviest free edge under fixed pseudo-random edge
 *                   weights: an edge selected by both ends is always the
 *                   heaviest free edge at both, so the process ends in the
 *                   greedy matching over edges in descending weight order.
 *                   This is that greedy matching, computed directly: sort the
 *                   undirected edges, then take each whose ends are free.
 *   oracle_edge_weight  The edge weight used by it: SplitMix64 (Steele, Lea
 *                   and Flood, OOPSLA 2014) of the seed, xor the edge key
 *                   (min << 32 | max), passed through SplitMix64 again.
 *
 * Graph format (Section II-A): CSR offsets (n+1 entries, int32 or int64) and
 * neighbours (int32). A non-symmetric CSR is read as the undirected union of
 * its entries (Section V-C, input format).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline int64_t off_at(const void *off, int off64, int64_t i) {
  return off64 ? ((const int64_t *)off)[i] : (int64_t)((const int32_t *)off)[i];
}

/*
 * Sequential Greedy MM over the sources 0 .. x_end-1 (x_end = n runs the whole
 * algorithm; a smaller x_end stops the outer loop early, which is the state
 * SGMM reaches after that many vertices). mt receives the mate of every
 * vertex, -1 if unmatched. *touched receives the number of neighbour ids read.
 * Returns the number of matched pairs.
 */
int64_t oracle_sgmm(int64_t n, const void *off, int32_t off64, const int32_t *nbr, int32_t *mt,
                    int64_t x_end, int64_t *touched) {
  int64_t pairs = 0, t = 0;
  for (int64_t v = 0; v < n; ++v) mt[v] = -1;
  if (x_end > n) x_end = n;
  for (int64_t x = 0; x < x_end; ++x) {
    if (mt[x] != -1) continue; /* x is already marked: its list is skipped */
    const int64_t b = off_at(off, off64, x), e = off_at(off, off64, x + 1);
    for (int64_t i = b; i < e; ++i) {
      const int32_t y = nbr[i];
      ++t;
      if (y == x) continue;
      if (mt[y] == -1) {
        mt[x] = y;
        mt[y] = (int32_t)x;
        ++pairs;
        break; /* x is now marked: the rest of N_x need not be read */
      }
    }
  }
  if (touched) *touched = t;
  return pairs;
}

/* 1 if y appears in N_x. */
static int has_entry(const void *off, int off64, const int32_t *nbr, int64_t x, int64_t y) {
  const int64_t b = off_at(off, off64, x), e = off_at(off, off64, x + 1);
  for (int64_t i = b; i < e; ++i)
    if (nbr[i] == y) return 1;
  return 0;
}

/*
 * Exact checker. out[0..7]:
 *   0  V1 mate out of range (mt[x] < -1 or mt[x] >= n)
 *   1  V2 self-mate (mt[x] == x)
 *   2  V3 asymmetric mate (mt[x] = y >= 0 but mt[y] != x); a vertex claimed by
 *      two others always shows up here
 *   3  V4 mate is not an edge (y not in N_x and x not in N_y)
 *   4  V5 uncovered edge: a CSR entry (x, y), x != y, with both ends unmatched
 *   5  size: number of vertices with mt >= 0, halved (rounded down)
 *   6  CSR entries whose neighbour id is out of range (input error)
 *   7  number of vertices with mt >= 0
 * The output passes iff out[0..4] are all zero (and out[6] is zero).
 */
void oracle_check(int64_t n, const void *off, int32_t off64, const int32_t *nbr,
                  const int32_t *mt, int64_t *out) {
  int64_t v1 = 0, v2 = 0, v3 = 0, v4 = 0, v5 = 0, matched = 0, bad_in = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : v1, v2, v3, v4, matched)
  for (int64_t x = 0; x < n; ++x) {
    const int64_t y = mt[x];
    if (y < -1 || y >= n) {
      ++v1;
      continue;
    }
    if (y == -1) continue;
    ++matched;
    if (y == x) {
      ++v2;
      continue;
    }
    if ((int64_t)mt[y] != x) ++v3;
    if (!has_entry(off, off64, nbr, x, y) && !has_entry(off, off64, nbr, y, x)) ++v4;
  }
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : v5, bad_in)
  for (int64_t x = 0; x < n; ++x) {
    const int64_t b = off_at(off, off64, x), e = off_at(off, off64, x + 1);
    for (int64_t i = b; i < e; ++i) {
      const int64_t y = nbr[i];
      if (y < 0 || y >= n) {
        ++bad_in;
        continue;
      }
      if (y == x) continue;
      if (mt[x] == -1 && mt[y] == -1) ++v5;
    }
  }
  out[0] = v1;
  out[1] = v2;
  out[2] = v3;
  out[3] = v4;
  out[4] = v5;
  out[5] = matched / 2;
  out[6] = bad_in;
  out[7] = matched;
}

/* ---- weighted greedy (the fixed point of iterated mutual selection) ---- */

/* One SplitMix64 output for state x: the state advanced by the golden gamma,
   then the published mixing function. */
static uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t oracle_splitmix64(uint64_t x) { return splitmix64(x); }

uint64_t oracle_edge_weight(int64_t a, int64_t b, uint64_t seed) {
  const uint64_t u = (uint64_t)(a < b ? a : b), v = (uint64_t)(a < b ? b : a);
  return splitmix64(splitmix64(seed) ^ ((u << 32) | v));
}

typedef struct {
  uint64_t w, key;
} wedge;

/* heavier first; equal weights: smaller key first */
static int wedge_cmp(const void *pa, const void *pb) {
  const wedge *a = (const wedge *)pa, *b = (const wedge *)pb;
  if (a->w != b->w) return a->w > b->w ? -1 : 1;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  return 0;
}

/* mt receives the mate of every vertex (-1: unmatched); returns the number
   of pairs, or -1 if memory runs out. Entries are read as undirected edges. */
int64_t oracle_greedy_weighted(int64_t n, const void *off, int32_t off64, const int32_t *nbr,
                               uint64_t seed, int32_t *mt) {
  const int64_t m = off_at(off, off64, n);
  wedge *e = (wedge *)malloc(sizeof(wedge) * (size_t)(m > 0 ? m : 1));
  if (!e) return -1;
  int64_t k = 0;
  for (int64_t x = 0; x < n; ++x)
    for (int64_t i = off_at(off, off64, x); i < off_at(off, off64, x + 1); ++i) {
      const int64_t y = nbr[i];
      if (y == x) continue;
      const uint64_t u = (uint64_t)(x < y ? x : y), v = (uint64_t)(x < y ? y : x);
      e[k].key = (u << 32) | v;
      e[k].w = oracle_edge_weight(x, y, seed);
      ++k;
    }
  qsort(e, (size_t)k, sizeof(wedge), wedge_cmp); /* both orientations sort together */
  for (int64_t v = 0; v < n; ++v) mt[v] = -1;
  int64_t pairs = 0;
  for (int64_t j = 0; j < k; ++j) {
    const int64_t u = (int64_t)(e[j].key >> 32), v = (int64_t)(e[j].key & 0xffffffffu);
    if (mt[u] == -1 && mt[v] == -1) {
      mt[u] = (int32_t)v;
      mt[v] = (int32_t)u;
      ++pairs;
    }
  }
  free(e);
  return pairs;
}

/* ---- brute-force enumeration (n <= 20) ---- */

typedef struct {
  int n;
  uint32_t adj[20]; /* undirected union of CSR entries, loops removed */
  int32_t mate[20];
  int maximal_only;
  int32_t *out;
  int64_t cap;
  int64_t count;
} enum_ctx;

static void enum_rec(enum_ctx *c, int v) {
  while (v < c->n && c->mate[v] != -2) ++v; /* -2 marks "undecided" */
  if (v == c->n) {
    /* leaf: every vertex decided; -3 marks "left unmatched" */
    if (c->maximal_only) {
      for (int a = 0; a < c->n; ++a) {
        if (c->mate[a] >= 0) continue;
        for (int b = a + 1; b < c->n; ++b)
          if (((c->adj[a] >> b) & 1u) && c->mate[b] < 0) return; /* uncovered edge */
      }
    }
    if (c->out && c->count < c->cap) {
      int32_t *o = c->out + c->count * c->n;
      for (int a = 0; a < c->n; ++a) o[a] = c->mate[a] >= 0 ? c->mate[a] : -1;
    }
    ++c->count;
    return;
  }
  c->mate[v] = -3;
  enum_rec(c, v + 1);
  for (int w = v + 1; w < c->n; ++w) {
    if (((c->adj[v] >> w) & 1u) && c->mate[w] == -2) {
      c->mate[v] = w;
      c->mate[w] = v;
      enum_rec(c, v + 1);
      c->mate[w] = -2;
    }
  }
  c->mate[v] = -2;
}

/*
 * Enumerates every matching (maximal_only = 0) or every maximal matching
 * (maximal_only = 1) of the undirected union of the CSR entries. Up to `cap`
 * of them are written to out as mate arrays of n entries each. Returns the
 * total count, or -1 if n is out of range or an id is invalid.
 */
int64_t oracle_enumerate(int64_t n, const void *off, int32_t off64, const int32_t *nbr,
                         int32_t maximal_only, int32_t *out, int64_t cap) {
  if (n < 0 || n > 20) return -1;
  enum_ctx c;
  memset(&c, 0, sizeof(c));
  c.n = (int)n;
  c.maximal_only = maximal_only;
  c.out = out;
  c.cap = cap;
  for (int64_t x = 0; x < n; ++x) {
    const int64_t b = off_at(off, off64, x), e = off_at(off, off64, x + 1);
    for (int64_t i = b; i < e; ++i) {
      const int32_t y = nbr[i];
      if (y < 0 || y >= n) return -1;
      if (y == x) continue;
      c.adj[x] |= 1u << y;
      c.adj[y] |= 1u << x;
    }
  }
  for (int a = 0; a < c.n; ++a) c.mate[a] = -2;
  enum_rec(&c, 0);
  return c.count;
}
