"""Pins of the oracle against what the paper and mathematics fix.

* the worked example of Fig. 1 / Fig. 6 (tests/golden/fig6_example.json);
* closed forms of SGMM on paths, stars, cliques, complete bipartite graphs,
  disjoint edges and row-major grids (derived next to each assertion);
* brute force: on every labelled graph with up to 5 vertices and on random
  graphs with 6-12 vertices, SGMM is the lexicographically first maximal
  matching under CSR edge rank, and the checker's verdict equals brute-force
  maximality for every matching;
* maximal-matching bounds nu/2 <= size <= nu against networkx's maximum
  matching;
* checker mutations: each violation class is detected with its exact count.
"""
import itertools
import json
import os
import random

import numpy as np
import pytest

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def pairs_of(mate):
    return sorted((int(a), int(b)) for a, b in enumerate(mate) if b > a)


# ---------------------------------------------------------------- worked example

def test_fig6_worked_example():
    fx = json.load(open(os.path.join(GOLDEN, "fig6_example.json")))
    g = graphgen.from_edges(fx["n"], fx["edges"])
    r = oracle.sgmm(g)
    assert pairs_of(r.mate) == [tuple(p) for p in fx["sgmm_pairs"]]
    assert r.touched == fx["sgmm_touched"]
    assert r.pairs == len(fx["sgmm_pairs"])
    mm = oracle.enumerate_matchings(g, maximal_only=True)
    got = sorted(pairs_of(m) for m in mm)
    want = sorted(sorted(tuple(p) for p in s) for s in fx["maximal_matchings"])
    assert got == want
    # the two-thread trace of Fig. 6 ends in one of the maximal matchings
    assert sorted(tuple(p) for p in fx["skipper_two_thread_result"]) in got
    assert oracle.check(g, r.mate).ok


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8, 9, 64, 65])
def test_path(k):
    # P_k with ids in path order: vertex 2i meets 2i+1 unmarked first, so
    # SGMM pairs (0,1), (2,3), ...: floor(k/2) pairs.
    g = graphgen.from_edges(k, [(i, i + 1) for i in range(k - 1)])
    r = oracle.sgmm(g)
    assert pairs_of(r.mate) == [(2 * i, 2 * i + 1) for i in range(k // 2)]
    assert oracle.check(g, r.mate).ok


@pytest.mark.parametrize("k", [1, 2, 7, 100])
def test_star(k):
    # K_{1,k}, centre 0: every maximal matching has one pair; SGMM takes (0,1).
    g = graphgen.from_edges(k + 1, [(0, j) for j in range(1, k + 1)])
    r = oracle.sgmm(g)
    assert pairs_of(r.mate) == [(0, 1)]
    assert r.touched == 1 + (k - 1)  # leaf j>1 reads its only neighbour 0
    if k <= 12:
        assert {len(pairs_of(m)) for m in oracle.enumerate_matchings(g)} == {1}


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 9, 10])
def test_clique(n):
    # K_n (triangle for n=3): floor(n/2) pairs in every maximal matching;
    # SGMM pairs (0,1), (2,3), ...
    g = graphgen.from_edges(n, list(itertools.combinations(range(n), 2)))
    r = oracle.sgmm(g)
    assert pairs_of(r.mate) == [(2 * i, 2 * i + 1) for i in range(n // 2)]
    assert {len(pairs_of(m)) for m in oracle.enumerate_matchings(g)} == {n // 2}


@pytest.mark.parametrize("a,b", [(1, 1), (2, 3), (3, 2), (4, 4), (5, 2), (2, 6)])
def test_complete_bipartite(a, b):
    # K_{a,b}, left 0..a-1, right a..a+b-1: left vertex i finds right a+i as
    # its first unmarked neighbour, so SGMM pairs (i, a+i), i < min(a, b);
    # every maximal matching has min(a, b) pairs.
    g = graphgen.from_edges(a + b, [(i, a + j) for i in range(a) for j in range(b)])
    r = oracle.sgmm(g)
    assert pairs_of(r.mate) == [(i, a + i) for i in range(min(a, b))]
    assert {len(pairs_of(m)) for m in oracle.enumerate_matchings(g)} == {min(a, b)}


def test_disjoint_edges_unique():
    # A union of disjoint K2's has exactly one maximal matching: all of it.
    k = 6
    g = graphgen.from_edges(2 * k, [(2 * i, 2 * i + 1) for i in range(k)])
    mm = oracle.enumerate_matchings(g)
    assert mm.shape[0] == 1
    np.testing.assert_array_equal(oracle.sgmm(g).mate, mm[0])


def test_empty_isolated_loops():
    g = graphgen.from_edges(0, np.zeros((0, 2)))
    assert oracle.sgmm(g).pairs == 0
    g = graphgen.from_edges(5, np.zeros((0, 2)))
    r = oracle.sgmm(g)
    assert (r.mate == -1).all() and r.touched == 0
    # self-loops only: never matched, and not counted as uncovered edges
    g = graphgen.from_edges(4, [(0, 0), (2, 2)], symmetric=False)
    r = oracle.sgmm(g)
    assert (r.mate == -1).all() and r.touched == 2
    assert oracle.check(g, r.mate).ok


@pytest.mark.parametrize("H,W", [(1, 2), (2, 2), (3, 4), (4, 6), (5, 8), (7, 10), (16, 16), (33, 64)])
def test_grid_closed_form(H, W):
    # Row-major H x W grid, W even, lists ascending (up, left, right, down).
    # Row 0: vertex 0 reads 1 and pairs with it; every later even column reads
    # its (marked) left neighbour, then its right one. A later row: column 0
    # reads up (marked), then right; every later even column reads up, left
    # (both marked), then right. All pairs are horizontal: H*W/2 pairs, and
    # 1 + 2(W/2-1) + (H-1)(2 + 3(W/2-1)) ids read.
    g = graphgen.grid(H, W)
    assert g.m == 4 * H * W - 2 * H - 2 * W
    r = oracle.sgmm(g)
    assert r.pairs == H * W // 2
    assert all(b == a + 1 and a % 2 == 0 for a, b in pairs_of(r.mate))
    assert r.touched == 1 + 2 * (W // 2 - 1) + (H - 1) * (2 + 3 * (W // 2 - 1))


def test_grid_16384_closed_form_values():
    # The benchmark-size grid, by the same closed forms.
    H = W = 16384
    assert 4 * H * W - 2 * H - 2 * W == 1_073_676_288
    assert H * W // 2 == 134_217_728
    assert 1 + 2 * (W // 2 - 1) + (H - 1) * (2 + 3 * (W // 2 - 1)) == 402_628_608


def test_sgmm_prefix():
    # x_end stops the outer loop: the state after the first x_end vertices.
    g = graphgen.er(500, 6, seed=3)
    full = oracle.sgmm(g)
    part = oracle.sgmm(g, x_end=250)
    assert part.pairs <= full.pairs
    # every pair found on the prefix is also a pair of the full run
    for a, b in pairs_of(part.mate):
        assert full.mate[a] == b and full.mate[b] == a
    assert oracle.sgmm(g, x_end=0).pairs == 0


# ---------------------------------------------------------------- brute force

def edge_ranks(csr):
    """rank of each undirected edge = position of its first CSR entry."""
    rank = {}
    pos = 0
    for x in range(csr.n):
        for i in range(int(csr.off[x]), int(csr.off[x + 1])):
            y = int(csr.nbr[i])
            if y != x:
                rank.setdefault((min(x, y), max(x, y)), pos)
            pos += 1
    return rank


def lex_first(csr, matchings):
    rank = edge_ranks(csr)
    best = None
    for m in matchings:
        key = sorted(rank[e] for e in pairs_of(m))
        if best is None or key < best[0]:
            best = (key, m)
    return best[1]


def maximal_by_definition(csr, mate):
    # Section II-B: every edge shares an endpoint with a selected edge.
    for x in range(csr.n):
        for i in range(int(csr.off[x]), int(csr.off[x + 1])):
            y = int(csr.nbr[i])
            if y != x and mate[x] == -1 and mate[y] == -1:
                return False
    return True


def brute_force_case(csr):
    mm = oracle.enumerate_matchings(csr, maximal_only=True)
    allm = oracle.enumerate_matchings(csr, maximal_only=False)
    r = oracle.sgmm(csr)
    # (i) SGMM is a maximal matching and is the lexicographically first one
    #     under CSR edge rank (greedy over edges in first-occurrence order)
    assert any((r.mate == m).all() for m in mm)
    np.testing.assert_array_equal(r.mate, lex_first(csr, mm))
    # (ii) checker verdict == maximality, for every matching
    maximal_set = {tuple(m) for m in mm}
    for m in allm:
        c = oracle.check(csr, m)
        assert c.out_of_range == c.self_mate == c.asymmetric == c.not_an_edge == 0
        is_max = tuple(m) in maximal_set
        assert is_max == maximal_by_definition(csr, m)
        assert (c.uncovered == 0) == is_max


def test_brute_force_all_graphs_up_to_5():
    count = 0
    for n in range(0, 6):
        pairs = list(itertools.combinations(range(n), 2))
        for bits in range(1 << len(pairs)):
            edges = [p for k, p in enumerate(pairs) if bits >> k & 1]
            g = graphgen.from_edges(n, edges if edges else np.zeros((0, 2)))
            brute_force_case(g)
            count += 1
    assert count == 1 + 1 + 2 + 8 + 64 + 1024


@pytest.mark.parametrize("seed", range(40))
def test_brute_force_random_small(seed):
    rng = random.Random(seed)
    n = rng.randint(6, 12)
    p = rng.choice([0.15, 0.3, 0.5, 0.8])
    edges = [e for e in itertools.combinations(range(n), 2) if rng.random() < p]
    # random stored order of each list, plus some loops and duplicates
    if edges and seed % 3 == 0:
        edges += [edges[0]]
    edges += [(v, v) for v in range(n) if rng.random() < 0.1]
    g = graphgen.from_edges(n, edges if edges else np.zeros((0, 2)), sort=(seed % 2 == 0),
                            dedup=(seed % 3 != 0))
    if seed % 2:
        # shuffle each list so SGMM's order is not the id order
        nbr = g.nbr.copy()
        for x in range(n):
            seg = nbr[g.off[x]:g.off[x + 1]]
            rng.shuffle(seg)
            nbr[g.off[x]:g.off[x + 1]] = seg
        g = graphgen.CSR(g.off, nbr)
    if len(oracle.enumerate_matchings(g, maximal_only=False)) > 200000:
        pytest.skip("too many matchings for the per-matching checker loop")
    brute_force_case(g)


def test_brute_force_non_symmetric():
    # Section V-C: an edge needs to appear in one endpoint's list only.
    rng = random.Random(7)
    for _ in range(30):
        n = rng.randint(2, 9)
        edges = [e for e in itertools.combinations(range(n), 2) if rng.random() < 0.4]
        edges = [(b, a) if rng.random() < 0.5 else (a, b) for a, b in edges]
        g = graphgen.from_edges(n, edges if edges else np.zeros((0, 2)), symmetric=False)
        brute_force_case(g)


@pytest.mark.parametrize("seed", range(6))
def test_size_bounds_against_maximum_matching(seed):
    nx = pytest.importorskip("networkx")
    g = graphgen.er(300 + 50 * seed, 3 + seed, seed=seed + 1)
    r = oracle.sgmm(g)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    for x in range(g.n):
        for y in g.nbr[g.off[x]:g.off[x + 1]]:
            G.add_edge(x, int(y))
    nu = len(nx.max_weight_matching(G, maxcardinality=True))
    # any maximal matching has at least half the pairs of a maximum one
    assert (nu + 1) // 2 <= r.pairs <= nu


# ---------------------------------------------------------------- checker mutations

def _valid_case(seed=5):
    g = graphgen.er(2000, 8, seed=seed)
    r = oracle.sgmm(g)
    assert oracle.check(g, r.mate).ok
    return g, r.mate.copy()


def _uncovered_by_definition(g, mate):
    src = np.repeat(np.arange(g.n), np.diff(g.off))
    dst = g.nbr.astype(np.int64)
    keep = src != dst
    return int(np.sum((mate[src[keep]] == -1) & (mate[dst[keep]] == -1)))


def test_checker_drop_pair():
    g, mate = _valid_case()
    a, b = pairs_of(mate)[3]
    mate[a] = mate[b] = -1
    c = oracle.check(g, mate)
    assert c.uncovered == _uncovered_by_definition(g, mate) and c.uncovered >= 2
    assert c.out_of_range == c.self_mate == c.asymmetric == c.not_an_edge == 0


def test_checker_out_of_range():
    g, mate = _valid_case()
    a, b = pairs_of(mate)[0]
    mate[a] = g.n  # a now claims a vertex that does not exist; b still claims a
    c = oracle.check(g, mate)
    assert c.out_of_range == 1 and c.asymmetric == 1
    mate[a] = -7
    assert oracle.check(g, mate).out_of_range == 1


def test_checker_self_mate():
    g, mate = _valid_case()
    a, b = pairs_of(mate)[1]
    mate[a] = a
    c = oracle.check(g, mate)
    assert c.self_mate == 1 and c.asymmetric == 1  # b -> a, but a -> a


def test_checker_shared_endpoint():
    g, mate = _valid_case()
    (a, b), (c_, d) = pairs_of(mate)[:2]
    mate[c_] = b  # two vertices now claim b; b claims a
    c = oracle.check(g, mate)
    assert c.asymmetric == 2  # c_ -> b (b -> a) and d -> c_ (c_ -> b)


def test_checker_not_an_edge():
    g = graphgen.from_edges(4, [(0, 1), (2, 3)])
    mate = np.array([2, 3, 0, 1], dtype=np.int32)  # symmetric, but 0-2 and 1-3 are not edges
    c = oracle.check(g, mate)
    assert c.not_an_edge == 4 and c.asymmetric == 0 and c.uncovered == 0
    mate = np.array([1, 0, 3, 2], dtype=np.int32)
    assert oracle.check(g, mate).ok


def test_checker_counts_every_uncovered_entry():
    g = graphgen.from_edges(3, [(0, 1), (1, 2), (0, 2)])
    c = oracle.check(g, np.full(3, -1, dtype=np.int32))
    assert c.uncovered == 6  # every directed entry of the triangle
    assert c.size == 0


def test_checker_bad_input_ids():
    g = graphgen.CSR(np.array([0, 1, 2], dtype=np.int64), np.array([1, 5], dtype=np.int32))
    c = oracle.check(g, np.array([1, 0], dtype=np.int32))
    assert c.bad_input == 1 and not c.ok


def test_checker_int32_offsets():
    g, mate = _valid_case(9)
    g32 = g.with_int32_offsets()
    assert oracle.check(g32, mate).ok
    np.testing.assert_array_equal(oracle.sgmm(g32).mate, oracle.sgmm(g).mate)


# ---------------------------------------------------------------- weighted greedy (EMS fixed point)

def test_splitmix64_published_sequence():
    # SplitMix64 from seed 1234567: the first outputs of the published reference
    # generator (state advanced by the golden gamma before each output)
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    state = 1234567
    got = []
    for _ in range(5):
        got.append(oracle.splitmix64(state))
        state = (state + 0x9E3779B97F4A7C15) % (1 << 64)
    assert got == want


def test_edge_weight_is_symmetric_and_seeded():
    for a, b in [(0, 1), (5, 3), (1000, 7), (2**31 - 2, 2**31 - 1)]:
        assert oracle.edge_weight(a, b, 9) == oracle.edge_weight(b, a, 9)
    assert oracle.edge_weight(0, 1, 1) != oracle.edge_weight(0, 1, 2)
    assert oracle.edge_weight(0, 1, 1) != oracle.edge_weight(0, 2, 1)
    # the published mix of the seed, xor the key, mixed again
    assert oracle.edge_weight(3, 5, 7) == oracle.splitmix64(oracle.splitmix64(7) ^ ((3 << 32) | 5))


def weight_rank(csr, seed):
    ws = {}
    for x in range(csr.n):
        for i in range(int(csr.off[x]), int(csr.off[x + 1])):
            y = int(csr.nbr[i])
            if y != x:
                e = (min(x, y), max(x, y))
                ws[e] = oracle.edge_weight(x, y, seed)
    order = sorted(ws, key=lambda e: (-ws[e], e))
    return {e: r for r, e in enumerate(order)}


def lex_first_by(rank, matchings):
    best = None
    for m in matchings:
        key = sorted(rank[e] for e in pairs_of(m))
        if best is None or key < best[0]:
            best = (key, m)
    return best[1]


@pytest.mark.parametrize("seed", range(25))
def test_greedy_weighted_is_lex_first_under_weight_order(seed):
    rng = random.Random(seed)
    n = rng.randint(1, 10)
    edges = [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < 0.45]
    if rng.random() < 0.3 and n > 1:
        edges.append((0, 0))  # loops are never selected
    g = graphgen.from_edges(n, edges or np.zeros((0, 2)), drop_loops=False)
    mate, pairs = oracle.greedy_weighted(g, seed)
    assert oracle.check(g, mate).ok
    mm = oracle.enumerate_matchings(g, maximal_only=True)
    np.testing.assert_array_equal(mate, lex_first_by(weight_rank(g, seed), mm))
    assert pairs == int((mate >= 0).sum()) // 2


def test_greedy_weighted_closed_forms():
    # every maximal matching of K_n has floor(n/2) pairs, of a star 1, of a
    # disjoint K2 union all of them (the unique one)
    for n in (2, 3, 8, 11):
        k = graphgen.from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])
        assert oracle.greedy_weighted(k, 3)[1] == n // 2
    star = graphgen.from_edges(50, [(0, j) for j in range(1, 50)])
    mate, pairs = oracle.greedy_weighted(star, 4)
    assert pairs == 1 and mate[0] > 0
    # the star's heaviest edge is the one taken
    ws = [oracle.edge_weight(0, j, 4) for j in range(1, 50)]
    assert mate[0] == 1 + int(np.argmax(ws))
    k2 = graphgen.from_edges(10, [(0, 1), (2, 3), (4, 5), (6, 7), (8, 9)])
    np.testing.assert_array_equal(oracle.greedy_weighted(k2, 1)[0], np.arange(10) ^ 1)


def test_greedy_weighted_orientation_free():
    # the result depends on the undirected edge set only: list order,
    # duplicates and one-sided entries do not change it
    g = graphgen.er(300, 5, seed=2)
    e = [(x, int(y)) for x in range(g.n) for y in g.nbr[g.off[x]:g.off[x + 1]] if x < y]
    one_sided = graphgen.from_edges(g.n, e, symmetric=False)
    shuffled = graphgen.from_edges(g.n, list(reversed(e)) + e[:50], symmetric=True, dedup=False,
                                   sort=False)
    a = oracle.greedy_weighted(g, 8)[0]
    np.testing.assert_array_equal(a, oracle.greedy_weighted(one_sided, 8)[0])
    np.testing.assert_array_equal(a, oracle.greedy_weighted(shuffled, 8)[0])
