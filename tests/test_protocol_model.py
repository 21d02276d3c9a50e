"""The reservation protocol under every schedule, in a CPU model of the
sweep's lanes (tests/model/protocol_model.c; test infrastructure, no code
shared with the library).

Section V-A argues that the JIT protocol of Algorithm 1 is safe and ends;
the library runs it in forms the argument does not cover: lanes of a
wavefront advance together and poll instead of spinning, every memory
operation of a trip is in flight until the wavefront's next trip, cached
reads may be stale, and the options take v in two phases, give u back while
waiting for v (wait_release), keep states in packed words whose CAS must be
retried when another field changes, write unmatched outputs lazily, or
examine each edge only from its lower endpoint (upper_only), or read the
states of a step's candidates one at a time (probe_first). The model runs
the lanes' state machine with the memory operations applied in an order an
adversary picks. Pins:

* exhaustive: on every graph of up to 4 vertices (two-wavefront placements
  of the packed layouts: the sparser ones), every state reachable under any
  schedule can still reach the end of the sweep (no deadlock, and no
  livelock under fair scheduling), and every output at the end is a maximal
  matching of the graph (a member of the oracle's brute-force set);
* adversarial schedules: on every graph of up to 6 vertices, under four
  scheduling strategies (uniform, operations in flight as long as possible,
  near lockstep, one wavefront starved), the sweep ends within its trip
  bound with an output in the brute-force set; the same on random 8-vertex
  graphs with four lanes in two wavefronts;
* the order of a list is free: with every list shuffled, the adversarial
  schedules still end in the brute-force set;
* a scan may end at the first neighbour below its source when every list
  holds the neighbours above its vertex first (each part in any order); the
  same cut on lists in another order is caught;
* the model is sharp: three mistakes planted in it (no id order, no release
  of u, v taken by a plain store) are each caught on a small graph.
"""
import itertools

import numpy as np
import pytest

import graphgen
import oracle

from model import explore, graph, lanes, load, run, variant

VARIANTS = {
    "word_cas": dict(layout="word"),
    "word_cas_wait_release": dict(layout="word", wait_release=1),
    "word_two_phase": dict(layout="word", two_phase=1),
    "word_two_phase_lazy_wait_release": dict(layout="word", two_phase=1, lazy=1, wait_release=1),
    "word_cas_upper": dict(layout="word", upper=1),
    "u8_cas_word_retries": dict(layout="u8"),
    "u8_cas_lazy_wait_release": dict(layout="u8", lazy=1, wait_release=1),
    "u8_two_phase": dict(layout="u8", two_phase=1),
    "u2_cas_upper_wait_release": dict(layout="u2", upper=1, wait_release=1),
    "u2_two_phase_lazy": dict(layout="u2", two_phase=1, lazy=1),
    # state reads of one candidate: a source's first, or every one
    "word_cas_upper_probe_first": dict(layout="word", upper=1, probe=1, scan_width=3),
    "u8_two_phase_probe_each": dict(layout="u8", two_phase=1, probe=2),
}
STRATEGIES = (0, 1, 2, 3)


def all_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        yield graphgen.from_edges(n, [pairs[i] for i in range(len(pairs)) if mask >> i & 1])


_MAXIMAL = {}


def maximal_set(csr):
    """The maximal matchings of a small graph as mate tuples (brute force)."""
    key = (csr.n, tuple(csr.off.tolist()), tuple(csr.nbr.tolist()))
    if key not in _MAXIMAL:
        _MAXIMAL[key] = {tuple(int(v) for v in m)
                         for m in oracle.enumerate_matchings(csr, maximal_only=True)}
    return _MAXIMAL[key]


@pytest.fixture(scope="module", autouse=True)
def _built():
    load()


def test_model_on_the_worked_example():
    # the graph of Figs. 1 and 6: two lanes in one wavefront reach one of its
    # three maximal matchings on every schedule
    g = graphgen.from_edges(4, [(0, 1), (0, 2), (0, 3), (1, 2), (2, 3)])
    ok = maximal_set(g)
    assert ok == {(2, -1, 0, -1), (1, 0, 3, 2), (3, 2, 1, 0)}
    for name, v in VARIANTS.items():
        wave_of, src = lanes(4, 1, 2, "round")
        states, stuck, n_outs, outs = explore(graph(g), variant(**v), wave_of, src)
        assert states > 0 and stuck == 0 and n_outs > 0, name
        assert {tuple(o.tolist()) for o in outs} <= ok, name


EXHAUSTIVE_CONFIGS = [(2, 1, "round"), (1, 2, "round"), (2, 1, "blocks")]


@pytest.mark.parametrize("name", sorted(VARIANTS))
def test_every_schedule_ends_in_a_maximal_matching(name):
    # all 64 graphs on 4 vertices (smaller graphs are among them, with
    # isolated vertices). Word layouts: every placement of the sources on
    # lanes below. Packed layouts: stale reads are left to the random
    # schedules (a stale copy of a shared word multiplies the states), two
    # lanes of one wavefront on every graph, and two wavefronts on the
    # sparser graphs (at most 4 edges for the CAS protocol, 2 for two-phase,
    # whose commits of u and v and their mate writes interleave in every
    # order)
    v = dict(VARIANTS[name])
    packed = v["layout"] != "word"
    if packed:
        v["stale"] = 0
    var = variant(**v)
    graphs = list(all_graphs(4))
    total = 0
    for w, p, mode in EXHAUSTIVE_CONFIGS:
        wave_of, src = lanes(4, w, p, mode)
        for idx, g in enumerate(graphs):
            edges = bin(idx).count("1")
            if packed and w > 1 and (mode != "round" or edges > (2 if v.get("two_phase") else 4)):
                continue
            states, stuck, n_outs, outs = explore(graph(g), var, wave_of, src, max_states=400000)
            assert states > 0, (name, idx, (w, p, mode), states)
            assert stuck == 0, (name, idx, (w, p, mode), stuck)
            assert n_outs > 0, (name, idx, n_outs)
            ok = maximal_set(g)
            for o in outs:
                assert tuple(o.tolist()) in ok, (name, idx, o)
            total += states
    assert total > 1000


def _adversarial(graphs, lanes_cfg, name, strategies=STRATEGIES, seed0=1):
    var = variant(**VARIANTS[name])
    worst = 0
    for idx, g in enumerate(graphs):
        ok = maximal_set(g)
        G = graph(g)
        w, p, mode = lanes_cfg[idx % len(lanes_cfg)]
        wave_of, src = lanes(g.n, w, p, mode)
        for s in strategies:
            trips, mate = run(G, var, wave_of, src, strategy=s, seed=seed0 + 7919 * idx + s,
                              max_trips=20000)
            assert trips >= 0, (name, g.n, idx, s, trips)
            assert tuple(mate.tolist()) in ok, (name, g.n, idx, s, mate)
            worst = max(worst, trips)
    return worst


@pytest.mark.parametrize("name", sorted(VARIANTS))
def test_adversarial_schedules_on_every_graph_up_to_6_vertices(name):
    cfgs = [(2, 1, "round"), (1, 2, "blocks"), (2, 2, "round"), (3, 1, "blocks")]
    worst = 0
    for n in range(1, 6):
        worst = max(worst, _adversarial(list(all_graphs(n)), cfgs, name))
    # 6 vertices: every graph, one strategy each (all four over the set)
    var = variant(**VARIANTS[name])
    for idx, g in enumerate(all_graphs(6)):
        ok = maximal_set(g)
        w, p, mode = cfgs[idx % len(cfgs)]
        wave_of, src = lanes(6, w, p, mode)
        trips, mate = run(graph(g), var, wave_of, src, strategy=idx % 4, seed=idx, max_trips=20000)
        assert trips >= 0, (name, idx, trips)
        assert tuple(mate.tolist()) in ok, (name, idx, mate)
        worst = max(worst, trips)
    # far inside the bound: polling never runs away
    assert worst < 2000, worst


@pytest.mark.parametrize("name", sorted(VARIANTS))
def test_adversarial_schedules_on_larger_graphs(name):
    # 8 vertices, four lanes in two wavefronts (and the other placements)
    rng = np.random.default_rng(11)
    graphs = []
    for _ in range(150):
        p = rng.uniform(0.2, 0.8)
        E = [(a, b) for a, b in itertools.combinations(range(8), 2) if rng.random() < p]
        graphs.append(graphgen.from_edges(8, E))
    _adversarial(graphs, [(2, 2, "round"), (2, 2, "blocks"), (4, 1, "round"), (1, 4, "round")],
                 name, seed0=3)


class _Permuted:
    """A CSR with the entries of each list in another order (same edges)."""

    def __init__(self, csr, rng):
        self.n, self.m, self.off = csr.n, csr.m, csr.off
        nbr = csr.nbr.copy()
        for v in range(csr.n):
            b, e = int(csr.off[v]), int(csr.off[v + 1])
            nbr[b:e] = rng.permutation(nbr[b:e])
        self.nbr = nbr


@pytest.mark.parametrize("name", ["word_cas", "word_two_phase", "word_cas_upper", "u8_cas_word_retries",
                                  "u2_cas_upper_wait_release"])
def test_any_list_order(name):
    # the order in which a lane walks a list is free (the library may reorder
    # short lists by neighbour degree): every graph of up to 5 vertices and
    # random 7-vertex graphs with each list shuffled, under the four
    # adversarial strategies, still end in a maximal matching
    rng = np.random.default_rng(17)
    var = variant(**VARIANTS[name])
    graphs = [g for n in range(2, 6) for g in all_graphs(n)]
    for _ in range(120):
        p = rng.uniform(0.2, 0.8)
        graphs.append(graphgen.from_edges(7, [(a, b) for a, b in itertools.combinations(range(7), 2)
                                              if rng.random() < p]))
    cfgs = [(2, 1, "round"), (1, 2, "blocks"), (2, 2, "round")]
    for idx, g in enumerate(graphs):
        ok = maximal_set(g)
        G = graph(_Permuted(g, rng))
        w, p_, mode = cfgs[idx % len(cfgs)]
        wave_of, src = lanes(g.n, w, p_, mode)
        for st in STRATEGIES:
            trips, mate = run(G, var, wave_of, src, strategy=st, seed=idx * 13 + st, max_trips=20000)
            assert trips >= 0, (name, idx, st, trips)
            assert tuple(mate.tolist()) in ok, (name, idx, st, mate)


class _UpperFirst:
    """A CSR with each list's neighbours above its vertex first, each part
    shuffled (lower_first: those below first instead)."""

    def __init__(self, csr, rng, lower_first=False):
        self.n, self.m, self.off = csr.n, csr.m, csr.off
        nbr = csr.nbr.copy()
        for v in range(csr.n):
            b, e = int(csr.off[v]), int(csr.off[v + 1])
            seg = rng.permutation(nbr[b:e])
            below = seg < v
            nbr[b:e] = np.concatenate([seg[below], seg[~below]] if lower_first else
                                      [seg[~below], seg[below]])
        self.nbr = nbr


@pytest.mark.parametrize("name", ["word_cas_upper", "u2_cas_upper_wait_release", "u8_two_phase"])
def test_upper_first_scan_cut(name):
    # the reordered copy with the neighbours above each vertex first lets a
    # scan end at its first neighbour below the source: every graph of up to
    # 5 vertices and random 7-vertex graphs, under the four adversarial
    # strategies, still end in a maximal matching
    rng = np.random.default_rng(23)
    var = variant(**dict(VARIANTS[name], upper=2))
    graphs = [g for n in range(2, 6) for g in all_graphs(n)]
    for _ in range(120):
        p = rng.uniform(0.2, 0.8)
        graphs.append(graphgen.from_edges(7, [(a, b) for a, b in itertools.combinations(range(7), 2)
                                              if rng.random() < p]))
    cfgs = [(2, 1, "round"), (1, 2, "blocks"), (2, 2, "round")]
    for idx, g in enumerate(graphs):
        ok = maximal_set(g)
        G = graph(_UpperFirst(g, rng))
        w, p_, mode = cfgs[idx % len(cfgs)]
        wave_of, src = lanes(g.n, w, p_, mode)
        for st in STRATEGIES:
            trips, mate = run(G, var, wave_of, src, strategy=st, seed=idx * 11 + st, max_trips=20000)
            assert trips >= 0, (name, idx, st, trips)
            assert tuple(mate.tolist()) in ok, (name, idx, st, mate)


def test_scan_cut_needs_the_order():
    # the cut is sharp: on lists with the neighbours below each vertex first
    # it skips edges, and some small graph ends with an edge whose endpoints
    # are both unmatched
    var = variant(layout="word", upper=2)
    caught = 0
    for n in (3, 4):
        for g in all_graphs(n):
            ok = maximal_set(g)
            G = graph(_UpperFirst(g, np.random.default_rng(n), lower_first=True))
            wave_of, src = lanes(g.n, 1, 1, "blocks")
            trips, mate = run(G, var, wave_of, src, strategy=0, seed=1, max_trips=20000)
            caught += trips >= 0 and tuple(mate.tolist()) not in ok
    assert caught > 0


@pytest.mark.parametrize("mutant", [1, 2, 3])
def test_model_catches_planted_mistakes(mutant):
    # the model is sharp: each mistake planted in it (in the model, on the
    # CPU) is caught on some small graph as a state from which the sweep can
    # never end, or as an output that is not a maximal matching
    #   1: no id order (u = the source): two lanes hold each other's v
    #   2: u is never given back after a failed take of v: its holder's
    #      neighbours wait for it forever
    #   3: v taken by a plain store after a read saw it free: two lanes both
    #      "take" the same v
    caught = False
    for n in (2, 3, 4):
        for g in all_graphs(n):
            ok = maximal_set(g)
            for w, p, mode in EXHAUSTIVE_CONFIGS:
                wave_of, src = lanes(n, w, p, mode)
                states, stuck, n_outs, outs = explore(graph(g), variant("word", mutant=mutant),
                                                      wave_of, src, max_states=200000)
                if stuck > 0 or n_outs < 0 or any(tuple(o.tolist()) not in ok for o in outs):
                    caught = True
                    break
            if caught:
                break
        if caught:
            break
    assert caught, mutant
