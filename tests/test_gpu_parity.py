"""GPU parity: the HIP library against the oracle, through the C ABI.

Several maximal matchings are correct and the method is non-deterministic
(Section V-C), so parity means:
  * the exact checker finds zero violations of every class;
  * where the maximal matching is unique (disjoint edges, empty, isolated,
    loop-only graphs) the mate arrays are equal element by element;
  * where every maximal matching has the same size (cliques, K_{a,b}, stars)
    the sizes are equal;
  * on graphs with at most 12 vertices the output is one of the maximal
    matchings found by brute-force enumeration;
  * the size is reported beside SGMM's and is at least half of it (a maximal
    matching has at least half the pairs of any matching).
"""
import ctypes
import itertools
import random

import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2507_04420_amd as mm  # noqa: E402
from paper_2507_04420_amd import _lib  # noqa: E402

U8, U32, U2 = _lib.MM_LAYOUT_U8, _lib.MM_LAYOUT_U32, _lib.MM_LAYOUT_U2
CAS, TWO = _lib.MM_PROTOCOL_CAS, _lib.MM_PROTOCOL_TWO_PHASE
TUNINGS = {
    "default": mm.Tuning(),
    "u8_cas_lazy": mm.Tuning(layout=U8, lazy_init=1, assist_after=16),
    "u8_cas_eager": mm.Tuning(layout=U8, lazy_init=0),
    "u8_two_hint": mm.Tuning(layout=U8, protocol=TWO, hint=1, lazy_init=1),
    "u8_two_eager_w1": mm.Tuning(layout=U8, protocol=TWO, lazy_init=0, scan_width=1),
    "u32_cas": mm.Tuning(layout=U32, lazy_init=0),
    "u32_cas_hint_w1": mm.Tuning(layout=U32, hint=1, scan_width=1),
    "u32_two_lazy_hint": mm.Tuning(layout=U32, protocol=TWO, hint=1, lazy_init=1),
    "u32_two_eager": mm.Tuning(layout=U32, protocol=TWO, lazy_init=0, scan_width=3),
    "u8_disperse": mm.Tuning(layout=U8, disperse=1, protocol=TWO, lazy_init=1),
    "u8_small_blocks": mm.Tuning(layout=U8, wg_size=64, wave_vertices=64, assist_after=2,
                                 lazy_init=1),
    "u32_no_assist": mm.Tuning(layout=U32, protocol=TWO, assist_after=0, hint=1),
    "u2_two_eager": mm.Tuning(layout=U2, protocol=TWO, lazy_init=0),
    "u2_two_lazy": mm.Tuning(layout=U2, protocol=TWO, scan_width=2, lazy_init=1),
    "u2_cas_hint": mm.Tuning(layout=U2, protocol=CAS, hint=1, lazy_init=0),
    "u32_cas_hint_nt": mm.Tuning(layout=U32, hint=1, stream_loads=1),
    "relabel_u32_cas": mm.Tuning(relabel=1),
    "relabel_u32_cas_hint": mm.Tuning(relabel=1, hint=1, whole_graph_vertices=0,
                                      wave_vertices=64, wg_size=128),
    "relabel_u32_two": mm.Tuning(relabel=1, protocol=TWO, lazy_init=1, scan_width=2),
    "relabel_u8_cas": mm.Tuning(relabel=1, layout=U8, lazy_init=1, whole_graph_vertices=0),
    "relabel_u2_two_hint": mm.Tuning(relabel=1, layout=U2, protocol=TWO, hint=1, assist_after=4),
    "relabel_u32_bytehint": mm.Tuning(relabel=1, hint=2),
    "u8_two_bytehint": mm.Tuning(layout=U8, protocol=TWO, hint=2, lazy_init=1),
    "u32_cas_bytehint_w2": mm.Tuning(hint=2, scan_width=2, wave_vertices=128),
    "hub_every_entry": mm.Tuning(hub_degree=1, hub_chunk=1, hub_wave=0),
    "hub_small_u8_lazy": mm.Tuning(layout=U8, lazy_init=1, hub_degree=8, hub_chunk=3, hub_wave=0),
    "hub_relabel_two": mm.Tuning(relabel=1, protocol=TWO, hub_degree=5, hub_chunk=2, hint=2),
    "no_hub_tier": mm.Tuning(hub_degree=0),
    # small graphs are swept whole with their states in LDS by default; these
    # keep the states of a whole-graph sweep in device memory, or spread a
    # small graph over many wavefronts
    "whole_in_device_memory": mm.Tuning(whole_graph_lds=0),
    "whole_in_device_memory_u2_two": mm.Tuning(whole_graph_lds=0, layout=U2, protocol=TWO),
    "multi_wave_u8_lazy": mm.Tuning(layout=U8, lazy_init=1, whole_graph_vertices=0,
                                    wave_vertices=64, wg_size=64),
    "multi_wave_u32_two_bytehint": mm.Tuning(protocol=TWO, whole_graph_vertices=0,
                                             wave_vertices=64, hint=2),
    "wait_release_multi_wave": mm.Tuning(wait_release=1, whole_graph_vertices=0, wave_vertices=64),
    "wait_release_u8_two_lazy": mm.Tuning(layout=U8, protocol=TWO, wait_release=1, lazy_init=1,
                                          whole_graph_vertices=0, wave_vertices=64, wg_size=64),
    "wait_release_whole_lds": mm.Tuning(wait_release=1),
    # each undirected edge examined from its lower endpoint only
    "upper_only": mm.Tuning(upper_only=1),
    "upper_only_multi_wave_u8": mm.Tuning(upper_only=1, layout=U8, whole_graph_vertices=0,
                                          wave_vertices=64, lazy_init=1),
    "upper_only_relabel": mm.Tuning(upper_only=1, relabel=1),
    "upper_only_two_hub_assist": mm.Tuning(upper_only=1, protocol=TWO, hub_degree=5, hub_chunk=2,
                                           whole_graph_vertices=0, assist_after=2, scan_width=1),
    "upper_only_whole_device_wr": mm.Tuning(upper_only=1, whole_graph_lds=0, wait_release=1),
    # long lists swept by whole wavefronts, 64 ids per step
    "hub_wave_every_list": mm.Tuning(hub_wave=1, hub_degree=1, hub_chunk=3, whole_graph_vertices=0),
    "hub_wave_u8_relabel": mm.Tuning(hub_wave=1, hub_degree=5, hub_chunk=70, relabel=1, layout=U8),
    "hub_wave_two_upper_wr": mm.Tuning(hub_wave=1, hub_degree=8, hub_chunk=100, protocol=TWO,
                                       upper_only=1, wait_release=1, whole_graph_vertices=0),
    "hub_wave_bit_hint_u2": mm.Tuning(hub_wave=1, hub_degree=4, hub_chunk=64, hint=1, layout=U2,
                                      protocol=TWO, whole_graph_vertices=0),
    # the workgroup tier: wavefronts of a workgroup share the sources they found matched
    "hub_group_every_list": mm.Tuning(hub_wave=2, hub_degree=1, hub_chunk=3, whole_graph_vertices=0,
                                      wg_size=256),
    "hub_group_u8_upper_two_waves": mm.Tuning(hub_wave=2, hub_degree=4, hub_chunk=9, layout=U8,
                                              upper_only=1, wg_size=128, whole_graph_vertices=0),
    "hub_group_two_hint_relabel": mm.Tuning(hub_wave=2, hub_degree=6, hub_chunk=2, protocol=TWO,
                                            hint=2, relabel=1, wg_size=192),
    # short lists reordered by the degree of the neighbour
    "order_lists": mm.Tuning(order_lists=1),
    "order_lists_upper_multi_wave_u8": mm.Tuning(order_lists=1, upper_only=1, layout=U8,
                                                 whole_graph_vertices=0, wave_vertices=64),
    "order_lists_two_hubs_hint": mm.Tuning(order_lists=1, protocol=TWO, hint=2, hub_degree=5,
                                           hub_chunk=3, whole_graph_vertices=0),
    # the same with the neighbours above each vertex first, where a scan of a
    # short list ends at its first neighbour below the source: in the lane's
    # reads, in the wavefront assist's, and never in a hub piece
    "upper_first": mm.Tuning(order_lists=2, upper_only=1, whole_graph_vertices=0),
    "upper_first_assist_u8": mm.Tuning(order_lists=2, upper_only=1, layout=U8, assist_after=16,
                                       scan_width=2, whole_graph_vertices=0, wave_vertices=64),
    # the sweep kernel built for six wavefronts per SIMD
    "occupancy6_tuned_shape": mm.Tuning(occupancy=6, order_lists=2, upper_only=1, probe_first=1,
                                        assist_after=16, whole_graph_vertices=0),
    "occupancy6_u2_two_lazy_hubs": mm.Tuning(occupancy=6, layout=U2, protocol=TWO, lazy_init=1,
                                             hub_degree=5, hub_chunk=3, hub_wave=0,
                                             whole_graph_vertices=0),
    "occupancy6_u8_bytehint_release": mm.Tuning(occupancy=6, layout=U8, hint=2, wait_release=1,
                                                whole_graph_vertices=0, wave_vertices=64),
    # a source's first state read takes its first candidate only
    "probe_first_ordered": mm.Tuning(probe_first=1, order_lists=1, upper_only=1, whole_graph_vertices=0),
    "probe_each_upper_first_assist": mm.Tuning(probe_first=2, order_lists=2, upper_only=1, assist_after=8,
                                               whole_graph_vertices=0),
    "probe_first_u8_two_hint_w3": mm.Tuning(probe_first=1, layout=U8, protocol=TWO, hint=1, scan_width=3,
                                            whole_graph_vertices=0, wave_vertices=64),
    "upper_first_two_lane_pieces": mm.Tuning(order_lists=2, upper_only=1, protocol=TWO, hub_degree=5,
                                             hub_chunk=3, hub_wave=0, whole_graph_vertices=0),
    # relabelled with the vertices of more than hot_degree entries last
    "relabel_hot_u32_cas": mm.Tuning(relabel=2, hot_degree=4),
    "relabel_hot_upper_multi_wave": mm.Tuning(relabel=2, hot_degree=8, upper_only=1,
                                              whole_graph_vertices=0, wave_vertices=64),
    "relabel_hot_u8_two_bytehint": mm.Tuning(relabel=2, hot_degree=2, layout=U8, protocol=TWO,
                                             hint=2, lazy_init=1),
    "relabel_hot_hub_wave_upper": mm.Tuning(relabel=2, hot_degree=3, hub_wave=1, hub_degree=5,
                                            hub_chunk=7, upper_only=1, whole_graph_vertices=0),
}


def to_dev(csr):
    return torch.from_numpy(np.ascontiguousarray(csr.off)).cuda(), torch.from_numpy(
        np.ascontiguousarray(csr.nbr)).cuda()


def gpu_match(csr, tuning=None, symmetric=True, stats=False, validate=True):
    off, nbr = to_dev(csr)
    g = mm.Graph(off, nbr, symmetric=symmetric, validate=validate, tuning=tuning, stats=stats)
    out = g.run()
    g.sync()
    mate = out.cpu().numpy()
    st = g.stats() if stats else None
    g.close()
    return mate, st


def assert_parity(csr, mate, exact=None, same_size_as=None):
    c = oracle.check(csr, mate)
    assert c.violations == 0, c
    assert c.bad_input == 0
    r = oracle.sgmm(csr)
    assert 2 * c.size >= r.pairs, (c.size, r.pairs)
    if exact is not None:
        np.testing.assert_array_equal(mate, exact)
    if same_size_as is not None:
        assert c.size == same_size_as
    return c


def pairs_of(mate):
    return sorted((int(a), int(b)) for a, b in enumerate(mate) if b > a)


@pytest.fixture(params=sorted(TUNINGS))
def tuning(request):
    return TUNINGS[request.param]


# ---------------------------------------------------------------- small graphs

def test_fig6_worked_example(tuning):
    g = graphgen.from_edges(4, [(0, 1), (0, 2), (0, 3), (1, 2), (2, 3)])
    mate, _ = gpu_match(g, tuning)
    assert_parity(g, mate)
    assert pairs_of(mate) in ([(0, 2)], [(0, 1), (2, 3)], [(0, 3), (1, 2)])


@pytest.mark.parametrize("k", [1, 2, 3, 64, 65, 1000])
def test_path(tuning, k):
    g = graphgen.from_edges(k, [(i, i + 1) for i in range(k - 1)] or np.zeros((0, 2)))
    mate, _ = gpu_match(g, tuning)
    c = assert_parity(g, mate)
    assert (k - 1 + 2) // 3 <= c.size <= k // 2


@pytest.mark.parametrize("k", [1, 5, 63, 64, 65, 5000])
def test_star(tuning, k):
    g = graphgen.from_edges(k + 1, [(0, j) for j in range(1, k + 1)])
    mate, _ = gpu_match(g, tuning)
    assert_parity(g, mate, same_size_as=1)


@pytest.mark.parametrize("n", [2, 3, 17, 64, 130])
def test_clique(tuning, n):
    g = graphgen.from_edges(n, list(itertools.combinations(range(n), 2)))
    mate, _ = gpu_match(g, tuning)
    assert_parity(g, mate, same_size_as=n // 2)


@pytest.mark.parametrize("a,b", [(1, 1), (3, 70), (70, 3), (64, 64), (100, 37)])
def test_complete_bipartite(tuning, a, b):
    g = graphgen.from_edges(a + b, [(i, a + j) for i in range(a) for j in range(b)])
    mate, _ = gpu_match(g, tuning)
    assert_parity(g, mate, same_size_as=min(a, b))


@pytest.mark.parametrize("k", [1, 64, 1000, 4099])
def test_disjoint_edges_bitwise(tuning, k):
    g = graphgen.from_edges(2 * k, [(2 * i, 2 * i + 1) for i in range(k)])
    exact = np.arange(2 * k, dtype=np.int32) ^ 1
    mate, _ = gpu_match(g, tuning)
    assert_parity(g, mate, exact=exact)


def test_empty_isolated_loops(tuning):
    for n in (1, 63, 64, 65, 3000):
        g = graphgen.from_edges(n, np.zeros((0, 2)))
        mate, _ = gpu_match(g, tuning)
        assert_parity(g, mate, exact=np.full(n, -1, dtype=np.int32))
    g = graphgen.from_edges(130, [(v, v) for v in range(0, 130, 3)], symmetric=False)
    mate, _ = gpu_match(g, tuning)
    assert_parity(g, mate, exact=np.full(130, -1, dtype=np.int32))


def test_zero_vertices():
    off = torch.zeros(1, dtype=torch.int64, device="cuda")
    nbr = torch.zeros(0, dtype=torch.int32, device="cuda")
    g = mm.Graph(off, nbr, symmetric=True, validate=True)
    out = g.run()
    g.sync()
    assert out.numel() == 0


@pytest.mark.parametrize("seed", range(30))
def test_random_small_in_bruteforce_set(seed):
    rng = random.Random(1000 + seed)
    n = rng.randint(2, 12)
    p = rng.choice([0.2, 0.4, 0.7])
    edges = [e for e in itertools.combinations(range(n), 2) if rng.random() < p]
    g = graphgen.from_edges(n, edges if edges else np.zeros((0, 2)))
    mset = {tuple(m) for m in oracle.enumerate_matchings(g)}
    for name in sorted(TUNINGS):
        mate, _ = gpu_match(g, TUNINGS[name])
        assert tuple(mate) in mset, (name, pairs_of(mate))


# ---------------------------------------------------------------- mid-size, ragged, skewed

@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_er_65536_deg16(tuning, seed):
    g = graphgen.er(65536, 16, seed=seed)
    mate, _ = gpu_match(g, tuning)
    assert_parity(g, mate)


def test_er_int32_offsets(tuning):
    g = graphgen.er(65536, 16, seed=11).with_int32_offsets()
    mate, _ = gpu_match(g, tuning)
    assert_parity(g, mate)


@pytest.mark.parametrize("n", [100_003, 4097, 1025])
def test_er_ragged(tuning, n):
    g = graphgen.er(n, 9, seed=n)
    mate, _ = gpu_match(g, tuning)
    assert_parity(g, mate)


@pytest.mark.parametrize("scale", [12, 16, 18])
def test_rmat(tuning, scale):
    g = graphgen.rmat(scale, seed=scale)
    mate, _ = gpu_match(g, tuning)
    assert_parity(g, mate)


@pytest.mark.parametrize("H,W", [(1, 1), (7, 9), (301, 517), (1024, 1024)])
def test_grid(tuning, H, W):
    g = graphgen.grid(H, W)
    mate, _ = gpu_match(g, tuning)
    assert_parity(g, mate)


def test_non_symmetric_input(tuning):
    # Section V-C: each edge stored in one endpoint's list only; the result must
    # be maximal for the union (no lazy output is used for such input)
    rng = np.random.default_rng(5)
    n = 20000
    e = rng.integers(0, n, size=(120000, 2))
    g = graphgen.from_edges(n, e, symmetric=False)
    mate, _ = gpu_match(g, tuning, symmetric=False)
    assert_parity(g, mate)


def test_duplicates_and_loops(tuning):
    rng = np.random.default_rng(9)
    n = 5000
    e = rng.integers(0, n, size=(40000, 2))
    e = np.concatenate([e, e[:5000], np.stack([np.arange(n)] * 2, 1)])
    g = graphgen.from_edges(n, e, symmetric=True, dedup=False, sort=False)
    mate, _ = gpu_match(g, tuning)
    assert_parity(g, mate)


# ---------------------------------------------------------------- contention

@pytest.mark.parametrize("rep", range(3))
def test_contention_star_and_clique(rep):
    for name in sorted(TUNINGS):
        t = TUNINGS[name]
        g = graphgen.from_edges(200_001, [(0, j) for j in range(1, 200_001)])
        mate, _ = gpu_match(g, t)
        assert_parity(g, mate, same_size_as=1)
        g = graphgen.from_edges(600, list(itertools.combinations(range(600), 2)))
        mate, _ = gpu_match(g, t)
        assert_parity(g, mate, same_size_as=300)


def test_contention_unpermuted_rmat(tuning):
    g = graphgen.rmat(16, seed=3, permute=False)
    mate, _ = gpu_match(g, tuning)
    assert_parity(g, mate)


# ---------------------------------------------------------------- handle behaviour

def test_repeated_runs_same_handle(tuning):
    g = graphgen.rmat(15, seed=7)
    off, nbr = to_dev(g)
    h = mm.Graph(off, nbr, symmetric=True, tuning=tuning)
    for _ in range(4):
        out = h.run()
        h.sync()
        assert_parity(g, out.cpu().numpy())


def test_stats_consistent():
    g = graphgen.rmat(16, seed=1)
    mate, st = gpu_match(g, mm.Tuning(), stats=True)
    c = assert_parity(g, mate)
    assert st["pairs"] == c.size
    assert st["sources"] == g.n
    assert st["touched"] <= g.m
    assert st["match_attempts"] >= st["pairs"]


def test_validate_rejects_bad_graph():
    off = torch.tensor([0, 2, 3], dtype=torch.int64, device="cuda")
    nbr = torch.tensor([1, 7, 0], dtype=torch.int32, device="cuda")
    with pytest.raises(mm.MMError) as ei:
        mm.Graph(off, nbr, validate=True)
    assert ei.value.status == _lib.MM_ERR_INVALID_GRAPH
    off = torch.tensor([0, 2, 1, 3], dtype=torch.int64, device="cuda")
    nbr = torch.tensor([1, 2, 0], dtype=torch.int32, device="cuda")
    with pytest.raises(mm.MMError):
        mm.Graph(off, nbr, validate=True)


def test_loop_budget_reports_no_progress():
    # A one-trip budget cannot finish a clique; every wavefront still exits
    # normally and the failure surfaces at sync.
    g = graphgen.from_edges(300, list(itertools.combinations(range(300), 2)))
    off, nbr = to_dev(g)
    h = mm.Graph(off, nbr, symmetric=True, tuning=mm.Tuning(iter_cap=1))
    h.run()
    with pytest.raises(mm.MMError) as ei:
        h.sync()
    assert ei.value.status == _lib.MM_ERR_NO_PROGRESS
    h2 = mm.Graph(off, nbr, symmetric=True)
    out = h2.run()
    h2.sync()
    assert_parity(g, out.cpu().numpy(), same_size_as=150)


# ---------------------------------------------------------------- Table II instrumentation

def check_conflict_row(row, st):
    hist = st["conflict_hist"]
    edges = sum(hist)
    # every failed take of u or v is a conflict (Table II), whether it met a
    # reservation or a match made since the lane's cached read
    total = (st["reserve_conflicts"] + st["match_conflicts"] + st["reserve_matched"]
             + st["match_matched"])
    assert row["edges"] == edges and row["total"] == total
    assert row["met_reserved"] + row["met_matched"] == total
    # each conflicting edge met at least its bin's lower bound, at most its upper
    lo = [1, 2, 3, 5, 9, 17, 33, 65, 129, 257]
    hi = [1, 2, 4, 8, 16, 32, 64, 128, 256, None]
    assert sum(l * c for l, c in zip(lo, hist)) <= total
    if hist[-1] == 0:
        assert total <= sum(h * c for h, c in zip(hi[:9], hist[:9]))
    if edges == 0:
        assert total == 0 and st["conflict_max"] == 0
    else:
        top = max(b for b in range(10) if hist[b])
        assert lo[top] <= st["conflict_max"] and (hi[top] is None or st["conflict_max"] <= hi[top])
        assert st["conflict_max"] <= total


@pytest.mark.parametrize("graph", ["star", "clique", "rmat_unpermuted", "rmat"])
def test_conflict_histogram_invariants(graph):
    if graph == "star":
        g = graphgen.from_edges(100_001, [(0, j) for j in range(1, 100_001)])
    elif graph == "clique":
        g = graphgen.from_edges(400, list(itertools.combinations(range(400), 2)))
    elif graph == "rmat_unpermuted":
        g = graphgen.rmat(16, seed=3, permute=False)
    else:
        g = graphgen.rmat(18, seed=2)
    for t in (mm.Tuning(), mm.Tuning(layout=_lib.MM_LAYOUT_U8, lazy_init=1)):
        mate, st = gpu_match(g, t, stats=True)
        assert_parity(g, mate)
        check_conflict_row(mm.conflict_row(st), st)


def test_conflict_table_worst_of_runs():
    g = graphgen.from_edges(600, list(itertools.combinations(range(600), 2)))
    off, nbr = to_dev(g)
    row = mm.conflict_table(off, nbr, runs=5)
    assert row["runs"] == 5 and row["entries"] == g.m
    assert 0 <= row["edge_ratio"] <= 1
    assert sum(row["distribution"].values()) == row["edges"]


# ---------------------------------------------------------------- pair-list output

@pytest.mark.parametrize("graph", ["rmat", "grid", "empty", "single_edge"])
def test_pair_list_matches_mates(graph):
    if graph == "rmat":
        g = graphgen.rmat(16, seed=5)
    elif graph == "grid":
        g = graphgen.grid(129, 77)
    elif graph == "empty":
        g = graphgen.from_edges(7, np.zeros((0, 2)))
    else:
        g = graphgen.from_edges(2, [(0, 1)])
    off, nbr = to_dev(g)
    h = mm.Graph(off, nbr, symmetric=True)
    mate = h.run()
    h.sync()
    pairs = h.pairs(mate).cpu().numpy()
    mt = mate.cpu().numpy()
    c = assert_parity(g, mt)
    assert pairs.shape == (c.size, 2)
    assert (pairs[:, 0] < pairs[:, 1]).all()
    assert (mt[pairs[:, 0]] == pairs[:, 1]).all() and (mt[pairs[:, 1]] == pairs[:, 0]).all()
    assert len(set(map(tuple, pairs.tolist()))) == c.size  # each pair once


def test_pair_list_small_buffer_reports_count():
    g = graphgen.from_edges(8, [(0, 1), (2, 3), (4, 5), (6, 7)])
    off, nbr = to_dev(g)
    h = mm.Graph(off, nbr, symmetric=True)
    mate = h.run()
    h.sync()
    buf = torch.full((4,), -5, dtype=torch.int32, device="cuda")  # room for 2 pairs
    cnt = ctypes.c_int64()
    st = _lib.load().mm_pairs(h.handle, None, ctypes.c_void_p(mate.data_ptr()),
                              ctypes.c_void_p(buf.data_ptr()), 2, ctypes.byref(cnt))
    assert st == _lib.MM_ERR_OUT_OF_MEMORY and cnt.value == 4
    b = buf.cpu().numpy().reshape(2, 2)
    assert all(row[1] == row[0] + 1 and row[0] % 2 == 0 for row in b)


# ---------------------------------------------------------------- relabelled sweep

@pytest.mark.parametrize("mode", [1, 2])
def test_relabel_all_isolated_and_stats(mode):
    # every vertex isolated: the relabelled sweep has no source at all
    g = graphgen.from_edges(1000, np.zeros((0, 2)))
    mate, st = gpu_match(g, mm.Tuning(relabel=mode), stats=True)
    assert (mate == -1).all() and st["sources"] == 0
    # sources visited = vertices with entries
    g = graphgen.rmat(14, seed=6)
    mate, st = gpu_match(g, mm.Tuning(relabel=mode, hot_degree=40, whole_graph_vertices=0),
                         stats=True)
    assert_parity(g, mate)
    assert st["sources"] == int((np.diff(g.off) > 0).sum())
    assert st["pairs"] == oracle.check(g, mate).size


def test_relabel_workspace_sizing():
    g = graphgen.rmat(12, seed=2)
    off, nbr = to_dev(g)
    t = mm.Tuning(relabel=1).to_c()
    lib = _lib.load()
    assert lib.mm_workspace_bytes(g.n, ctypes.byref(t)) == 0
    need = lib.mm_workspace_bytes_graph(g.n, g.m, ctypes.byref(t))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    st = lib.mm_create(ctypes.c_void_p(off.data_ptr()), _lib.MM_OFF_I64, ctypes.c_void_p(nbr.data_ptr()),
                       g.n, g.m, ctypes.c_void_p(ws.data_ptr()), need - 256, 0, ctypes.byref(t), None,
                       ctypes.byref(h))
    assert st == _lib.MM_ERR_OUT_OF_MEMORY and not h.value


@pytest.mark.parametrize("name", ["default", "u8_cas_eager", "relabel_u32_cas", "relabel_u8_cas",
                                  "u32_two_eager", "relabel_hot_u32_cas"])
@pytest.mark.parametrize("shift", [1, 2, 3])
def test_unaligned_output(name, shift):
    # an output view at any 4-byte offset: fills and sweep write exactly its n entries
    g = graphgen.rmat(13, seed=8)
    off, nbr = to_dev(g)
    h = mm.Graph(off, nbr, symmetric=True, tuning=TUNINGS[name])
    buf = torch.full((g.n + 8,), 12345, dtype=torch.int32, device="cuda")
    out = buf[shift:shift + g.n]
    h.run(out)
    h.sync()
    b = buf.cpu().numpy()
    assert (b[:shift] == 12345).all() and (b[shift + g.n:] == 12345).all()
    assert_parity(g, b[shift:shift + g.n])


def expected_relabel(csr, mode, hot):
    """The relabelled copy relabel.hip builds, computed here: new -> given map
    (a stable sort by the mode's key), int64 offsets in the new order, and the
    lists with ids mapped (mode 1: lists of at most 64 entries sorted by new
    id; mode 2: given order)."""
    deg = np.diff(csr.off.astype(np.int64))
    if mode == 1:
        key = np.zeros(csr.n, dtype=np.int64)
        nz = deg > 0
        key[nz] = np.floor(np.log2(deg[nz])).astype(np.int64) + 1
    else:
        key = np.where(deg == 0, 0, np.where(deg > hot, 2, 1))
    orig = np.argsort(key, kind="stable").astype(np.int32)
    inv = np.empty(csr.n, dtype=np.int64)
    inv[orig] = np.arange(csr.n)
    roff = np.zeros(csr.n + 1, dtype=np.int64)
    roff[1:] = np.cumsum(deg[orig])
    rnbr = np.empty(csr.m, dtype=np.int32)
    for v in range(csr.n):
        x = orig[v]
        lst = inv[csr.nbr[csr.off[x]:csr.off[x + 1]]]
        if mode == 1 and len(lst) <= 64:
            lst = np.sort(lst)
        rnbr[roff[v]:roff[v + 1]] = lst
    return orig, roff, rnbr


@pytest.mark.parametrize("mode", [1, 2])
def test_relabelled_copy_is_the_stated_order(mode):
    # white box, bit for bit: with the word layout and no hint the workspace
    # holds the 4 KiB control block, the states in new ids (4n), then the
    # relabelled offsets, the new -> given map and the lists
    csr = graphgen.rmat(13, seed=4)
    hot = 40
    off, nbr = to_dev(csr)
    h = mm.Graph(off, nbr, symmetric=True, tuning=mm.Tuning(relabel=mode, hot_degree=hot))
    r256 = lambda b: (b + 255) // 256 * 256
    base = h.workspace.data_ptr()
    region = (base + 255) // 256 * 256 - base + 4096 + r256(4 * csr.n)
    ws = h.workspace
    roff = ws[region:region + 8 * (csr.n + 1)].view(torch.int64).cpu().numpy()
    o0 = region + r256(8 * (csr.n + 1))
    orig = ws[o0:o0 + 4 * csr.n].view(torch.int32).cpu().numpy()
    n0 = o0 + r256(4 * csr.n)
    rnbr = ws[n0:n0 + 4 * csr.m].view(torch.int32).cpu().numpy()
    e_orig, e_roff, e_rnbr = expected_relabel(csr, mode, hot)
    np.testing.assert_array_equal(orig, e_orig)
    np.testing.assert_array_equal(roff, e_roff)
    np.testing.assert_array_equal(rnbr, e_rnbr)
    out = h.run()
    h.sync()
    assert_parity(csr, out.cpu().numpy())
    h.close()


# ---------------------------------------------------------------- reordered lists

def expected_order(csr, upper_first=False):
    """The copy order_lists builds, computed here: each list of at most 256
    entries stably sorted by 1 + floor(log2 degree) of the neighbour, longer
    lists as given; with upper_first, stably sorted first by whether the
    neighbour is below the list's vertex."""
    deg = np.diff(csr.off.astype(np.int64))
    bucket = np.zeros(csr.n, dtype=np.int64)
    nz = deg > 0
    bucket[nz] = np.floor(np.log2(deg[nz])).astype(np.int64) + 1
    out = csr.nbr.copy()
    for v in range(csr.n):
        b, e = int(csr.off[v]), int(csr.off[v + 1])
        if 1 < e - b <= 256:
            seg = csr.nbr[b:e]
            seg = seg[np.argsort(bucket[seg], kind="stable")]
            if upper_first:
                seg = seg[np.argsort(seg < v, kind="stable")]
            out[b:e] = seg
    return out


@pytest.mark.parametrize("upper_first", [False, True])
@pytest.mark.parametrize("make", [lambda: graphgen.rmat(14, seed=3), lambda: graphgen.er(3000, 20, seed=1),
                                  lambda: hub_trap(300), lambda: hub_trap(100)])
def test_order_lists_copy_is_the_stable_degree_order(make, upper_first):
    # white box, bit for bit: with the word layout and no hint the workspace
    # holds the 4 KiB control block, then the reordered copy of the ids
    csr = make()
    off, nbr = to_dev(csr)
    t = mm.Tuning(order_lists=2, upper_only=1) if upper_first else mm.Tuning(order_lists=1)
    h = mm.Graph(off, nbr, symmetric=True, tuning=t)
    base = h.workspace.data_ptr()
    start = (base + 255) // 256 * 256 - base + 4096
    copy = h.workspace[start:start + 4 * csr.m].view(torch.int32).cpu().numpy()
    np.testing.assert_array_equal(copy, expected_order(csr, upper_first))
    out = h.run()
    h.sync()
    assert_parity(csr, out.cpu().numpy())
    h.close()


# ---------------------------------------------------------------- hub tier

def hub_trap(k):
    # k disjoint edges (2i, 2i+1) and one last vertex adjacent to all of them:
    # in id order every pair matches first, and the hub's whole list is dead
    pairs = np.stack([np.arange(0, 2 * k, 2), np.arange(1, 2 * k, 2)], 1)
    hub = np.stack([np.full(2 * k, 2 * k), np.arange(2 * k)], 1)
    return graphgen.from_edges(2 * k + 1, np.concatenate([pairs, hub]))


@pytest.mark.parametrize("name", ["default", "hub_every_entry", "hub_relabel_two", "no_hub_tier"])
def test_hub_trap(name):
    g = hub_trap(50_000)
    mate, _ = gpu_match(g, TUNINGS[name])
    assert_parity(g, mate)
    assert mate[2 * 50_000] == -1 or mate[mate[2 * 50_000]] == 2 * 50_000


def test_hub_tier_spreads_a_long_dead_list():
    # with the tier, the hub's dead list is swept by many lanes at once
    import time
    g = hub_trap(1_000_000)
    off, nbr = to_dev(g)
    times = {}
    for name, t in (("tier", mm.Tuning(hub_wave=0)), ("wave_tier", mm.Tuning(hub_wave=1)),
                    ("group_tier", mm.Tuning(hub_wave=2)), ("no_tier", mm.Tuning(hub_degree=0))):
        h = mm.Graph(off, nbr, symmetric=True, tuning=t, timing=True)
        out = h.run()
        h.sync()
        h.timing()
        h.run(out)
        h.sync()
        times[name] = h.timing()["mean_ms"]
        assert_parity(g, out.cpu().numpy())
        h.close()
    print("hub trap sweep ms:", times)
    assert times["tier"] * 5 < times["no_tier"]
    assert times["wave_tier"] * 5 < times["no_tier"]
    assert times["group_tier"] * 5 < times["no_tier"]
