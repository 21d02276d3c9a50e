"""The serving loop on the GPU, in the configuration the serving benchmark
runs (GpuExecutor.for_serving: the stored batch entry with whole-graph items
and lanes that release u while they wait; large jobs alone with their graph
class's tuning, ResidentGraph.for_serving). Every request of a Poisson trace
(small jobs coalesced into list batches, large jobs on solo streams,
overlapping) gets a maximal matching, and each result is the same in the mix
as alone within the alone-vs-mix tolerance: identical checker verdicts;
bitwise equality where the maximal matching is unique or the graph is swept
whole by one wavefront; equal size where every maximal matching has the same
size; otherwise |size_mix - size_alone| <= max(2, 1% of SGMM's)."""
import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2507_04420_amd as mm  # noqa: E402
from paper_2507_04420_amd import autotune, serve  # noqa: E402

WHOLE = mm.Tuning().whole_graph_vertices  # serve.batch_tuning() keeps it
SMALL_EDGES = 200_000


def k2_union(k):
    return graphgen.from_edges(2 * k, [(2 * i, 2 * i + 1) for i in range(k)]), "unique"


def clique(n):
    return graphgen.from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)]), "same_size"


def kab(a, b):
    return graphgen.from_edges(a + b, [(i, a + j) for i in range(a) for j in range(b)]), "same_size"


def star(k):
    return graphgen.from_edges(k + 1, [(0, i) for i in range(1, k + 1)]), "same_size"


# General graphs that run alone, one or more per class a serving request can
# fall in below 2^25 vertices (the classes tuned under the spread limit).
GENERAL_SOLO = [
    (lambda: graphgen.rmat(15, seed=2), "rmat_small", "rmat15_ef16_s2"),
    (lambda: graphgen.er(40000, 12, seed=3), "er_small", "er40000_d12_s3"),
    (lambda: graphgen.grid(300, 301), "grid_small", "grid300x301"),
    (lambda: graphgen.rmat(18, 8, seed=1), "rmat_mid", "rmat18_ef8_s1"),
    (lambda: graphgen.grid(724, 724), "grid_mid", "grid724x724"),
]

_POOL = None


def pool():
    global _POOL
    if _POOL is not None:
        return _POOL
    items = [k2_union(500), k2_union(3), clique(9), clique(40), kab(7, 30), star(200),
             (graphgen.from_edges(6, np.zeros((0, 2))), "unique")]
    mix = graphgen.mixture(16, seed=21, nmin=200, nmax=20000)
    items += [(mix.member(g), "general") for g in range(mix.num_graphs)]
    for make, cls, name in GENERAL_SOLO:
        csr = make()
        assert csr.name == name and autotune.classify(csr.off) == cls, (csr.name, cls)
        items.append((csr, "general"))
    out = []
    for csr, cls in items:
        off64 = csr.off.astype(np.int64)
        off = torch.from_numpy(off64).cuda()
        nbr = torch.from_numpy(csr.nbr).cuda()
        out.append((serve.ResidentGraph.for_serving(off, nbr, off64, True, csr.name), csr, cls))
    _POOL = out
    return out


def scheduler(**kw):
    ex = serve.GpuExecutor.for_serving(batch_slots=2, solo_slots=2)
    free, _ = torch.cuda.mem_get_info()
    args = dict(hbm_budget=free // 4, small_edges=SMALL_EDGES, max_batch=64, batch_slots=2,
                solo_slots=2)
    args.update(kw)
    return serve.Scheduler(ex, **args)


def run(reqs, **kw):
    s = scheduler(**kw)
    comps, wall = serve.run_trace(s, reqs, timeout=60)
    torch.cuda.synchronize()
    return {c.rid: c for c in comps}, s


_SGMM = {}


def sgmm_pairs(csr):
    if csr.name not in _SGMM:
        _SGMM[csr.name] = oracle.sgmm(csr).pairs
    return _SGMM[csr.name]


def bound(csr):
    return max(2, 0.01 * sgmm_pairs(csr))


def test_pool_covers_every_serving_class_and_route():
    P = pool()
    classes = {autotune.classify(csr.off) for _, csr, cls in P if cls == "general" and csr.n > WHOLE}
    assert classes >= {"rmat_small", "er_small", "grid_small", "rmat_mid", "grid_mid"}
    s = scheduler()
    routes = {(s.route(serve.Request(0, rg, 0.0)), csr.n > WHOLE) for rg, csr, cls in P}
    # small jobs swept whole, small jobs swept in blocks inside a batch, and
    # large jobs alone (some of them swept whole too)
    assert ("batch", False) in routes and ("batch", True) in routes and ("solo", True) in routes


def test_mix_equals_alone():
    P = pool()
    rng = np.random.default_rng(5)
    n_req = 160
    gid = rng.integers(0, len(P), size=n_req)
    # every general graph that runs alone is in the trace at least twice
    solo_general = [g for g, (rg, csr, cls) in enumerate(P) if cls == "general" and csr.m > SMALL_EDGES]
    gid[:2 * len(solo_general)] = np.repeat(solo_general, 2)
    rng.shuffle(gid)
    arr = serve.poisson_arrivals(n_req, 4000.0, seed=6)
    reqs = [serve.Request(i, P[g][0], float(arr[i])) for i, g in enumerate(gid)]
    mix, s = run(reqs)
    assert len(mix) == n_req
    routes = {c.route for c in mix.values()}
    assert routes == {"batch", "solo"}
    # continuous batching: some launch served several requests
    assert max(len([c for c in mix.values() if c.launch == L]) for L in {c.launch for c in mix.values()}) > 1
    worst = {}
    for i, g in enumerate(gid):
        rg, csr, cls = P[g]
        m_mix = mix[i].mate.cpu().numpy()
        alone, _ = run([serve.Request(0, rg, 0.0)])
        m_alone = alone[0].mate.cpu().numpy()
        c_mix, c_alone = oracle.check(csr, m_mix), oracle.check(csr, m_alone)
        assert c_mix.ok and c_alone.ok, (i, csr.name, c_mix, c_alone)
        if cls == "unique" or csr.n <= WHOLE:
            # unique result, or a graph small enough for one wavefront: the
            # sweep does not depend on what else runs
            np.testing.assert_array_equal(m_mix, m_alone)
        elif cls == "same_size":
            assert c_mix.size == c_alone.size
        else:
            d = abs(c_mix.size - c_alone.size)
            worst[csr.name] = max(worst.get(csr.name, 0.0), d / bound(csr))
            assert d <= bound(csr), (csr.name, c_mix.size, c_alone.size, bound(csr))
    print("alone vs mix, worst |difference| / bound per general graph:",
          {k: round(v, 3) for k, v in sorted(worst.items())})


@pytest.mark.parametrize("which,name", [(cls, name) for _, cls, name in GENERAL_SOLO])
def test_alone_spread_is_recorded(which, name):
    # ten alone runs of each general graph that runs alone with a tuning of
    # the serving classes: the spread shows that the size bound of the mix
    # test is not vacuous (sizes do vary between schedules) and how far inside
    # it the serving shapes keep a job
    P = pool()
    rg, csr = next((rg, csr) for rg, csr, cls in P if csr.name == name)
    assert csr.n > WHOLE and autotune.classify(csr.off) == which
    assert csr.m > SMALL_EDGES  # the mix test's scheduler runs it alone
    sizes = []
    for rep in range(10):
        alone, _ = run([serve.Request(0, rg, 0.0)])
        c = oracle.check(csr, alone[0].mate.cpu().numpy())
        assert c.ok
        sizes.append(c.size)
    spread = max(sizes) - min(sizes)
    print("alone sizes %s (%s): %d..%d spread %d, bound %.1f (%.2f of it)" % (
        csr.name, which, min(sizes), max(sizes), spread, bound(csr), spread / bound(csr)))
    assert spread <= bound(csr)


def test_budget_limits_admission():
    # an HBM budget that holds two of the six requests at once: the
    # scheduler admits them two at a time, and every result is correct
    P = pool()
    rg, csr = next((rg, csr) for rg, csr, cls in P if csr.name == "grid300x301")
    ex = serve.GpuExecutor.for_serving()
    fp = ex.footprint(serve.Request(0, rg, 0.0), "batch")
    reqs = [serve.Request(i, rg, 0.0) for i in range(6)]
    mix, s = run(reqs, hbm_budget=2 * fp + 1, small_edges=10**9)
    assert s.peak_in_use == 2 * fp  # the budget binds: never three at once
    assert len(mix) == 6
    assert len({c.launch for c in mix.values()}) >= 3
    for c in mix.values():
        assert oracle.check(csr, c.mate.cpu().numpy()).ok


def test_budget_limits_solo_admission():
    # solo jobs: a budget for one at a time serialises them even with two
    # free solo slots
    P = pool()
    rg, csr = next((rg, csr) for rg, csr, cls in P if csr.name.startswith("rmat18"))
    ex = serve.GpuExecutor.for_serving()
    fp = ex.footprint(serve.Request(0, rg, 0.0), "solo")
    # the footprint covers the workspace, the create call's own allocations
    # and the output
    import ctypes
    from paper_2507_04420_amd import _lib
    lib = _lib.load()
    ct = rg.tuning.to_c()
    assert fp >= (lib.mm_workspace_bytes_graph(csr.n, csr.m, ctypes.byref(ct))
                  + lib.mm_create_device_bytes(csr.n, csr.m, ctypes.byref(ct)) + 4 * csr.n)
    reqs = [serve.Request(i, rg, 0.0) for i in range(3)]
    mix, s = run(reqs, hbm_budget=fp + 1, small_edges=0)
    assert s.peak_in_use == fp
    assert {c.route for c in mix.values()} == {"solo"}
    for c in mix.values():
        assert oracle.check(csr, c.mate.cpu().numpy()).ok
