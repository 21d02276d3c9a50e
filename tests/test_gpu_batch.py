"""GPU parity of the batched path (one persistent launch over many graphs).

Every member graph's slice of the output is checked against the oracle on
that graph alone; graphs with a unique maximal matching must match exactly.
The hipGraph-captured pass is replayed several times with host work and
synchronisation in between, and every replay is checked.
"""
import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2507_04420_amd as mm  # noqa: E402
from paper_2507_04420_amd import _lib  # noqa: E402

TUNINGS = {
    "u8_cas": mm.Tuning(layout=_lib.MM_LAYOUT_U8, lazy_init=0),
    "u32_cas": mm.Tuning(),
    "u2_two_hint": mm.Tuning(layout=_lib.MM_LAYOUT_U2, protocol=_lib.MM_PROTOCOL_TWO_PHASE, hint=1,
                             lazy_init=1),
    "u32_two_lazy": mm.Tuning(layout=_lib.MM_LAYOUT_U32, protocol=_lib.MM_PROTOCOL_TWO_PHASE,
                              lazy_init=1),
    "u8_small": mm.Tuning(layout=_lib.MM_LAYOUT_U8, wave_vertices=64, wg_size=64, assist_after=2,
                          lazy_init=1),
    "u32_bytehint": mm.Tuning(hint=2, whole_graph_vertices=0),
    "u32_whole_in_device_memory": mm.Tuning(whole_graph_lds=0),
    "u32_mesh128": mm.Tuning(whole_graph_vertices=0, mesh_wave_vertices=128),
    "u32_upper_only": mm.Tuning(upper_only=1, whole_graph_vertices=0, hint=2),
    "u32_probe_first_upper": mm.Tuning(probe_first=1, upper_only=1, whole_graph_vertices=0),
    "u32_hub_wave": mm.Tuning(hub_wave=1, hub_degree=6, hub_chunk=65, whole_graph_vertices=0),
    # the workgroup tier is taken as the wavefront tier in batches
    "u32_hub_group": mm.Tuning(hub_wave=2, hub_degree=5, hub_chunk=7, whole_graph_vertices=0,
                               wg_size=256),
    "u2_two_hub_wave_upper": mm.Tuning(hub_wave=1, hub_degree=3, hub_chunk=5, layout=_lib.MM_LAYOUT_U2,
                                       protocol=_lib.MM_PROTOCOL_TWO_PHASE, upper_only=1,
                                       whole_graph_vertices=0),
    "u8_upper_only_lazy_hubs": mm.Tuning(upper_only=1, layout=_lib.MM_LAYOUT_U8, lazy_init=1,
                                         hub_degree=6, hub_chunk=3, hub_wave=0),
    "u8_mesh64_hubs": mm.Tuning(layout=_lib.MM_LAYOUT_U8, whole_graph_vertices=0, mesh_wave_vertices=64,
                                hub_degree=8, hub_chunk=4, lazy_init=1),
    "u32_mesh128_wait_release": mm.Tuning(whole_graph_vertices=0, mesh_wave_vertices=128,
                                          wait_release=1),
    "u2_two_whole_lds_wg64": mm.Tuning(layout=_lib.MM_LAYOUT_U2, protocol=_lib.MM_PROTOCOL_TWO_PHASE,
                                       wg_size=64),
}


def check_members(mix, mate):
    for g in range(mix.num_graphs):
        v0, v1 = int(mix.vtx_off[g]), int(mix.vtx_off[g + 1])
        sub = mix.member(g)
        c = oracle.check(sub, mate[v0:v1])
        assert c.violations == 0, (g, c)
        assert 2 * c.size >= oracle.sgmm(sub).pairs


def mixture_small(G=40, seed=3):
    return graphgen.mixture(G, seed=seed, nmin=50, nmax=5000)


@pytest.mark.parametrize("name", sorted(TUNINGS))
def test_batch_mixture(name):
    mix = mixture_small()
    off = torch.from_numpy(mix.off).cuda()
    nbr = torch.from_numpy(mix.nbr).cuda()
    b = mm.Batch(off, nbr, mix.vtx_off, symmetric=True, validate=True, tuning=TUNINGS[name])
    out = b.run()
    b.sync()
    check_members(mix, out.cpu().numpy())


@pytest.mark.parametrize("name", ["u8_cas", "u2_two_hint"])
def test_batch_capture_replays(name):
    mix = mixture_small(G=30, seed=5)
    off = torch.from_numpy(mix.off).cuda()
    nbr = torch.from_numpy(mix.nbr).cuda()
    b = mm.Batch(off, nbr, mix.vtx_off, symmetric=True, capture=True, tuning=TUNINGS[name])
    out = torch.empty(mix.n, dtype=torch.int32, device="cuda")
    for rep in range(4):
        out.fill_(12345)  # eager work between replays
        b.run(out)
        b.sync()
        torch.cuda.synchronize()
        check_members(mix, out.cpu().numpy())
    # a second output buffer re-binds and re-captures
    out2 = b.run()
    b.sync()
    check_members(mix, out2.cpu().numpy())


def test_batch_unique_results_and_edge_cases():
    # members: disjoint edges (unique), isolated vertices, a single vertex,
    # an empty graph (0 vertices), a triangle
    parts = [graphgen.from_edges(8, [(0, 1), (2, 3), (4, 5), (6, 7)]),
             graphgen.from_edges(5, np.zeros((0, 2))),
             graphgen.from_edges(1, np.zeros((0, 2))),
             graphgen.from_edges(0, np.zeros((0, 2))),
             graphgen.from_edges(3, [(0, 1), (1, 2), (0, 2)])]
    vtx = np.cumsum([0] + [p.n for p in parts])
    eoff = np.cumsum([0] + [p.m for p in parts])
    off = np.concatenate([p.off[:-1] + eoff[k] for k, p in enumerate(parts)] + [[eoff[-1]]]).astype(np.int64)
    nbr = np.concatenate([p.nbr for p in parts]).astype(np.int32)
    b = mm.Batch(torch.from_numpy(off).cuda(), torch.from_numpy(nbr).cuda(), vtx, symmetric=True,
                 validate=True)
    mate = b.run().cpu().numpy()
    b.sync()
    np.testing.assert_array_equal(mate[0:8], np.arange(8) ^ 1)
    np.testing.assert_array_equal(mate[8:14], -1)
    tri = mate[14:17]
    assert sorted(tri.tolist()).count(-1) == 1 and oracle.check(parts[4], tri).ok


def test_batch_matches_single_graph_path():
    # the same graph alone through mm_run and inside a batch: both maximal,
    # sizes within the alone-vs-mix tolerance
    g = graphgen.rmat(14, seed=9)
    mix = graphgen.concat([(graphgen.KIND_ER, 3000, 6.0)] * 3, seed=2)
    parts = [g, mix.member(0), mix.member(1)]
    vtx = np.cumsum([0] + [p.n for p in parts])
    eoff = np.cumsum([0] + [p.m for p in parts])
    off = np.concatenate([p.off[:-1] + eoff[k] for k, p in enumerate(parts)] + [[eoff[-1]]]).astype(np.int64)
    nbr = np.concatenate([p.nbr for p in parts]).astype(np.int32)
    b = mm.Batch(torch.from_numpy(off).cuda(), torch.from_numpy(nbr).cuda(), vtx, symmetric=True)
    bm = b.run().cpu().numpy()
    b.sync()
    alone = mm.maximal_matching(torch.from_numpy(g.off).cuda(), torch.from_numpy(g.nbr).cuda(),
                                symmetric=True).cpu().numpy()
    c1, c2 = oracle.check(g, bm[:g.n]), oracle.check(g, alone)
    assert c1.ok and c2.ok
    assert abs(c1.size - c2.size) <= max(2, 0.01 * oracle.sgmm(g).pairs)


def test_batch_validate_rejects_foreign_ids():
    off = torch.tensor([0, 1, 2, 3], dtype=torch.int64, device="cuda")
    nbr = torch.tensor([1, 0, 2], dtype=torch.int32, device="cuda")  # graph 1 has one vertex: id 2 is foreign
    with pytest.raises(mm.MMError) as ei:
        mm.Batch(off, nbr, [0, 2, 3], validate=True)
    assert ei.value.status == _lib.MM_ERR_INVALID_GRAPH


def test_batch_stats():
    mix = mixture_small(G=12, seed=8)
    b = mm.Batch(torch.from_numpy(mix.off).cuda(), torch.from_numpy(mix.nbr).cuda(), mix.vtx_off,
                 symmetric=True, stats=True)
    out = b.run()
    b.sync()
    st = b.stats()
    mate = out.cpu().numpy()
    check_members(mix, mate)
    assert st["sources"] == mix.n
    assert st["pairs"] == int((mate >= 0).sum()) // 2


def list_of(parts):
    return [(torch.from_numpy(p.off.astype(np.int64)).cuda(), torch.from_numpy(p.nbr).cuda())
            for p in parts]


@pytest.mark.parametrize("name", ["u32_cas", "u8_cas", "u2_two_hint"])
def test_list_batch_mixture(name):
    mix = mixture_small(G=30, seed=12)
    parts = [mix.member(g) for g in range(mix.num_graphs)]
    b = mm.Batch.from_list(list_of(parts), symmetric=True, validate=True, tuning=TUNINGS[name])
    np.testing.assert_array_equal(b.vtx_off, mix.vtx_off)
    out = b.run()
    b.sync()
    check_members(mix, out.cpu().numpy())
    assert b.check(out)["ok"]


def test_list_batch_edge_cases_and_capture():
    parts = [graphgen.from_edges(8, [(0, 1), (2, 3), (4, 5), (6, 7)]),
             graphgen.from_edges(0, np.zeros((0, 2))),
             graphgen.from_edges(5, np.zeros((0, 2))),
             graphgen.from_edges(3, [(0, 1), (1, 2), (0, 2)]),
             graphgen.rmat(12, seed=4)]
    b = mm.Batch.from_list(list_of(parts), symmetric=True, validate=True, capture=True)
    out = torch.empty(b.N, dtype=torch.int32, device="cuda")
    for rep in range(3):
        out.fill_(-77)
        b.run(out)
        b.sync()
        torch.cuda.synchronize()
        mate = out.cpu().numpy()
        np.testing.assert_array_equal(mate[0:8], np.arange(8) ^ 1)
        np.testing.assert_array_equal(mate[8:13], -1)
        v = b.vtx_off
        for g, p in enumerate(parts):
            assert oracle.check(p, mate[v[g]:v[g + 1]]).ok, (rep, g)


def test_empty_list_batch():
    b = mm.Batch.from_list([], symmetric=True)
    assert b.N == 0 and b.items == 0
    b.run(torch.empty(0, dtype=torch.int32, device="cuda"))
    b.sync()


@pytest.mark.parametrize("bad", ["foreign_id", "offsets_end", "offsets_start"])
def test_list_batch_validate_rejects(bad):
    good = graphgen.from_edges(4, [(0, 1), (2, 3)])
    off = good.off.astype(np.int64).copy()
    nbr = good.nbr.copy()
    if bad == "foreign_id":
        nbr[1] = 4
    elif bad == "offsets_end":
        off[-1] -= 1
    else:
        off[0] = 1
    parts = [(torch.from_numpy(good.off.astype(np.int64)).cuda(), torch.from_numpy(good.nbr).cuda()),
             (torch.from_numpy(off).cuda(), torch.from_numpy(nbr).cuda())]
    with pytest.raises(mm.MMError) as ei:
        mm.Batch.from_list(parts, validate=True)
    assert ei.value.status == _lib.MM_ERR_INVALID_GRAPH


def test_batch_validate_rejects_offsets_beyond_m():
    # offsets that point past the neighbour array are reported, never followed
    off = torch.tensor([0, 5000000, 2, 3], dtype=torch.int64, device="cuda")
    nbr = torch.tensor([1, 0, 0], dtype=torch.int32, device="cuda")
    with pytest.raises(mm.MMError) as ei:
        mm.Batch(off, nbr, [0, 2, 3], validate=True)
    assert ei.value.status == _lib.MM_ERR_INVALID_GRAPH


def test_batch_rejects_relabel():
    mix = mixture_small(G=3, seed=1)
    with pytest.raises(mm.MMError) as ei:
        mm.Batch(torch.from_numpy(mix.off).cuda(), torch.from_numpy(mix.nbr).cuda(), mix.vtx_off,
                 tuning=mm.Tuning(relabel=1))
    assert ei.value.status in (_lib.MM_ERR_UNSUPPORTED, _lib.MM_ERR_INVALID_ARG)


def hub_trap(k):
    pairs = np.stack([np.arange(0, 2 * k, 2), np.arange(1, 2 * k, 2)], 1)
    hub = np.stack([np.full(2 * k, 2 * k), np.arange(2 * k)], 1)
    return graphgen.from_edges(2 * k + 1, np.concatenate([pairs, hub]))


@pytest.mark.parametrize("tuning", [mm.Tuning(whole_graph_vertices=0),
                                    mm.Tuning(hub_degree=3, hub_chunk=2, whole_graph_vertices=0),
                                    mm.Tuning(hub_degree=3, hub_chunk=2, layout=_lib.MM_LAYOUT_U8,
                                              lazy_init=1),
                                    mm.Tuning(hub_degree=0)])
def test_batch_hub_pieces(tuning):
    # hub traps and mixture members in one batch, captured and replayed
    parts = [hub_trap(20_000), mixture_small(G=1, seed=31).member(0), hub_trap(300),
             graphgen.rmat(13, seed=2)]
    b = mm.Batch.from_list(list_of(parts), symmetric=True, capture=True, tuning=tuning)
    out = torch.empty(b.N, dtype=torch.int32, device="cuda")
    for rep in range(2):
        out.fill_(-9)
        b.run(out)
        b.sync()
        torch.cuda.synchronize()
        mate = out.cpu().numpy()
        v = b.vtx_off
        for g, p in enumerate(parts):
            assert oracle.check(p, mate[v[g]:v[g + 1]]).ok, (rep, g)
    st_b = mm.Batch.from_list(list_of(parts), symmetric=True, stats=True, tuning=tuning)
    st_b.run()
    st_b.sync()
    assert st_b.stats()["sources"] == b.N


def test_batch_hub_pieces_are_fast():
    import time
    parts = [hub_trap(100_000)]
    for name, t in (("tier", mm.Tuning(whole_graph_vertices=0, hub_wave=0)),
                    ("wave_tier", mm.Tuning(whole_graph_vertices=0, hub_wave=1)),
                    ("no_tier", mm.Tuning(whole_graph_vertices=0, hub_degree=0))):
        b = mm.Batch.from_list(list_of(parts), symmetric=True, tuning=t)
        out = b.run()
        b.sync()
        t0 = time.perf_counter()
        b.run(out)
        b.sync()
        dt = time.perf_counter() - t0
        assert oracle.check(parts[0], out.cpu().numpy()).ok
        print("batch hub trap", name, "%.3f ms" % (dt * 1e3))
        if name != "no_tier":
            tier = max(dt, tier if name == "wave_tier" else 0.0)
        else:
            assert tier * 3 < dt


LDS_CASES = [
    mm.Tuning(),
    mm.Tuning(layout=_lib.MM_LAYOUT_U8, lazy_init=1),
    mm.Tuning(layout=_lib.MM_LAYOUT_U2, protocol=_lib.MM_PROTOCOL_TWO_PHASE),
    mm.Tuning(protocol=_lib.MM_PROTOCOL_TWO_PHASE, lazy_init=1, hint=1),
]


@pytest.mark.parametrize("case", range(len(LDS_CASES)))
def test_whole_graph_lds_same_alone_as_in_batch(case):
    # graphs swept whole keep their states in LDS, in a batch and alone; the
    # result depends on the graph and the tuning only: a batch member's slice
    # equals the graph matched alone (mm_run), element by element
    t = LDS_CASES[case]
    mix = graphgen.mixture(24, seed=11 + case, nmin=60, nmax=9000)
    assert int(np.diff(mix.vtx_off).max()) <= t.whole_graph_vertices
    off = torch.from_numpy(mix.off).cuda()
    nbr = torch.from_numpy(mix.nbr).cuda()
    b = mm.Batch(off, nbr, mix.vtx_off, symmetric=True, validate=True, tuning=t)
    assert b.items == mix.num_graphs
    out = b.run()
    b.sync()
    mate = out.cpu().numpy()
    check_members(mix, mate)
    for g in range(mix.num_graphs):
        sub = mix.member(g)
        gg = mm.Graph(torch.from_numpy(sub.off).cuda(), torch.from_numpy(sub.nbr).cuda(),
                      symmetric=True, tuning=t)
        alone = gg.run()
        gg.sync()
        gg.close()
        v0, v1 = int(mix.vtx_off[g]), int(mix.vtx_off[g + 1])
        np.testing.assert_array_equal(mate[v0:v1], alone.cpu().numpy(), err_msg=sub.name)


def test_whole_graph_lds_largest_and_beyond():
    # a member at the LDS limit (16384 vertices) and one just above it (swept
    # whole from device memory), beside small ones; alone and in the batch
    t = mm.Tuning(whole_graph_vertices=20000)
    parts = [graphgen.grid(128, 128), graphgen.grid(128, 129), graphgen.er(3000, 6, seed=2),
             graphgen.from_edges(3, [(0, 1), (1, 2)])]
    assert parts[0].n == 16384 and parts[1].n == 16512
    dev = [(torch.from_numpy(p.off.astype(np.int64)).cuda(), torch.from_numpy(p.nbr).cuda())
           for p in parts]
    b = mm.Batch.from_list(dev, symmetric=True, validate=True, tuning=t)
    out = b.run()
    b.sync()
    mate = out.cpu().numpy()
    for k, p in enumerate(parts):
        v0, v1 = int(b.vtx_off[k]), int(b.vtx_off[k + 1])
        c = oracle.check(p, mate[v0:v1])
        assert c.violations == 0, (k, c)
        g = mm.Graph(dev[k][0], dev[k][1], symmetric=True, tuning=t)
        alone = g.run()
        g.sync()
        g.close()
        np.testing.assert_array_equal(mate[v0:v1], alone.cpu().numpy(), err_msg=str(k))


def test_mesh_members_get_short_blocks():
    # a grid member (no list longer than 4) is cut into mesh_wave_vertices
    # blocks, the others into wave_vertices blocks (the batch is large enough
    # that neither is shortened for size)
    parts = [graphgen.grid(512, 512), graphgen.er(20000, 8, seed=4)]
    dev = [(torch.from_numpy(p.off.astype(np.int64)).cuda(), torch.from_numpy(p.nbr).cuda())
           for p in parts]
    base = dict(whole_graph_vertices=0, wave_vertices=64)
    counts = {}
    for mesh in (0, 128):
        b = mm.Batch.from_list(dev, symmetric=True, validate=True,
                               tuning=mm.Tuning(**base, mesh_wave_vertices=mesh))
        out = b.run()
        b.sync()
        mate = out.cpu().numpy()
        for k, p in enumerate(parts):
            c = oracle.check(p, mate[int(b.vtx_off[k]):int(b.vtx_off[k + 1])])
            assert c.violations == 0, (mesh, k, c)
        counts[mesh] = b.items
        b.close()
    er_blocks = (20000 + 63) // 64
    assert counts[0] == 512 * 512 // 64 + er_blocks
    assert counts[128] == 512 * 512 // 128 + er_blocks


def test_small_batch_gets_short_blocks():
    # too few sources for min_waves = 2048 wavefronts of wave_vertices: blocks of 64
    parts = [graphgen.er(20000, 8, seed=5), graphgen.rmat(14, 8, seed=5)]
    dev = [(torch.from_numpy(p.off.astype(np.int64)).cuda(), torch.from_numpy(p.nbr).cuda())
           for p in parts]
    b = mm.Batch.from_list(dev, symmetric=True, validate=True,
                           tuning=mm.Tuning(whole_graph_vertices=0, wave_vertices=2048,
                                            min_waves=2048))
    assert b.items == sum((p.n + 63) // 64 for p in parts)
    out = b.run()
    b.sync()
    mate = out.cpu().numpy()
    for k, p in enumerate(parts):
        c = oracle.check(p, mate[int(b.vtx_off[k]):int(b.vtx_off[k + 1])])
        assert c.violations == 0, (k, c)
    b.close()


def test_small_batch_keeps_about_min_waves_wavefronts():
    # the default min_waves = 32: the 36384 blocked sources take blocks of
    # 1152 (about 32 wavefronts), not of 64
    parts = [graphgen.er(20000, 8, seed=5), graphgen.rmat(14, 8, seed=5)]
    dev = [(torch.from_numpy(p.off.astype(np.int64)).cuda(), torch.from_numpy(p.nbr).cuda())
           for p in parts]
    t = mm.Tuning(whole_graph_vertices=0, wave_vertices=2048)
    assert t.min_waves == 32
    b = mm.Batch.from_list(dev, symmetric=True, validate=True, tuning=t)
    blocked = sum(p.n for p in parts)
    w = (blocked // 32 + 63) // 64 * 64
    assert w == 1152
    assert b.items == sum((p.n + w - 1) // w for p in parts)
    out = b.run()
    b.sync()
    mate = out.cpu().numpy()
    for k, p in enumerate(parts):
        c = oracle.check(p, mate[int(b.vtx_off[k]):int(b.vtx_off[k + 1])])
        assert c.violations == 0, (k, c)
    b.close()
