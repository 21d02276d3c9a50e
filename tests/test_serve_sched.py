"""Scheduling rules of the serving loop, on the CPU with a simulated
executor (launch durations are a function of the jobs; nothing touches a
device): arrival-order admission within the memory budget, small jobs
coalesced into the next free batch slot, large jobs on solo slots, every
request completed exactly once."""
import numpy as np
import pytest

from paper_2507_04420_amd.serve import Completion, Request, ResidentGraph, Scheduler, run_trace


class FakeExecutor:
    def __init__(self):
        self.now = 0.0
        self.launches = []
        self.live = 0
        self.peak_live = 0

    def footprint(self, req, route):
        return 8 * req.graph.n + 4096

    def launch(self, route, reqs, slot):
        dur = 1e-3 + 1e-9 * sum(r.graph.m for r in reqs)
        h = {"route": route, "reqs": [r.rid for r in reqs], "slot": slot, "end": self.now + dur}
        self.launches.append(h)
        self.live += 1
        self.peak_live = max(self.peak_live, self.live)
        return h

    def done(self, h):
        return self.now >= h["end"]

    def finish(self, h):
        self.live -= 1
        return [("mate", rid) for rid in h["reqs"]]


def graph(n, m):
    return ResidentGraph(None, None, n, m)


def drive(sched, ex, reqs, dt=1e-4):
    reqs = sorted(reqs, key=lambda r: r.arrival)
    i, t, done = 0, 0.0, 0
    seen_in_use = []
    while done < len(reqs):
        ex.now = t
        while i < len(reqs) and reqs[i].arrival <= t:
            sched.submit(reqs[i])
            i += 1
        done += sched.step(t)
        seen_in_use.append(sched.in_use)
        t += dt
        assert t < 100
    return seen_in_use


def test_every_request_completes_once_and_budget_holds():
    rng = np.random.default_rng(1)
    ex = FakeExecutor()
    budget = 8 * 3_000_000
    s = Scheduler(ex, hbm_budget=budget, small_edges=100_000, max_batch=16)
    reqs = []
    t = 0.0
    for rid in range(400):
        t += rng.exponential(1 / 2000)
        m = int(np.exp(rng.uniform(np.log(1e4), np.log(5e6))))
        reqs.append(Request(rid, graph(max(2, m // 8), m), t))
    in_use = drive(s, ex, reqs)
    assert max(in_use) <= budget and s.peak_in_use <= budget
    assert sorted(c.rid for c in s.completions) == list(range(400))
    assert s.in_use == 0 and not s.inflight
    for c in s.completions:
        assert c.arrival <= c.admitted <= c.launched <= c.done
        assert c.mate == ("mate", c.rid)
        route = "batch" if reqs[c.rid].graph.m <= 100_000 else "solo"
        assert c.route == route


def test_small_jobs_arriving_during_a_batch_join_the_next_launch():
    ex = FakeExecutor()
    s = Scheduler(ex, hbm_budget=1 << 40, small_edges=10**6, batch_slots=1, max_batch=100)
    # one job at t=0 occupies the only batch slot for ~1 ms + 1e-9*m s
    reqs = [Request(0, graph(1000, 900_000), 0.0)]
    reqs += [Request(k, graph(100, 1000), 1e-4 * k) for k in range(1, 6)]  # arrive while busy
    drive(s, ex, reqs)
    first, second = ex.launches[0], ex.launches[1]
    assert first["reqs"] == [0]
    assert second["reqs"] == [1, 2, 3, 4, 5]  # coalesced into one launch
    assert len(ex.launches) == 2


def test_batch_size_cap_and_parallel_slots():
    ex = FakeExecutor()
    s = Scheduler(ex, hbm_budget=1 << 40, small_edges=10**6, batch_slots=2, max_batch=3)
    reqs = [Request(k, graph(100, 1000), 0.0) for k in range(7)]
    drive(s, ex, reqs)
    sizes = [len(L["reqs"]) for L in ex.launches]
    assert sizes[:2] == [3, 3] and sum(sizes) == 7
    assert ex.peak_live == 2  # both batch slots were busy at once


def test_large_jobs_use_solo_slots_and_overlap():
    ex = FakeExecutor()
    s = Scheduler(ex, hbm_budget=1 << 40, small_edges=1000, solo_slots=2)
    reqs = [Request(k, graph(10**5, 10**6), 0.0) for k in range(3)]
    reqs.append(Request(3, graph(10, 100), 0.0))
    drive(s, ex, reqs)
    solo = [L for L in ex.launches if L["route"] == "solo"]
    assert len(solo) == 3 and {L["slot"] for L in solo} == {0, 1}
    assert ex.launches[0]["reqs"] == [0] and ex.launches[1]["reqs"] == [1]
    # the third solo job waits for a slot with its memory held; the small job
    # behind it needs no solo slot and is batched at once, ahead of it
    order = [L["reqs"] for L in ex.launches]
    assert order.index([3]) < order.index([2])
    c = {x.rid: x for x in s.completions}
    assert c[3].launched < c[2].launched


def test_waiting_solo_job_keeps_its_place_for_memory():
    # a large job waiting for a solo slot holds its memory: later small jobs
    # are admitted only into what is left, so they cannot starve it
    ex = FakeExecutor()
    fp_big = 8 * 100_000 + 4096
    budget = 3 * fp_big
    s = Scheduler(ex, hbm_budget=budget, small_edges=1000, solo_slots=1, batch_slots=4)
    reqs = [Request(0, graph(100_000, 10**6), 0.0), Request(1, graph(100_000, 10**6), 0.0)]
    reqs += [Request(2 + k, graph(50_000, 500), 1e-5) for k in range(10)]
    seen = drive(s, ex, reqs)
    assert max(seen) <= budget
    c = {x.rid: x for x in s.completions}
    # job 1 was admitted (memory granted) before any of the later small jobs
    assert all(c[1].admitted <= c[k].admitted for k in range(2, 12))


def test_head_of_line_blocks_on_memory():
    ex = FakeExecutor()
    budget = 8 * 200_000 + 4096 * 3
    s = Scheduler(ex, hbm_budget=budget, small_edges=10**9, batch_slots=4)
    reqs = [Request(0, graph(150_000, 10**6), 0.0),   # takes most of the budget
            Request(1, graph(100_000, 10**5), 1e-5),  # does not fit until 0 is done
            Request(2, graph(10, 100), 2e-5)]         # fits, but must not pass 1
    drive(s, ex, reqs)
    order = [rid for L in ex.launches for rid in L["reqs"]]
    assert order == [0, 1, 2]
    c = {x.rid: x for x in s.completions}
    assert c[1].admitted >= c[0].done and c[2].admitted >= c[1].admitted
    # request 1 waited for memory (counted once, however many rounds it waited)
    assert s.memory_waits == 1


def test_oversized_request_is_rejected():
    s = Scheduler(FakeExecutor(), hbm_budget=1000)
    with pytest.raises(ValueError):
        s.submit(Request(0, graph(10**6, 10), 0.0))


def test_run_trace_with_simulated_clock():
    ex = FakeExecutor()
    s = Scheduler(ex, hbm_budget=1 << 40, small_edges=10**6)
    clock = {"t": 0.0}

    def tick():
        clock["t"] += 5e-5
        ex.now = clock["t"]
        return clock["t"]

    reqs = [Request(k, graph(100, 1000), 1e-3 * k) for k in range(20)]
    comps, wall = run_trace(s, reqs, clock=tick)
    assert len(comps) == 20 and all(isinstance(c, Completion) for c in comps)
    assert wall > 0.019


def test_run_trace_freezes_the_collector_only_while_it_runs():
    # the objects alive at the start are out of the collector's view during
    # the trace (a full collection cannot stall the loop), and back after it,
    # also when the trace fails
    import gc
    ex = FakeExecutor()
    seen = []

    class Probe(Scheduler):
        def step(self, now):
            seen.append(gc.get_freeze_count())
            ex.now = now + 1.0
            return super().step(now)

    assert gc.get_freeze_count() == 0
    comps, _ = run_trace(Probe(ex, hbm_budget=1 << 40, small_edges=10**6),
                         [Request(k, graph(100, 1000), 0.0) for k in range(3)])
    assert len(comps) == 3 and min(seen) > 0 and gc.get_freeze_count() == 0
    seen.clear()
    run_trace(Probe(ex, hbm_budget=1 << 40, small_edges=10**6), [Request(0, graph(100, 1000), 0.0)],
              freeze_gc=False)
    assert max(seen) == 0

    class Stuck(Scheduler):
        def step(self, now):
            return 0

    clock = iter(range(10**6))
    with pytest.raises(TimeoutError):
        run_trace(Stuck(ex, hbm_budget=1 << 40, small_edges=10**6), [Request(0, graph(100, 1000), 0.0)],
                  clock=lambda: float(next(clock)), timeout=5.0)
    assert gc.get_freeze_count() == 0


def _lib_or_skip():
    from paper_2507_04420_amd import _lib
    return _lib.load()


def test_footprint_covers_a_relabelled_copy():
    # a relabel-tuned request holds the relabelled CSR (int64 offsets, the
    # id map, m ids) and its states in the workspace, plus its output
    import ctypes
    from paper_2507_04420_amd import Tuning
    from paper_2507_04420_amd.serve import request_footprint
    lib = _lib_or_skip()
    n, m = 100_000, 1_600_000
    t = Tuning(relabel=1)
    fp = request_footprint(lib, n, m, t, "solo")
    relabelled = 8 * (n + 1) + 4 * n + 4 * m + 4 * n   # offsets, map, ids, states
    assert fp >= relabelled + 4 * n
    # the create call's own temporaries (degree keys, sorted keys, inverse
    # map, degrees in new ids) are counted too
    ct = t.to_c()
    assert lib.mm_create_device_bytes(n, m, ctypes.byref(ct)) >= 20 * n
    assert fp >= lib.mm_workspace_bytes_graph(n, m, ctypes.byref(ct)) + 20 * n + 4 * n
    # the n-only size cannot know the copy: it reports 0, never too little
    assert lib.mm_workspace_bytes(n, ctypes.byref(ct)) == 0


def test_footprint_covers_a_reordered_copy():
    # a request tuned with reordered lists holds a copy of the ids, and the
    # create call allocates the neighbours' degree buckets
    import ctypes
    from paper_2507_04420_amd import Tuning
    from paper_2507_04420_amd.serve import request_footprint
    lib = _lib_or_skip()
    n, m = 100_000, 1_600_000
    t = Tuning(order_lists=1)
    fp = request_footprint(lib, n, m, t, "solo")
    base = lib.mm_workspace_bytes_graph(n, m, ctypes.byref(Tuning().to_c()))
    assert fp >= base + 4 * m + n + 4 * n


def test_solo_requests_build_no_copy(monkeypatch):
    # a serving request creates its handle and runs one pass: whatever its
    # class's stored entry says, it runs without a relabelled or reordered copy
    from paper_2507_04420_amd import Tuning, autotune, serve
    monkeypatch.setattr(autotune, "tuned", lambda cls, key=None: Tuning(relabel=1, order_lists=1))
    off = np.arange(0, 2 * 400_001, 2, dtype=np.int64)  # 400000 vertices of degree 2
    t = serve.solo_tuning(off)
    assert t.relabel == 0 and t.order_lists == 0


def test_footprint_covers_the_hub_table():
    # every list longer than hub_degree gives ceil(d / hub_chunk) pieces of
    # 24 bytes each, kept by the handle; the bound covers any degree sequence
    import ctypes
    import graphgen
    from paper_2507_04420_amd import Tuning
    from paper_2507_04420_amd.serve import request_footprint
    lib = _lib_or_skip()
    g = graphgen.rmat(16, seed=3)
    deg = np.diff(g.off)
    for hd, chunk in ((4096, 256), (64, 16), (8, 1)):
        t = Tuning(hub_degree=hd, hub_chunk=chunk, whole_graph_vertices=0)
        pieces = int(sum((d + chunk - 1) // chunk for d in deg if d > hd))
        ct = t.to_c()
        extra = lib.mm_create_device_bytes(g.n, g.m, ctypes.byref(ct))
        assert extra >= 24 * pieces, (hd, chunk, extra, pieces)
        fp = request_footprint(lib, g.n, g.m, t, "solo")
        assert fp >= lib.mm_workspace_bytes_graph(g.n, g.m, ctypes.byref(ct)) + 24 * pieces + 4 * g.n
    # no list can be long: nothing is allocated
    ct = Tuning(hub_degree=4096).to_c()
    assert lib.mm_create_device_bytes(1000, 4000, ctypes.byref(ct)) == 0


def test_batch_footprint_covers_items_and_pieces():
    import ctypes
    import graphgen
    from paper_2507_04420_amd import Tuning
    from paper_2507_04420_amd.serve import request_footprint
    lib = _lib_or_skip()
    g = graphgen.rmat(15, seed=4)
    deg = np.diff(g.off)
    t = Tuning(hub_degree=32, hub_chunk=8, whole_graph_vertices=0)
    pieces = int(sum((d + 7) // 8 for d in deg if d > 32))
    vtx = np.array([0, g.n], dtype=np.int64)
    ct = t.to_c()
    ws = lib.mm_batch_workspace_bytes(1, ctypes.c_void_p(vtx.ctypes.data), ctypes.byref(ct))
    extra = lib.mm_batch_create_device_bytes(1, ctypes.c_void_p(vtx.ctypes.data), g.m, ctypes.byref(ct))
    assert extra >= 24 * pieces + 16 * (pieces // 64)
    assert request_footprint(lib, g.n, g.m, t, "batch") == ws + extra + 256 + 4 * g.n
    # graphs swept whole get no pieces
    t2 = Tuning(hub_degree=32, hub_chunk=8, whole_graph_vertices=1 << 20)
    ct2 = t2.to_c()
    assert lib.mm_batch_create_device_bytes(1, ctypes.c_void_p(vtx.ctypes.data), g.m,
                                            ctypes.byref(ct2)) == 0


def test_two_phase_word_layout_rejects_the_sentinel_ids():
    # ACC = INT32_MAX and RSVD = INT32_MAX - 1 share the word with mate ids:
    # at most 2^31 - 2 vertices, so that no id equals RSVD
    import ctypes
    from paper_2507_04420_amd import Tuning, _lib
    lib = _lib_or_skip()
    two = Tuning(layout=_lib.MM_LAYOUT_U32, protocol=_lib.MM_PROTOCOL_TWO_PHASE).to_c()
    cas = Tuning(layout=_lib.MM_LAYOUT_U32, protocol=_lib.MM_PROTOCOL_CAS).to_c()
    big = (1 << 31) - 1
    assert lib.mm_workspace_bytes_graph(big, 0, ctypes.byref(two)) == 0
    assert lib.mm_workspace_bytes_graph(big - 1, 0, ctypes.byref(two)) > 0
    assert lib.mm_workspace_bytes_graph(big, 0, ctypes.byref(cas)) > 0
    h = ctypes.c_void_p()
    st = lib.mm_create(ctypes.c_void_p(256), _lib.MM_OFF_I64, ctypes.c_void_p(256), big, 0,
                       ctypes.c_void_p(256), 1 << 40, 0, ctypes.byref(two), None, ctypes.byref(h))
    assert st == _lib.MM_ERR_INVALID_ARG and not h.value
    assert b"2^31-2" in lib.mm_last_error()
