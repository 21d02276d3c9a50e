"""Serving loop: a stream of matching requests over graphs resident on the GPU.

A request names a resident graph (its CSR already in device memory) and asks
for a maximal matching of it. The server

* admits requests in arrival order while their device footprint (status
  words, hint bits, mate output and workspace; the CSR is already resident)
  fits the HBM budget, and, for large jobs, while a solo slot is free;
* coalesces admitted small jobs into list batches (one persistent launch over
  all of them, ``mm_batch_create_list``) that start as soon as a batch slot
  is free, so requests that arrive while earlier ones are on the GPU join the
  next launch (continuous batching);
* runs large jobs alone (``mm_create``/``mm_run``) on their own streams, where
  they overlap with the batches and with each other;
* retires launches as their completion events fire, releases their footprint
  and records arrival -> result-ready latency.

The scheduling core (:class:`Scheduler`) is independent of the device: it
drives an executor object, so its admission and batching rules are tested on
the CPU with a simulated executor; :class:`GpuExecutor` is the real one.
"""
from __future__ import annotations

import gc
import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import _lib


@dataclass
class ResidentGraph:
    """A graph whose CSR (int64 offsets, int32 neighbours) is on the device."""
    off: object
    nbr: object
    n: int
    m: int
    symmetric: bool = True
    name: str = ""
    tuning: object = None  # used when the graph runs alone (large jobs)

    @classmethod
    def from_tensors(cls, off, nbr, symmetric=True, name="", tuning=None):
        return cls(off, nbr, off.numel() - 1, nbr.numel(), symmetric, name, tuning)

    @classmethod
    def for_serving(cls, off, nbr, off_host, symmetric=True, name=""):
        """A resident graph that runs alone with its class's serving tuning
        (see solo_tuning); off_host: the offsets as a host array."""
        return cls.from_tensors(off, nbr, symmetric, name, solo_tuning(off_host))


def solo_tuning(off_host):
    """The tuning a large job runs alone with: the stored entry of its graph
    class (autotune.classify), without a relabelled or reordered copy of the
    graph. A request creates its own handle and runs one pass, and a copy
    built at create time pays off only for a handle that runs many. The
    classes a request can fall in below 2^25 vertices are tuned under the
    autotuner's spread limit (and without copies), so that a job's result
    alone and in the mix stay within the serving tolerance."""
    from . import autotune
    t = autotune.tuned(autotune.classify(np.asarray(off_host)))
    for field, value in autotune.COPIES.items():
        setattr(t, field, value)
    return t


def batch_tuning():
    """The tuning of the list batches small jobs are coalesced into: the
    stored batch entry, with the library's whole-graph threshold (a small
    graph's result must not depend on the jobs it shares a launch with) and
    lanes that release u while they wait (a serving batch holds a few jobs,
    all of whose vertices are swept at once, so that no chain of waiting
    holders forms)."""
    from . import Tuning, autotune
    t = autotune.tuned("batch")
    t.whole_graph_vertices = Tuning().whole_graph_vertices
    t.wait_release = 1
    return t


def request_footprint(lib, n: int, m: int, tuning, route: str) -> int:
    """Device bytes a request holds while admitted: its mate output, the
    workspace it alone would need (with the relabelled copy when the tuning
    asks for one) and everything the create call allocates by itself (hub
    piece table, relabelling temporaries; batches: item and piece tables),
    as upper bounds the library reports. The CSR is already resident."""
    ct = tuning.to_c()
    if route == "solo":
        ws = lib.mm_workspace_bytes_graph(n, m, _byref(ct))
        extra = lib.mm_create_device_bytes(n, m, _byref(ct))
    else:
        vtx = np.array([0, n], dtype=np.int64)
        ws = lib.mm_batch_workspace_bytes(1, _ptr(vtx), _byref(ct))
        extra = lib.mm_batch_create_device_bytes(1, _ptr(vtx), m, _byref(ct))
    if ws == 0:
        raise ValueError("the library rejects n=%d, m=%d under this tuning" % (n, m))
    # + the 256 bytes the binding adds to align the workspace
    return int(ws) + int(extra) + 256 + 4 * n


@dataclass
class Request:
    rid: int
    graph: ResidentGraph
    arrival: float  # seconds from the start of the trace


@dataclass
class Completion:
    rid: int
    route: str          # "batch" or "solo"
    launch: int         # id of the launch that served the request
    arrival: float
    admitted: float
    launched: float
    done: float
    mate: object = None  # int32 device tensor of n local mates (kept if asked)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class _Launch:
    lid: int
    route: str
    reqs: list
    slot: int
    handle: object
    launched: float
    footprint: int


@dataclass
class Scheduler:
    """Admission, continuous batching and retirement over an executor.

    executor must provide footprint(req, route) -> bytes,
    launch(route, reqs, slot) -> handle, done(handle) -> bool and
    finish(handle) -> list of per-request mates (or Nones).
    """
    executor: object
    hbm_budget: int
    small_edges: int = 2_000_000
    max_batch: int = 1024
    batch_slots: int = 2
    solo_slots: int = 2
    keep_results: bool = True
    pending: deque = field(default_factory=deque)   # arrived, not admitted
    ready: deque = field(default_factory=deque)     # admitted small jobs awaiting a batch
    solo_ready: deque = field(default_factory=deque)  # admitted large jobs awaiting a solo slot
    inflight: list = field(default_factory=list)
    completions: list = field(default_factory=list)
    in_use: int = 0
    peak_in_use: int = 0
    memory_waits: int = 0   # requests that waited at the head for memory to free up
    _admit_time: dict = field(default_factory=dict)
    _blocked: int = -1      # the request last counted in memory_waits
    _fp: dict = field(default_factory=dict)
    _free_batch: list = None
    _free_solo: list = None
    _next_lid: int = 0

    def __post_init__(self):
        self._free_batch = list(range(self.batch_slots))
        self._free_solo = list(range(self.solo_slots))

    def route(self, req) -> str:
        return "batch" if req.graph.m <= self.small_edges else "solo"

    def submit(self, req) -> None:
        fp = self.executor.footprint(req, self.route(req))
        if fp > self.hbm_budget:
            raise ValueError("request %d needs %d bytes, more than the whole budget" % (req.rid, fp))
        self._fp[req.rid] = fp
        self.pending.append(req)

    def idle(self) -> bool:
        return not (self.pending or self.ready or self.solo_ready or self.inflight)

    def step(self, now: float) -> int:
        """One scheduling round; returns the number of requests completed."""
        done = self._retire(now)
        self._admit(now)
        self._launch_solos(now)
        self._launch_batches(now)
        return done

    def _retire(self, now):
        count = 0
        still = []
        for L in self.inflight:
            if not self.executor.done(L.handle):
                still.append(L)
                continue
            mates = self.executor.finish(L.handle)
            for r, mt in zip(L.reqs, mates):
                self.completions.append(Completion(
                    r.rid, L.route, L.lid, r.arrival, self._admit_time.pop(r.rid), L.launched, now,
                    mt if self.keep_results else None))
                count += 1
            self.in_use -= L.footprint
            (self._free_batch if L.route == "batch" else self._free_solo).append(L.slot)
        self.inflight = still
        return count

    def _admit(self, now):
        # memory is granted in strict arrival order: a request that does not
        # fit blocks those behind it, so a large job is never starved by a
        # stream of small ones. A large job that fits waits for a solo slot
        # with its memory held, and the small jobs behind it, which need no
        # solo slot, go on into batches
        while self.pending:
            r = self.pending[0]
            fp = self._fp[r.rid]
            if self.in_use + fp > self.hbm_budget:
                if r.rid != self._blocked:
                    self.memory_waits += 1
                    self._blocked = r.rid
                break
            self.pending.popleft()
            self.in_use += fp
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            self._admit_time[r.rid] = now
            if self.route(r) == "solo":
                self.solo_ready.append(r)
            else:
                self.ready.append(r)

    def _launch_solos(self, now):
        while self.solo_ready and self._free_solo:
            r = self.solo_ready.popleft()
            slot = self._free_solo.pop(0)
            self._start("solo", [r], slot, now, self._fp[r.rid])

    def _launch_batches(self, now):
        while self.ready and self._free_batch:
            take = []
            while self.ready and len(take) < self.max_batch:
                take.append(self.ready.popleft())
            slot = self._free_batch.pop(0)
            self._start("batch", take, slot, now, sum(self._fp[r.rid] for r in take))

    def _start(self, route, reqs, slot, now, fp):
        h = self.executor.launch(route, reqs, slot)
        self.inflight.append(_Launch(self._next_lid, route, reqs, slot, h, now, fp))
        self._next_lid += 1
        for r in reqs:
            del self._fp[r.rid]


class GpuExecutor:
    """Runs launches through the library: list batches for small jobs, one
    graph handle per large job, each slot on its own stream."""

    def __init__(self, batch_slots=2, solo_slots=2, tuning_batch=None, tuning_solo=None,
                 device="cuda"):
        import torch
        from . import Batch, Graph, Tuning  # noqa: F401
        self.torch = torch
        self.device = torch.device(device)
        self.batch_streams = [torch.cuda.Stream(device=self.device) for _ in range(batch_slots)]
        self.solo_streams = [torch.cuda.Stream(device=self.device) for _ in range(solo_slots)]
        self.tuning_batch = tuning_batch if tuning_batch is not None else Tuning.default()
        self.tuning_solo = tuning_solo if tuning_solo is not None else Tuning.default()
        self._lib = _lib.load()

    @classmethod
    def for_serving(cls, batch_slots=2, solo_slots=2, device="cuda") -> "GpuExecutor":
        """The executor the serving benchmark runs: batch_tuning() for the
        batches; large jobs run with their graph's own tuning
        (ResidentGraph.for_serving)."""
        return cls(batch_slots, solo_slots, tuning_batch=batch_tuning(), device=device)

    def footprint(self, req, route) -> int:
        """See request_footprint."""
        t = (req.graph.tuning or self.tuning_solo) if route == "solo" else self.tuning_batch
        return request_footprint(self._lib, req.graph.n, req.graph.m, t, route)

    def launch(self, route, reqs, slot):
        from . import Batch, Graph
        torch = self.torch
        if route == "solo":
            r = reqs[0]
            s = self.solo_streams[slot]
            with torch.cuda.stream(s):
                g = Graph(r.graph.off, r.graph.nbr, symmetric=r.graph.symmetric,
                          tuning=r.graph.tuning or self.tuning_solo, stream=s)
                out = torch.empty(r.graph.n, dtype=torch.int32, device=self.device)
                g.run(out, stream=s)
                ev = torch.cuda.Event()
                ev.record(s)
            return ("solo", g, out, ev, s, None)
        s = self.batch_streams[slot]
        sym = all(r.graph.symmetric for r in reqs)
        with torch.cuda.stream(s):
            b = Batch.from_list([(r.graph.off, r.graph.nbr) for r in reqs], symmetric=sym,
                                tuning=self.tuning_batch, stream=s)
            out = torch.empty(b.N, dtype=torch.int32, device=self.device)
            b.run(out, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        return ("batch", b, out, ev, s, b.vtx_off)

    def done(self, h) -> bool:
        return h[3].query()

    def finish(self, h):
        kind, obj, out, ev, s, vtx = h
        obj.sync(stream=s)  # raises if a wavefront ran out of its loop budget
        obj.close()
        if kind == "solo":
            return [out]
        return [out[int(vtx[g]):int(vtx[g + 1])] for g in range(len(vtx) - 1)]


def _byref(ct):
    import ctypes
    return ctypes.byref(ct)


def _ptr(a):
    import ctypes
    return ctypes.c_void_p(a.ctypes.data)


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of `rate` requests per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def run_trace(scheduler: Scheduler, requests, clock=time.perf_counter, timeout: float = 120.0,
              freeze_gc: bool = True):
    """Feeds requests to the scheduler at their arrival times (real time) and
    steps it until every request completed. Returns (completions, wall s).

    freeze_gc: the objects alive when the trace starts (the resident graphs,
    the requests, torch's and numpy's own) are moved out of the cyclic
    garbage collector's view until it ends (gc.freeze). A full collection
    otherwise walks every object of the process, about 45 ms with the bench's
    pool, and the loop stands still meanwhile: at 2000 req/s one such pause
    delays some 80 requests by 40 ms, which alone sets the p99."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    if freeze_gc:
        gc.freeze()
    try:
        t0 = clock()
        i = 0
        total = len(reqs)
        done = 0
        while done < total:
            now = clock() - t0
            while i < total and reqs[i].arrival <= now:
                scheduler.submit(reqs[i])
                i += 1
            done += scheduler.step(now)
            if now > timeout:
                raise TimeoutError("trace did not finish in %.0f s (%d of %d done)" % (
                    timeout, done, total))
        return scheduler.completions, clock() - t0
    finally:
        if freeze_gc:
            gc.unfreeze()


def summarize(completions, wall: float, edges: int) -> dict:
    lat = np.array([c.latency for c in completions]) * 1e3
    batches = {c.launch for c in completions if c.route == "batch"}
    per_batch = len([c for c in completions if c.route == "batch"]) / max(1, len(batches))
    return {"requests": len(completions),
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else math.nan,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else math.nan,
            "mean_ms": float(lat.mean()) if len(lat) else math.nan,
            "req_per_s": len(completions) / wall if wall > 0 else math.nan,
            "gedges_per_s": edges / wall / 1e9 if wall > 0 else math.nan,
            "batch_launches": len(batches),
            "mean_jobs_per_batch": per_batch,
            "solo_launches": len([c for c in completions if c.route == "solo"]),
            "wall_s": wall}
