"""Autotuner for the sweep's launch and layout parameters.

The matching itself has no parameters; what is tuned is how the sweep maps to
the device: the status layout and reservation protocol, degree relabelling
(single graphs), the matched hint (none, bits, bytes), vertices per wavefront
item (and, in batches, per mesh-like member), workgroup size, the list
length after which a wavefront scans one source together, the per-lane scan
width, lazy output, and whether a lane releases u while it waits for v. A
coordinate search starts from the stored entry (or the library defaults) and,
dimension by dimension, keeps the fastest value; every candidate's output must
pass the device check (zero violations) or the candidate is discarded.

Results are stored as JSON keyed by GPU architecture and compute-unit count,
then by graph class ("rmat", "grid", "er", and "rmat_mid", "grid_mid" for
grid and R-MAT graphs below MID_VERTICES, for single graphs; "batch" for
many-graph batches), and read back with :func:`tuned`.

    python -m paper_2507_04420_amd.autotune --classes batch,rmat --out tuned.json
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import Batch, Graph, Tuning, _lib

TUNED_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned")

# Values tried per dimension; the layout and protocol move together.
SPACE = {
    "layout_protocol": [(_lib.MM_LAYOUT_U32, _lib.MM_PROTOCOL_CAS),
                        (_lib.MM_LAYOUT_U8, _lib.MM_PROTOCOL_CAS),
                        (_lib.MM_LAYOUT_U2, _lib.MM_PROTOCOL_TWO_PHASE),
                        (_lib.MM_LAYOUT_U32, _lib.MM_PROTOCOL_TWO_PHASE)],
    "relabel": [0, 1, 2],
    "order_lists": [0, 1, 2],
    "probe_first": [0, 1, 2],
    "occupancy": [0, 6],
    "hot_degree": [512, 1024, 2048, 4096, 8192],
    "hint": [0, 1, 2],
    "disperse": [0, 1],
    "wave_vertices": [64, 128, 256, 512, 1024, 2048, 4096],
    "wg_size": [64, 128, 256],
    "assist_after": [16, 32, 64, 128, 256],
    "scan_width": [2, 3, 4],
    "lazy_init": [0, 1],
    "whole_graph_vertices": [0, 4096, 16384],
    "mesh_wave_vertices": [0, 128, 256, 512],
    # each edge from its lower end only, and waiting without holding u: on a
    # mesh the first needs the second (every lane would otherwise hold its
    # source while waiting for the next vertex of its row), so they move
    # together
    "upper_wait": [(0, 0), (0, 1), (1, 0), (1, 1)],
    "min_waves": [4, 8, 16, 32, 64, 2048, 16384],
    "hub_wave": [0, 1, 2],
    "hub_chunk": [64, 256, 1024, 4096],
}

# Costs outside the pass: relabelling keeps a second copy of the graph in the
# workspace and rebuilds it at every create, so a relabelled tuning counts
# 3% slower than it measures; reordering the lists keeps a copy of the ids
# (not of the offsets) and needs no sort, so 2%. A candidate then replaces
# the best so far if it is 1% better (against noise) after that.
PREMIUM = {"relabel": 1.03, "order_lists": 1.02}


def adjusted(t: Tuning, obj):
    """The objective with the premium of every costly choice t makes."""
    if obj is None:
        return None
    for field, factor in PREMIUM.items():
        if getattr(t, field):
            obj = obj / factor
    return obj


def device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "unknown").split(":")[0]
    return "%s_%dcu" % (arch, p.multi_processor_count)


# Dimensions that set two fields together.
PAIRS = {"layout_protocol": ("layout", "protocol"), "upper_wait": ("upper_only", "wait_release")}


def _with(t: Tuning, dim: str, value) -> Tuning:
    d = t.as_dict()
    if dim in PAIRS:
        d[PAIRS[dim][0]], d[PAIRS[dim][1]] = value
    else:
        d[dim] = value
    return Tuning(**d)


def _value(t: Tuning, dim: str):
    if dim in PAIRS:
        return (getattr(t, PAIRS[dim][0]), getattr(t, PAIRS[dim][1]))
    return getattr(t, dim)


# Reproducibility limit of the serving classes: over repeated passes of one
# graph alone, the standard deviation of the matching size may be at most this
# fraction of the size. Passes differ because concurrent lanes race (Section
# V-C); the serving loop promises a result in a batch or beside other jobs
# within 1% of SGMM's size of the result alone; a little under a tenth of
# that (the GPU's matchings are up to 8% larger than SGMM's) keeps the range
# of ten passes (about three standard deviations) under a third of it.
SPREAD_LIMIT = 0.0008


# Choices that build a copy of the graph at create time: they pay off only for
# a handle that runs many passes, not for a serving request, which creates its
# handle and runs one.
COPIES = {"relabel": 0, "order_lists": 0}


class SingleTarget:
    """One resident graph; objective = GEdges/s of a whole pass. With
    copies=False the tuning keeps the given graph (no relabelled or reordered
    copy, see COPIES). With
    spread_reps > 0 every candidate also runs that many checked passes, and
    one whose matching sizes vary by more than SPREAD_LIMIT (standard
    deviation over mean) is rejected."""

    unit = "GEdges/s"

    def __init__(self, csr, reps: int = 5, copies: bool = True, spread_reps: int = 0):
        # single graphs here are large: no whole-graph sweeps
        self.dims = [d for d in SPACE if d not in ("whole_graph_vertices", "mesh_wave_vertices") and
                     (copies or (d not in COPIES and d != "hot_degree"))]
        self.fixed = {} if copies else dict(COPIES)  # held for the whole search
        import torch
        self.off = torch.from_numpy(csr.off).cuda()
        self.nbr = torch.from_numpy(csr.nbr).cuda()
        self.m = csr.m
        self.reps = reps
        self.spread_reps = spread_reps
        self.sample = "%s (n=%d, m=%d)" % (csr.name, csr.n, csr.m)
        self.last_spread = None

    def measure(self, t: Tuning):
        import torch
        g = Graph(self.off, self.nbr, symmetric=True, tuning=t)
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
        try:
            g.run(out)
            g.sync()
            if not g.check(out)["ok"]:
                return None
            times = []
            for _ in range(self.reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                g.run(out)
                b.record()
                g.sync()
                times.append(a.elapsed_time(b) * 1e-3)
            if not g.check(out)["ok"]:
                return None
            if self.spread_reps > 0:
                sizes = []
                for _ in range(self.spread_reps):
                    g.run(out)
                    g.sync()
                    c = g.check(out)
                    if not c["ok"]:
                        return None
                    sizes.append(c["matched"] // 2)
                self.last_spread = float(np.std(sizes)) / max(float(np.mean(sizes)), 1.0)
                if self.last_spread > SPREAD_LIMIT:
                    return None
            return self.m / float(np.median(times)) / 1e9
        finally:
            g.close()


class MultiTarget:
    """Several resident graphs of one class, each its own handle; objective =
    their entries over the sum of their pass times, so that a tuning must
    serve every size of the class, not one graph."""

    unit = "GEdges/s"

    def __init__(self, csrs, reps: int = 5, copies: bool = False, spread_reps: int = 0):
        self.parts = [SingleTarget(c, reps=reps, copies=copies, spread_reps=spread_reps)
                      for c in csrs]
        self.dims = self.parts[0].dims
        self.fixed = self.parts[0].fixed
        self.sample = " + ".join(p.sample for p in self.parts)

    def measure(self, t: Tuning):
        seconds, m = 0.0, 0
        for p in self.parts:
            r = p.measure(t)
            if r is None:
                return None
            seconds += p.m / (r * 1e9)
            m += p.m
        return m / seconds / 1e9


class BatchTarget:
    """A many-graph batch; objective = graphs/s of a captured pass."""

    unit = "graphs/s"
    # the copies are for single graphs; whole-graph items trade batch throughput
    # for results independent of the rest of the batch (kept by the serving loop)
    dims = [d for d in SPACE if d not in COPIES and d != "hot_degree"]

    def __init__(self, mix, reps: int = 5):
        import torch
        self.off = torch.from_numpy(mix.off).cuda()
        self.nbr = torch.from_numpy(mix.nbr).cuda()
        self.vtx = mix.vtx_off
        self.G = mix.num_graphs
        self.reps = reps
        self.sample = "%s (%d graphs, N=%d, M=%d)" % (mix.name, mix.num_graphs, mix.n, mix.m)

    def measure(self, t: Tuning):
        import torch
        b = Batch(self.off, self.nbr, self.vtx, symmetric=True, capture=True, tuning=t)
        out = torch.empty(b.N, dtype=torch.int32, device="cuda")
        try:
            b.run(out)
            b.sync()
            if not b.check(out)["ok"]:
                return None
            times = []
            for _ in range(self.reps):
                a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                b.run(out)
                e.record()
                b.sync()
                times.append(a.elapsed_time(e) * 1e-3)
            if not b.check(out)["ok"]:
                return None
            return self.G / float(np.median(times))
        finally:
            b.close()


# Starting shapes tried, in order, when neither the stored entry nor the
# defaults pass: each halves the wavefronts a small graph keeps in flight.
CONSERVATIVE = [dict(wave_vertices=2048, min_waves=16), dict(wave_vertices=4096, min_waves=8),
                dict(wave_vertices=4096, min_waves=4)]


def search(target, start: Tuning | None = None, passes: int = 2, dims=None, log=print) -> dict:
    """Coordinate search; returns the best tuning, its objective and the
    number of candidates measured and rejected (failed check or error)."""
    best = start if start is not None else Tuning.default()
    best = Tuning(**dict(best.as_dict(), **getattr(target, "fixed", {})))
    cache = {}

    def score(t):
        key = tuple(sorted(t.as_dict().items()))
        if key not in cache:
            try:
                cache[key] = target.measure(t)
            except _lib.MMError as e:
                log("  rejected %s: %s" % (t.as_dict(), e))
                cache[key] = None
        return cache[key]

    default_obj = score(best)
    if default_obj is None:
        # a start that does not pass (a failed check, or the spread limit of a
        # reproducible class): the library defaults, then shapes with fewer
        # wavefronts of a small graph in flight at once (fewer lanes racing)
        fixed = getattr(target, "fixed", {})
        for over in [{}] + CONSERVATIVE:
            best = Tuning(**dict(Tuning.default().as_dict(), **over, **fixed))
            log("  the start is rejected; trying %s" % (over or "the library defaults"))
            default_obj = score(best)
            if default_obj is not None:
                break
    if default_obj is None:
        raise RuntimeError("no starting tuning passes the check")
    best_obj = default_obj
    dims = dims or getattr(target, "dims", list(SPACE))
    for p in range(passes):
        changed = False
        for dim in dims:
            for v in SPACE[dim]:
                if v == _value(best, dim):
                    continue
                cand = _with(best, dim, v)
                obj = score(cand)
                if obj is not None and adjusted(cand, obj) > adjusted(best, best_obj) * 1.01:
                    best, best_obj, changed = cand, obj, True
            log("  pass %d %-16s -> %s  %.4g %s" % (p, dim, _value(best, dim), best_obj, target.unit))
        if not changed:
            break
    rejected = sum(1 for v in cache.values() if v is None)
    return {"tuning": best.as_dict(), "objective": best_obj, "default_objective": default_obj,
            "unit": target.unit, "sample": target.sample, "candidates": len(cache),
            "rejected": rejected}


# Below MID_VERTICES a grid or R-MAT graph is of the "_mid" class (the
# serving workload's large jobs): the best launch shape differs there. Below
# SMALL_VERTICES any graph is of a "_small" class: a shape that runs the whole
# graph at once would let so many of its lanes race that the matching size
# varies from pass to pass by more than the serving loop allows, so these
# classes are tuned under SPREAD_LIMIT.
MID_VERTICES = 1 << 25
SMALL_VERTICES = 1 << 18
# Classes whose search rejects candidates above SPREAD_LIMIT (the ones the
# serving loop runs alone).
REPRODUCIBLE = ("rmat_small", "grid_small", "er_small", "rmat_mid", "grid_mid")
SPREAD_REPS = 20


def _targets(classes, seed, rmat_scale=27, grid_side=16384):
    import graphgen
    out = {}
    for c in classes:
        if c == "rmat":
            out[c] = lambda: SingleTarget(graphgen.rmat(rmat_scale, seed=seed))
        elif c == "rmat_mid":
            out[c] = lambda: MultiTarget([graphgen.rmat(18, 8, seed=seed), graphgen.rmat(21, 8, seed=seed)],
                                         spread_reps=SPREAD_REPS)
        elif c == "rmat_small":
            out[c] = lambda: MultiTarget([graphgen.rmat(15, 16, seed=seed), graphgen.rmat(17, 8, seed=seed)],
                                         spread_reps=SPREAD_REPS)
        elif c == "grid":
            out[c] = lambda: SingleTarget(graphgen.grid(grid_side, grid_side))
        elif c == "grid_mid":
            out[c] = lambda: MultiTarget([graphgen.grid(724, 724), graphgen.grid(3168, 3168)],
                                         spread_reps=SPREAD_REPS)
        elif c == "grid_small":
            out[c] = lambda: MultiTarget([graphgen.grid(200, 200), graphgen.grid(400, 401)],
                                         spread_reps=SPREAD_REPS)
        elif c == "er_small":
            out[c] = lambda: MultiTarget([graphgen.er(40000, 12, seed=seed), graphgen.er(150000, 8, seed=seed)],
                                         spread_reps=SPREAD_REPS)
        elif c == "er":
            # both sizes: the 65536-vertex graph is in flight whole, and the
            # best scan there is not the best on 4M vertices
            out[c] = lambda: MultiTarget([graphgen.er(1 << 16, 16, seed=seed),
                                          graphgen.er(1 << 22, 16, seed=seed)], copies=True)
        elif c == "batch":
            out[c] = lambda: BatchTarget(graphgen.mixture(4096, seed=seed))
        else:
            raise ValueError("unknown graph class %r" % c)
    return out


def tuned_path(key: str | None = None) -> str:
    return os.path.join(TUNED_DIR, "%s.json" % (key or device_key()))


def tuned(graph_class: str, key: str | None = None) -> Tuning:
    """The stored tuning for this device and graph class (a "_mid" class
    without an entry of its own takes its kind's), else the defaults (a
    "_small" class without an entry takes the defaults, whose blocks keep a
    small graph's lanes few)."""
    path = tuned_path(key)
    if os.path.exists(path):
        with open(path) as f:
            classes = json.load(f).get("classes", {})
        entry = classes.get(graph_class)
        if not entry and graph_class.endswith("_mid"):
            entry = classes.get(graph_class[:-len("_mid")])
        if entry:
            return Tuning(**entry["tuning"])
    return Tuning.default()


def classify(off: np.ndarray) -> str:
    """Graph class of a CSR from its degree sequence: 'grid' when no vertex has
    more than 4 entries, 'rmat' when the degrees are heavily skewed (largest
    over 32 times the mean), else 'er'; any graph of fewer than SMALL_VERTICES
    vertices is '<kind>_small', a grid or R-MAT graph of fewer than
    MID_VERTICES vertices 'grid_mid' / 'rmat_mid'."""
    deg = np.diff(off)
    if deg.size == 0 or deg.max() <= 4:
        kind = "grid"
    else:
        kind = "rmat" if deg.max() > 32 * max(deg.mean(), 1e-9) else "er"
    if deg.size < SMALL_VERTICES:
        return kind + "_small"
    return kind + "_mid" if kind != "er" and deg.size < MID_VERTICES else kind


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--classes",
                    default="batch,rmat,grid,er,rmat_mid,grid_mid,rmat_small,grid_small,er_small")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--passes", type=int, default=2)
    ap.add_argument("--rmat-scale", type=int, default=27)
    ap.add_argument("--grid-side", type=int, default=16384)
    ap.add_argument("--out", default=None, help="JSON file (default: the package's tuned/ entry)")
    ap.add_argument("--from-defaults", action="store_true",
                    help="start every search from the library defaults instead of the stored table")
    a = ap.parse_args(argv)
    key = device_key()
    out = a.out or tuned_path(key)
    doc = {"device": key, "classes": {}}
    if os.path.exists(out):
        with open(out) as f:
            doc = json.load(f)
    for c, make in _targets(a.classes.split(","), a.seed, a.rmat_scale, a.grid_side).items():
        t0 = time.time()
        print("== %s" % c, flush=True)
        start = None if a.from_defaults else tuned(c, key)
        r = search(make(), start=start, passes=a.passes, log=lambda s: print(s, flush=True))
        if c in REPRODUCIBLE:
            r["spread_limit"] = SPREAD_LIMIT
        r["seconds"] = round(time.time() - t0, 1)
        doc["classes"][c] = r
        print(json.dumps({c: r}), flush=True)
        os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
        with open(out, "w") as f:
            json.dump(doc, f, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
