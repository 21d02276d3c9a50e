"""Skipper maximal matching on MI355X (gfx950).

Python surface over the C ABI of include/mm.h. PyTorch supplies device
memory and streams; every step of a matching pass runs in the library's HIP
kernels.

    g = Graph(offsets, neighbors, symmetric=True)   # CSR on the GPU
    mate = g.run()                                  # int32[n], -1 = unmatched
"""
from __future__ import annotations

import ctypes
from dataclasses import asdict, dataclass

import numpy as np

from . import _lib
from ._lib import MMError  # noqa: F401

__all__ = ["Graph", "Batch", "Tuning", "MMError", "maximal_matching", "conflict_table", "conflict_row",
           "library_path", "version"]


def library_path() -> str:
    return _lib.LIB_PATH


def version() -> str:
    return _lib.load().mm_version().decode()


@dataclass
class Tuning:
    """Launch and layout parameters (see mm_tuning in include/mm.h)."""
    layout: int = _lib.MM_LAYOUT_U32
    protocol: int = _lib.MM_PROTOCOL_CAS
    hint: int = 0
    wg_size: int = 256
    wave_vertices: int = 1024
    disperse: int = 0
    assist_after: int = 64
    lazy_init: int = 0
    scan_width: int = 4
    stream_loads: int = 0
    whole_graph_vertices: int = 16384
    relabel: int = 0
    hub_degree: int = 4096
    hub_chunk: int = 256
    whole_graph_lds: int = 1
    mesh_wave_vertices: int = 0
    wait_release: int = 0
    upper_only: int = 0
    hub_wave: int = 1
    min_waves: int = 32
    hot_degree: int = 2048
    order_lists: int = 0
    probe_first: int = 0
    occupancy: int = 0
    iter_cap: int = 0

    @classmethod
    def default(cls) -> "Tuning":
        t = _lib.mm_tuning()
        _lib.load().mm_default_tuning(ctypes.byref(t))
        return cls(**{f: getattr(t, f) for f, _ in _lib.mm_tuning._fields_})

    def to_c(self) -> _lib.mm_tuning:
        return _lib.mm_tuning(**asdict(self))

    def as_dict(self) -> dict:
        return asdict(self)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_graph_tensors(offsets, neighbors):
    import torch
    if not (offsets.is_cuda and neighbors.is_cuda):
        raise ValueError("offsets and neighbors must be CUDA (HIP) tensors")
    if offsets.dim() != 1 or neighbors.dim() != 1:
        raise ValueError("offsets and neighbors must be 1-D")
    if not offsets.is_contiguous() or not neighbors.is_contiguous():
        raise ValueError("offsets and neighbors must be contiguous")
    if offsets.dtype == torch.int64:
        off_type = _lib.MM_OFF_I64
    elif offsets.dtype == torch.int32:
        off_type = _lib.MM_OFF_I32
    else:
        raise ValueError("offsets must be int32 or int64")
    if neighbors.dtype != torch.int32:
        raise ValueError("neighbors must be int32")
    if offsets.numel() < 1:
        raise ValueError("offsets needs n+1 >= 1 entries")
    return off_type


CHECK_FIELDS = ("out_of_range", "self_mate", "asymmetric", "not_edge", "uncovered", "matched")


def _check_mate(mate, n: int) -> None:
    import torch
    if mate.dtype != torch.int32 or mate.numel() != n or not mate.is_contiguous() or not mate.is_cuda:
        raise ValueError("mate must be a contiguous int32 GPU tensor of %d entries" % n)


def _check_result(c) -> dict:
    r = {f: int(c[i]) for i, f in enumerate(CHECK_FIELDS)}
    r["ok"] = all(r[f] == 0 for f in CHECK_FIELDS[:5])
    return r


class Graph:
    """One graph resident on the GPU, with its workspace.

    The CSR tensors are borrowed (kept referenced here). ``symmetric=True``
    asserts every entry has its reverse, which allows lazy mate output.
    """

    def __init__(self, offsets, neighbors, *, symmetric: bool = False, validate: bool = False,
                 stats: bool = False, timing: bool = False, tuning: Tuning | None = None,
                 stream=None):
        import torch
        lib = _lib.load()
        off_type = _check_graph_tensors(offsets, neighbors)
        self.offsets, self.neighbors = offsets, neighbors
        self.n = offsets.numel() - 1
        self.m = neighbors.numel()
        self.tuning = tuning if tuning is not None else Tuning.default()
        ct = self.tuning.to_c()
        nbytes = lib.mm_workspace_bytes_graph(self.n, self.m, ctypes.byref(ct))
        if nbytes == 0:
            raise MMError(_lib.MM_ERR_INVALID_ARG, "invalid n or tuning")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=offsets.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        flags = ((_lib.MM_VALIDATE if validate else 0) | (_lib.MM_SYMMETRIC if symmetric else 0)
                 | (_lib.MM_STATS if stats else 0) | (_lib.MM_TIMING if timing else 0))
        h = ctypes.c_void_p()
        _lib.check(lib.mm_create(ctypes.c_void_p(offsets.data_ptr()), off_type,
                                 ctypes.c_void_p(neighbors.data_ptr()), self.n, self.m,
                                 ctypes.c_void_p(aligned), nbytes, flags, ctypes.byref(ct),
                                 _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        self.device = offsets.device

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise ValueError("graph handle was closed")
        return self._h

    def run(self, out=None, stream=None):
        """Enqueues one matching pass; returns the int32 mate tensor."""
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.int32, device=self.device)
        elif out.dtype != torch.int32 or out.numel() != self.n or not out.is_contiguous():
            raise ValueError("out must be a contiguous int32 tensor of n entries")
        _lib.check(_lib.load().mm_run(self.handle, _stream_ptr(stream), ctypes.c_void_p(out.data_ptr())))
        return out

    def sync(self, stream=None) -> None:
        """Waits for the stream and raises if a pass ran out of its loop budget."""
        _lib.check(_lib.load().mm_sync(self.handle, _stream_ptr(stream)))

    def stats(self, stream=None) -> dict:
        s = _lib.mm_stats()
        _lib.check(_lib.load().mm_get_stats(self.handle, _stream_ptr(stream), ctypes.byref(s)))
        return _lib.stats_dict(s)

    def timing(self) -> dict:
        """Sweep-kernel durations of the passes since the last call (ms)."""
        cnt, tot, lo, hi = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _lib.check(_lib.load().mm_get_timing(self.handle, ctypes.byref(cnt), ctypes.byref(tot),
                                             ctypes.byref(lo), ctypes.byref(hi)))
        n = cnt.value
        return {"count": n, "total_ms": tot.value, "mean_ms": tot.value / n if n else 0.0,
                "min_ms": lo.value, "max_ms": hi.value}

    def check(self, mate, stream=None) -> dict:
        """Device verification of a mate tensor (mm_check): violation counts
        and ``ok`` (True iff the mates form a maximal matching)."""
        _check_mate(mate, self.n)
        c = (ctypes.c_int64 * 6)()
        _lib.check(_lib.load().mm_check(self.handle, _stream_ptr(stream),
                                         ctypes.c_void_p(mate.data_ptr()), c))
        return _check_result(c)

    def pairs(self, mate, stream=None):
        """The matched pairs of a mate tensor as an (P, 2) int32 tensor of
        (u, v), u < v (mm_pairs); the order of the rows is not specified."""
        import torch
        _check_mate(mate, self.n)
        cap = self.n // 2
        out = torch.empty(max(cap, 1) * 2, dtype=torch.int32, device=self.device)
        cnt = ctypes.c_int64()
        _lib.check(_lib.load().mm_pairs(self.handle, _stream_ptr(stream),
                                        ctypes.c_void_p(mate.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), cap, ctypes.byref(cnt)))
        return out[:2 * cnt.value].view(-1, 2)

    def ems(self, seed: int = 1, out=None, stream=None):
        """The iterated mutual-selection baseline (mm_ems_run) on this graph:
        returns (mate tensor, {"iterations", "touched", "pairs"})."""
        import torch
        lib = _lib.load()
        nb = lib.mm_ems_scratch_bytes(self.n)
        scratch = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        aligned = (scratch.data_ptr() + 255) // 256 * 256
        if out is None:
            out = torch.empty(max(self.n, 1), dtype=torch.int32, device=self.device)[:self.n]
        st = _lib.mm_ems_stats()
        _lib.check(lib.mm_ems_run(self.handle, _stream_ptr(stream), ctypes.c_uint64(seed),
                                  ctypes.c_void_p(aligned), nb, ctypes.c_void_p(out.data_ptr()),
                                  ctypes.byref(st)))
        return out, {"iterations": st.iterations, "touched": st.touched, "pairs": st.pairs}

    def reset_stats(self, stream=None) -> None:
        _lib.check(_lib.load().mm_reset_stats(self.handle, _stream_ptr(stream)))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            _lib.load().mm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many graphs matched in one persistent launch (see mm_batch_* in mm.h).

    offsets: int64 CUDA tensor of N+1 positions into `neighbors` (int32 CUDA
    tensor of local ids); vtx_off: host sequence of num_graphs+1 vertex
    offsets. run() returns the int32 tensor of LOCAL mates (-1 = unmatched).
    ``capture=True`` replays a hipGraph of the pass after the first run.
    ``Batch.from_list`` builds a batch over graphs held in separate tensors.
    """

    def __init__(self, offsets, neighbors, vtx_off, *, symmetric: bool = False,
                 validate: bool = False, stats: bool = False, capture: bool = False,
                 tuning: Tuning | None = None, stream=None):
        import torch
        if offsets.dtype != torch.int64:
            raise ValueError("batch offsets must be int64")
        _check_graph_tensors(offsets, neighbors)
        vtx = np.ascontiguousarray(np.asarray(vtx_off, dtype=np.int64))
        if offsets.numel() != int(vtx[-1]) + 1:
            raise ValueError("offsets must have vtx_off[-1] + 1 entries")
        self.offsets, self.neighbors = offsets, neighbors

        def create(lib, ws, nbytes, flags, ct, h):
            return lib.mm_batch_create(ctypes.c_void_p(offsets.data_ptr()),
                                       ctypes.c_void_p(neighbors.data_ptr()),
                                       ctypes.c_void_p(vtx.ctypes.data), len(vtx) - 1,
                                       neighbors.numel(), ws, nbytes, flags, ct, _stream_ptr(stream), h)

        self._setup(vtx, offsets.device, symmetric, validate, stats, capture, tuning, create)

    @classmethod
    def from_list(cls, graphs, *, symmetric: bool = False, validate: bool = False,
                  stats: bool = False, capture: bool = False, tuning: Tuning | None = None,
                  stream=None) -> "Batch":
        """A batch over separately held graphs: ``graphs`` is a sequence of
        (offsets int64, neighbors int32) CUDA tensor pairs, each a graph's own
        CSR. The output holds graph g's mates at vtx_off[g] .. vtx_off[g+1]-1,
        vtx_off being the prefix sums of the vertex counts."""
        import torch
        self = cls.__new__(cls)
        G = len(graphs)
        offs = (ctypes.c_void_p * max(G, 1))()
        nbrs = (ctypes.c_void_p * max(G, 1))()
        ns = np.zeros(max(G, 1), dtype=np.int64)
        ms = np.zeros(max(G, 1), dtype=np.int64)
        device = None
        for g, (o, nb) in enumerate(graphs):
            if o.dtype != torch.int64:
                raise ValueError("graph %d: offsets must be int64" % g)
            _check_graph_tensors(o, nb)
            offs[g], nbrs[g] = o.data_ptr(), nb.data_ptr()
            ns[g], ms[g] = o.numel() - 1, nb.numel()
            device = o.device if device is None else device
        self.graphs = list(graphs)  # borrowed: kept alive with the handle
        vtx = np.zeros(G + 1, dtype=np.int64)
        np.cumsum(ns[:G], out=vtx[1:])

        def create(lib, ws, nbytes, flags, ct, h):
            return lib.mm_batch_create_list(offs, nbrs, ctypes.c_void_p(ns.ctypes.data),
                                            ctypes.c_void_p(ms.ctypes.data), G, ws, nbytes, flags,
                                            ct, _stream_ptr(stream), h)

        self._setup(vtx, device if device is not None else torch.device("cuda"), symmetric,
                    validate, stats, capture, tuning, create)
        return self

    def _setup(self, vtx, device, symmetric, validate, stats, capture, tuning, create):
        import torch
        lib = _lib.load()
        self._h = None
        self._vtx = vtx
        self.vtx_off = vtx
        self.num_graphs = int(vtx.shape[0]) - 1
        self.N = int(vtx[-1])
        self.tuning = tuning if tuning is not None else Tuning.default()
        ct = self.tuning.to_c()
        nbytes = lib.mm_batch_workspace_bytes(self.num_graphs, ctypes.c_void_p(vtx.ctypes.data),
                                              ctypes.byref(ct))
        if nbytes == 0:
            raise MMError(_lib.MM_ERR_INVALID_ARG, "invalid vtx_off or tuning")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        flags = ((_lib.MM_VALIDATE if validate else 0) | (_lib.MM_SYMMETRIC if symmetric else 0)
                 | (_lib.MM_STATS if stats else 0) | (_lib.MM_CAPTURE if capture else 0))
        h = ctypes.c_void_p()
        _lib.check(create(lib, ctypes.c_void_p(aligned), nbytes, flags, ctypes.byref(ct),
                          ctypes.byref(h)))
        self._h = h
        self.device = device

    @property
    def items(self) -> int:
        return int(_lib.load().mm_batch_items(self._h))

    def run(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.N, dtype=torch.int32, device=self.device)
        elif out.dtype != torch.int32 or out.numel() != self.N or not out.is_contiguous():
            raise ValueError("out must be a contiguous int32 tensor of N entries")
        _lib.check(_lib.load().mm_batch_run(self._h, _stream_ptr(stream), ctypes.c_void_p(out.data_ptr())))
        return out

    def sync(self, stream=None) -> None:
        _lib.check(_lib.load().mm_batch_sync(self._h, _stream_ptr(stream)))

    def check(self, mate, stream=None) -> dict:
        """Device verification of a mate tensor of local ids (mm_batch_check),
        summed over the graphs of the batch."""
        _check_mate(mate, self.N)
        c = (ctypes.c_int64 * 6)()
        _lib.check(_lib.load().mm_batch_check(self._h, _stream_ptr(stream),
                                         ctypes.c_void_p(mate.data_ptr()), c))
        return _check_result(c)

    def stats(self, stream=None) -> dict:
        s = _lib.mm_stats()
        _lib.check(_lib.load().mm_batch_get_stats(self._h, _stream_ptr(stream), ctypes.byref(s)))
        return _lib.stats_dict(s)

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            _lib.load().mm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


CONFLICT_BINS = ("1", "2", "3-4", "5-8", "9-16", "17-32", "33-64", "65-128", "129-256", ">256")


def conflict_row(stats: dict) -> dict:
    """Table II's columns from one instrumented pass: the most conflicts met
    by one edge, the total conflicts (every failed take of u or v: those that
    met another lane's reservation and those that met a match made since the
    lane's cached read), the edges that met at least one, their mean, and the
    distribution of those edges over the table's bins. The two kinds are also
    reported apart."""
    hist = list(stats["conflict_hist"])
    edges = sum(hist)
    met_reserved = stats["reserve_conflicts"] + stats["match_conflicts"]
    met_matched = stats["reserve_matched"] + stats["match_matched"]
    total = met_reserved + met_matched
    return {"max_per_edge": stats["conflict_max"], "total": total, "edges": edges,
            "avg_per_edge": (total / edges) if edges else 0.0,
            "met_reserved": met_reserved, "met_matched": met_matched,
            "distribution": dict(zip(CONFLICT_BINS, hist))}


def conflict_table(offsets, neighbors, *, runs: int = 5, symmetric: bool = True,
                   tuning: Tuning | None = None) -> dict:
    """Table II for one graph: `runs` instrumented passes, keeping the one in
    which the most edges met a conflict (the paper's selection rule)."""
    best = None
    g = Graph(offsets, neighbors, symmetric=symmetric, stats=True, tuning=tuning)
    try:
        for _ in range(runs):
            g.reset_stats()
            g.run()
            g.sync()
            row = conflict_row(g.stats())
            if best is None or row["edges"] > best["edges"]:
                best = row
    finally:
        g.close()
    best["runs"] = runs
    best["entries"] = int(neighbors.numel())
    best["edge_ratio"] = best["edges"] / max(1, int(neighbors.numel()))
    return best


def maximal_matching(offsets, neighbors, *, symmetric: bool = False, tuning: Tuning | None = None,
                     stream=None):
    """One-shot helper: create, run, wait; returns the int32 mate tensor."""
    g = Graph(offsets, neighbors, symmetric=symmetric, tuning=tuning, stream=stream)
    out = g.run(stream=stream)
    g.sync(stream=stream)
    g.close()
    return out
