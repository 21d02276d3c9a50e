"""Seeded synthetic graph inputs, shared by the GPU path's tests and the oracle.

This module draws graphs and lays them out as CSR (Section II-A of the paper).
It holds none of the matching method's arithmetic. Every graph is a pure
function of its parameters and seed; see ``graphgen.cpp`` for the models and
the counter-based generator (SplitMix64 on a keyed counter).

Workload recipes (the paper's datasets are not available; these stand in):

* ``er(65536, 16)``            Erdos-Renyi, ~1M directed CSR entries
* ``rmat(24)`` / ``rmat(27)``  R-MAT, edge factor 16, (0.57, 0.19, 0.19, 0.05),
                               ids relabelled by a seeded bijection; a stand-in
                               for the paper's Kronecker graph (Table I, g500)
* ``grid(16384, 16384)``       4-neighbour mesh, row-major ids
* ``mixture(G, seed)``         G graphs, type uniform over {ER, grid, R-MAT},
                               vertex counts log-uniform in [1e3, 2e5]
* ``serve_pool(P, seed)``      P graphs of the same three types whose entry
                               counts are log-uniform in [1e4, 5e7]: the
                               resident graphs a stream of requests draws from
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None
_lock = threading.Lock()

KIND_ER, KIND_GRID, KIND_RMAT = 0, 1, 2
KIND_NAMES = {KIND_ER: "er", KIND_GRID: "grid", KIND_RMAT: "rmat"}


def build(force: bool = False) -> str:
    """Compiles libgraphgen.so next to its source (g++, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O3", "-march=x86-64-v2", "-std=c++17", "-fopenmp", "-shared", "-fPIC",
               _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.gg_rmat.restype = P
        lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32]
        lib.gg_er.restype = P
        lib.gg_er.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, ctypes.c_int32]
        lib.gg_grid.restype = P
        lib.gg_grid.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32]
        lib.gg_member.restype = P
        lib.gg_member.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                  ctypes.c_int32]
        lib.gg_concat.restype = P
        lib.gg_concat.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_int32]
        for name, rt in (("gg_n", ctypes.c_int64), ("gg_m", ctypes.c_int64),
                         ("gg_num_graphs", ctypes.c_int32)):
            getattr(lib, name).restype = rt
            getattr(lib, name).argtypes = [P]
        for name in ("gg_offsets", "gg_neighbors", "gg_vtx_off", "gg_kinds"):
            getattr(lib, name).restype = P
            getattr(lib, name).argtypes = [P]
        lib.gg_free.restype = None
        lib.gg_free.argtypes = [P]
        lib.gg_draw.restype = ctypes.c_uint64
        lib.gg_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        _lib = lib
        return lib


class CSR:
    """A graph in CSR form, with numpy-owned arrays.

    ``off`` has n+1 entries (int64 unless converted), ``nbr`` has m int32
    entries. Mixtures also carry ``vtx_off`` (num_graphs+1, int64) and
    ``kinds``; their ``off`` holds global positions while ``nbr`` holds ids
    local to each member graph.
    """

    def __init__(self, off, nbr, vtx_off=None, kinds=None, name=""):
        self.off = off
        self.nbr = nbr
        self.vtx_off = vtx_off
        self.kinds = kinds
        self.name = name

    @property
    def n(self) -> int:
        return int(self.off.shape[0]) - 1

    @property
    def m(self) -> int:
        return int(self.nbr.shape[0])

    @property
    def num_graphs(self) -> int:
        return 0 if self.vtx_off is None else int(self.vtx_off.shape[0]) - 1

    def with_int32_offsets(self) -> "CSR":
        if self.m > 2**31 - 1:
            raise ValueError("m does not fit int32 offsets")
        return CSR(self.off.astype(np.int32), self.nbr, self.vtx_off, self.kinds, self.name)

    def member(self, g: int) -> "CSR":
        """Member graph g of a mixture, as a standalone CSR."""
        v0, v1 = int(self.vtx_off[g]), int(self.vtx_off[g + 1])
        e0, e1 = int(self.off[v0]), int(self.off[v1])
        return CSR((self.off[v0:v1 + 1] - e0).astype(np.int64), self.nbr[e0:e1],
                   name="%s[%d]" % (self.name, g))


def _take(h, name="") -> CSR:
    lib = _load()
    if not h:
        raise MemoryError("graph generation failed (bad parameters or out of memory)")
    try:
        n, m = lib.gg_n(h), lib.gg_m(h)
        off = np.empty(n + 1, dtype=np.int64)
        nbr = np.empty(m, dtype=np.int32)
        ctypes.memmove(off.ctypes.data, lib.gg_offsets(h), 8 * (n + 1))
        if m:
            ctypes.memmove(nbr.ctypes.data, lib.gg_neighbors(h), 4 * m)
        vtx_off = kinds = None
        ng = lib.gg_num_graphs(h)
        if ng:
            vtx_off = np.empty(ng + 1, dtype=np.int64)
            kinds = np.empty(ng, dtype=np.int32)
            ctypes.memmove(vtx_off.ctypes.data, lib.gg_vtx_off(h), 8 * (ng + 1))
            ctypes.memmove(kinds.ctypes.data, lib.gg_kinds(h), 4 * ng)
        return CSR(off, nbr, vtx_off, kinds, name)
    finally:
        lib.gg_free(h)


def rmat(scale: int, edge_factor: float = 16.0, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 1, permute: bool = True, threads: int = 0) -> CSR:
    """Symmetrised, deduplicated, loop-free R-MAT graph with 2^scale vertices."""
    h = _load().gg_rmat(scale, edge_factor, a, b, c, seed, int(permute), threads)
    return _take(h, "rmat%d_ef%g_s%d" % (scale, edge_factor, seed))


def er(n: int, avg_deg: float, seed: int = 1, threads: int = 0) -> CSR:
    """G(n, p) with p = avg_deg / (n - 1), symmetrised."""
    return _take(_load().gg_er(n, avg_deg, seed, threads), "er%d_d%g_s%d" % (n, avg_deg, seed))


def grid(H: int, W: int, threads: int = 0) -> CSR:
    """H x W 4-neighbour grid, id = r * W + c, lists ascending."""
    return _take(_load().gg_grid(H, W, threads), "grid%dx%d" % (H, W))


def draw(seed: int, stream: int, ctr: int) -> int:
    """The module's counter-based 64-bit draw."""
    return int(_load().gg_draw(seed, stream, ctr))


def _u01(seed, stream, ctr):
    return ((draw(seed, stream, ctr) >> 11) + 0.5) / float(1 << 53)


def member_spec(g: int, seed: int, nmin: float = 1e3, nmax: float = 2e5):
    """(kind, n, param) of mixture member g: kind uniform over {ER, grid,
    R-MAT}; n log-uniform in [nmin, nmax]; ER average degree uniform in
    [4, 32]; R-MAT scale clamp(round(log2 n), 10, 17) with edge factor 8."""
    kind = int(draw(seed, 1000 + g, 0) % 3)
    n = int(round(math.exp(math.log(nmin) + _u01(seed, 1000 + g, 1) * (math.log(nmax) - math.log(nmin)))))
    n = max(int(nmin), min(int(nmax), n))
    if kind == KIND_ER:
        param = 4.0 + 28.0 * _u01(seed, 1000 + g, 2)
    elif kind == KIND_RMAT:
        param = float(min(17, max(10, int(round(math.log2(n))))))
        n = 1 << int(param)
    else:
        param = 0.0
    return kind, n, param


def serve_spec(i: int, seed: int, mmin: float = 1e4, mmax: float = 5e7):
    """(kind, n, param) of serving-pool graph i: kind uniform over {ER, grid,
    R-MAT}; a target entry count m log-uniform in [mmin, mmax]; ER average
    degree uniform in [4, 32] with n = m / degree; a grid of about m / 4
    vertices; R-MAT (edge factor 8) at scale clamp(round(log2(m / 16)), 6, 22)."""
    kind = int(draw(seed, 5000 + i, 0) % 3)
    lm = math.log(mmin) + _u01(seed, 5000 + i, 1) * (math.log(mmax) - math.log(mmin))
    m = math.exp(lm)
    if kind == KIND_ER:
        deg = 4.0 + 28.0 * _u01(seed, 5000 + i, 2)
        return kind, max(2, int(round(m / deg))), deg
    if kind == KIND_RMAT:
        sc = min(22, max(6, int(round(math.log2(m / 16.0)))))
        return kind, 1 << sc, float(sc)
    return kind, max(4, int(round(m / 4.0))), 0.0


def serve_pool(num_graphs: int, seed: int = 1, mmin: float = 1e4, mmax: float = 5e7,
               threads: int = 0) -> CSR:
    """The serving workload's resident graphs, concatenated like a mixture."""
    specs = [serve_spec(i, seed, mmin, mmax) for i in range(num_graphs)]
    return concat(specs, seed, threads, "pool%d_s%d" % (num_graphs, seed))


def concat(specs, seed: int, threads: int = 0, name: str = "mix") -> CSR:
    """Concatenates members described by (kind, n, param) tuples."""
    G = len(specs)
    kinds = np.array([s[0] for s in specs], dtype=np.int32)
    ns = np.array([s[1] for s in specs], dtype=np.int64)
    params = np.array([s[2] for s in specs], dtype=np.float64)
    seeds = np.array([draw(seed, 7, g) for g in range(G)], dtype=np.uint64)
    h = _load().gg_concat(G, kinds.ctypes.data, ns.ctypes.data, params.ctypes.data,
                          seeds.ctypes.data, threads)
    return _take(h, name)


def mixture(num_graphs: int, seed: int = 1, nmin: float = 1e3, nmax: float = 2e5,
            threads: int = 0) -> CSR:
    """The batched workload: num_graphs members, concatenated."""
    specs = [member_spec(g, seed, nmin, nmax) for g in range(num_graphs)]
    return concat(specs, seed, threads, "mix%d_s%d" % (num_graphs, seed))


def from_edges(n: int, edges, symmetric: bool = True, dedup: bool = True, sort: bool = True,
               drop_loops: bool = False) -> CSR:
    """Small-graph helper: CSR from an (E, 2) edge list.

    With ``symmetric`` both orientations are stored. Lists keep insertion
    order unless ``sort`` is set. Used for hand-built test graphs.
    """
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if drop_loops:
        e = e[e[:, 0] != e[:, 1]]
    if symmetric:
        rev = e[:, ::-1]
        keep = rev[:, 0] != rev[:, 1]
        e = np.concatenate([e, rev[keep]], axis=0)
    if sort:
        order = np.lexsort((e[:, 1], e[:, 0]))
    else:
        order = np.argsort(e[:, 0], kind="stable")
    e = e[order]
    if dedup and len(e):
        keep = np.ones(len(e), dtype=bool)
        if sort:
            keep[1:] = np.any(e[1:] != e[:-1], axis=1)
        else:
            seen = set()
            for i, (a, b) in enumerate(map(tuple, e)):
                if (a, b) in seen:
                    keep[i] = False
                seen.add((a, b))
        e = e[keep]
    deg = np.bincount(e[:, 0], minlength=n) if len(e) else np.zeros(n, dtype=np.int64)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=off[1:])
    return CSR(off, e[:, 1].astype(np.int32), name="edges%d" % n)
