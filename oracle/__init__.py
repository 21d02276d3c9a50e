"""Oracle for maximal matching: TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never imports, links or
calls it, and shares no code with it.

Functions (all CPU; see ``oracle.c`` for the definitions they follow):

* ``sgmm(csr, x_end=None)``   Sequential Greedy MM (Section II-B), with the
                              early exit of the CSR form; returns the mate
                              array, pair count and neighbour ids read.
* ``check(csr, mate)``        Exact validity + maximality check
                              (Section II-B's two conditions, plus mate-array
                              well-formedness), with per-class counts.
* ``enumerate_matchings(csr, maximal_only)``  brute force, n <= 20.
* ``greedy_weighted(csr, seed)``  the matching iterated Endpoints Mutual
                              Selection (Section II-C) reaches with fixed
                              pseudo-random edge weights: the greedy matching
                              in descending weight order.
* ``edge_weight(u, v, seed)``, ``splitmix64(x)``  its weights.

Pins (tests/test_oracle.py): the worked example of Fig. 1 / Fig. 6, closed
forms on paths, stars, cliques, complete bipartite graphs, grids and disjoint
edges, brute-force enumeration (SGMM is the lexicographically first maximal
matching under CSR edge rank; the checker agrees with brute-force maximality
on every matching of every small graph), and mutation of valid outputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp],
                       check=True)
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
        P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.oracle_sgmm.restype = I64
        lib.oracle_sgmm.argtypes = [I64, P, I32, P, P, I64, P]
        lib.oracle_check.restype = None
        lib.oracle_check.argtypes = [I64, P, I32, P, P, P]
        lib.oracle_enumerate.restype = I64
        lib.oracle_enumerate.argtypes = [I64, P, I32, P, I32, P, I64]
        lib.oracle_greedy_weighted.restype = I64
        lib.oracle_greedy_weighted.argtypes = [I64, P, I32, P, ctypes.c_uint64, P]
        lib.oracle_edge_weight.restype = ctypes.c_uint64
        lib.oracle_edge_weight.argtypes = [I64, I64, ctypes.c_uint64]
        lib.oracle_splitmix64.restype = ctypes.c_uint64
        lib.oracle_splitmix64.argtypes = [ctypes.c_uint64]
        _lib = lib
        return lib


def _graph_args(csr):
    off = np.ascontiguousarray(csr.off)
    nbr = np.ascontiguousarray(csr.nbr, dtype=np.int32)
    if off.dtype == np.int64:
        off64 = 1
    elif off.dtype == np.int32:
        off64 = 0
    else:
        off = off.astype(np.int64)
        off64 = 1
    return off, off64, nbr


@dataclass
class SGMMResult:
    mate: np.ndarray
    pairs: int
    touched: int


def sgmm(csr, x_end: int | None = None) -> SGMMResult:
    """Sequential Greedy MM over sources 0..x_end-1 (default: all)."""
    off, off64, nbr = _graph_args(csr)
    n = csr.n
    mate = np.empty(n, dtype=np.int32)
    touched = ctypes.c_int64(0)
    pairs = _load().oracle_sgmm(n, off.ctypes.data, off64, nbr.ctypes.data, mate.ctypes.data,
                                n if x_end is None else int(x_end), ctypes.byref(touched))
    return SGMMResult(mate, int(pairs), int(touched.value))


@dataclass
class CheckResult:
    out_of_range: int
    self_mate: int
    asymmetric: int
    not_an_edge: int
    uncovered: int
    size: int
    bad_input: int
    matched_vertices: int

    @property
    def violations(self) -> int:
        return (self.out_of_range + self.self_mate + self.asymmetric + self.not_an_edge
                + self.uncovered)

    @property
    def ok(self) -> bool:
        return self.violations == 0 and self.bad_input == 0


def check(csr, mate) -> CheckResult:
    """Counts every violation class of a mate array against the graph."""
    off, off64, nbr = _graph_args(csr)
    mate = np.ascontiguousarray(mate, dtype=np.int32)
    if mate.shape[0] != csr.n:
        raise ValueError("mate array has %d entries, graph has %d vertices" % (mate.shape[0], csr.n))
    out = np.zeros(8, dtype=np.int64)
    _load().oracle_check(csr.n, off.ctypes.data, off64, nbr.ctypes.data, mate.ctypes.data,
                         out.ctypes.data)
    return CheckResult(*[int(v) for v in out])


def enumerate_matchings(csr, maximal_only: bool = True) -> np.ndarray:
    """All (maximal) matchings of a graph with n <= 20, as an (K, n) array of
    mate arrays."""
    off, off64, nbr = _graph_args(csr)
    lib = _load()
    n = csr.n
    cnt = lib.oracle_enumerate(n, off.ctypes.data, off64, nbr.ctypes.data, int(maximal_only), None, 0)
    if cnt < 0:
        raise ValueError("enumeration needs n <= 20 and valid ids")
    out = np.empty((cnt, max(n, 1)), dtype=np.int32)
    lib.oracle_enumerate(n, off.ctypes.data, off64, nbr.ctypes.data, int(maximal_only),
                         out.ctypes.data, cnt)
    return out[:, :n]


def greedy_weighted(csr, seed: int):
    """(mate, pairs): the greedy matching over undirected edges in descending
    order of edge_weight (ties: smaller (min, max) key first)."""
    off, off64, nbr = _graph_args(csr)
    mate = np.empty(csr.n, dtype=np.int32)
    pairs = _load().oracle_greedy_weighted(csr.n, off.ctypes.data, off64, nbr.ctypes.data,
                                           seed, mate.ctypes.data)
    if pairs < 0:
        raise MemoryError("oracle_greedy_weighted ran out of memory")
    return mate, int(pairs)


def edge_weight(u: int, v: int, seed: int) -> int:
    return int(_load().oracle_edge_weight(u, v, seed))


def splitmix64(x: int) -> int:
    return int(_load().oracle_splitmix64(x))
