"""ctypes binding of the protocol model (protocol_model.c): test
infrastructure only. The C file is compiled with gcc on first use."""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "protocol_model.c")
_LIB = os.path.join(_HERE, "libprotocol_model.so")
_lock = threading.Lock()
_lib = None

MAXN, MAXM, MAXL, MAXS = 8, 64, 4, 8
LAYOUTS = {"word": 0, "u8": 1, "u2": 2}


class Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("off", ctypes.c_int * (MAXN + 1)), ("nbr", ctypes.c_int * MAXM)]


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", _SRC, "-o", tmp],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            P, I, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
            lib.pm_run.restype = I64
            lib.pm_run.argtypes = [ctypes.POINTER(Graph), P, I, P, P, I, I, ctypes.c_uint64, I64, P]
            lib.pm_explore.restype = I64
            lib.pm_explore.argtypes = [ctypes.POINTER(Graph), P, I, P, P, I, I64,
                                       ctypes.POINTER(I64), P, I, ctypes.POINTER(I)]
            lib.pm_sizeof_graph.restype = I
            assert lib.pm_sizeof_graph() == ctypes.sizeof(Graph)
            _lib = lib
        return _lib


def graph(csr) -> Graph:
    g = Graph()
    assert csr.n <= MAXN and csr.m <= MAXM
    g.n = csr.n
    for i, o in enumerate(csr.off):
        g.off[i] = int(o)
    for i, y in enumerate(csr.nbr):
        g.nbr[i] = int(y)
    return g


def variant(layout="word", two_phase=0, wait_release=0, lazy=0, scan_width=2, stale=1, upper=0,
            mutant=0, probe=0):
    """upper: 1 each edge from its lower end, 2 the same with a scan ending at
    the first neighbour below its source (lists ordered upper neighbours
    first). probe: 1 a source's first state read takes its first candidate
    only, 2 every state read takes one. mutant: a planted mistake (1 no id
    order, 2 no release of u, 3 v taken by a plain store after a read); 0 for
    the protocol itself."""
    return np.array([LAYOUTS[layout], two_phase, wait_release, lazy, scan_width, stale, upper,
                     mutant, probe], dtype=np.int32)


def lanes(n, waves, per_wave, mode="blocks"):
    """Sources 0 .. n-1 dealt to waves x per_wave lanes: in consecutive blocks
    (each lane a run of ids, as a wavefront's block) or round robin."""
    L = waves * per_wave
    src = -np.ones((L, MAXS), dtype=np.int32)
    if mode == "blocks":
        per = (n + L - 1) // L
        for l in range(L):
            ids = list(range(l * per, min(n, (l + 1) * per)))
            src[l, :len(ids)] = ids
    else:
        for l in range(L):
            ids = list(range(l, n, L))
            src[l, :len(ids)] = ids
    wave_of = np.array([l // per_wave for l in range(L)], dtype=np.int32)
    return wave_of, src


def run(g: Graph, var, wave_of, src, strategy=0, seed=1, max_trips=100000):
    lib = load()
    mate = np.full(g.n, -7, dtype=np.int32)
    r = lib.pm_run(ctypes.byref(g), var.ctypes.data, len(wave_of), wave_of.ctypes.data,
                   src.ctypes.data, src.shape[1], strategy, seed, max_trips, mate.ctypes.data)
    return int(r), mate


def explore(g: Graph, var, wave_of, src, max_states=400000, max_outs=256):
    lib = load()
    stuck = ctypes.c_int64(0)
    n_outs = ctypes.c_int(0)
    outs = np.zeros((max_outs, max(g.n, 1)), dtype=np.int32)
    states = lib.pm_explore(ctypes.byref(g), var.ctypes.data, len(wave_of), wave_of.ctypes.data,
                            src.ctypes.data, src.shape[1], max_states, ctypes.byref(stuck),
                            outs.ctypes.data, max_outs, ctypes.byref(n_outs))
    k = max(n_outs.value, 0)
    return int(states), int(stuck.value), n_outs.value, [outs[i, :g.n].copy() for i in range(k)]
