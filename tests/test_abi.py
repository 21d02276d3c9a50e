"""The C-ABI library loads and exports every entry point of include/mm.h;
host-side argument checks return their documented status codes (no GPU call
is made before these checks)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2507_04420_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(mm_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for must in ("mm_create", "mm_run", "mm_destroy", "mm_workspace_bytes", "mm_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_version_and_defaults():
    lib = _lib.load()
    assert lib.mm_version().startswith(b"skipper-gfx950")
    t = _lib.mm_tuning()
    lib.mm_default_tuning(ctypes.byref(t))
    assert t.layout in (_lib.MM_LAYOUT_U8, _lib.MM_LAYOUT_U32, _lib.MM_LAYOUT_U2)
    assert t.wg_size % 64 == 0 and t.wave_vertices % 64 == 0
    # the ctypes mirror has the C layout: the last fields read back as written
    assert t.whole_graph_vertices == 16384 and t.iter_cap == 0 and t.whole_graph_lds == 1
    assert t.hot_degree == 2048 and t.probe_first == 0 and t.occupancy == 0
    assert ctypes.sizeof(_lib.mm_tuning) == 104
    from paper_2507_04420_amd import Tuning
    assert Tuning.default() == Tuning()  # the Python defaults mirror the library's


def test_workspace_bytes():
    lib = _lib.load()
    t = _lib.mm_tuning()
    lib.mm_default_tuning(ctypes.byref(t))
    t.layout = _lib.MM_LAYOUT_U8
    small = lib.mm_workspace_bytes(0, ctypes.byref(t))
    big = lib.mm_workspace_bytes(1 << 20, ctypes.byref(t))
    assert small > 0 and big >= small + (1 << 20) // 4 * 4
    t.layout = _lib.MM_LAYOUT_U2
    assert lib.mm_workspace_bytes(1 << 20, ctypes.byref(t)) == small + (1 << 20) // 4
    assert lib.mm_workspace_bytes(-1, ctypes.byref(t)) == 0
    assert lib.mm_workspace_bytes(1 << 31, ctypes.byref(t)) == 0
    t.layout = _lib.MM_LAYOUT_U32
    assert lib.mm_workspace_bytes(1 << 20, ctypes.byref(t)) == small
    t.hint = 1
    assert lib.mm_workspace_bytes(1 << 20, ctypes.byref(t)) == small + (1 << 20) // 8
    t.wg_size = 100
    assert lib.mm_workspace_bytes(10, ctypes.byref(t)) == 0


def _create(lib, **kw):
    args = dict(off=ctypes.c_void_p(0x1000), off_type=_lib.MM_OFF_I64, nbr=ctypes.c_void_p(0x2000),
                n=10, m=20, ws=ctypes.c_void_p(0x100000), ws_bytes=1 << 20, flags=0, tuning=None)
    args.update(kw)
    h = ctypes.c_void_p()
    st = lib.mm_create(args["off"], args["off_type"], args["nbr"], args["n"], args["m"], args["ws"],
                       args["ws_bytes"], args["flags"], args["tuning"], None, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("kw,status", [
    (dict(off=None), _lib.MM_ERR_INVALID_ARG),
    (dict(nbr=None), _lib.MM_ERR_INVALID_ARG),
    (dict(ws=None), _lib.MM_ERR_INVALID_ARG),
    (dict(ws=ctypes.c_void_p(0x100004)), _lib.MM_ERR_INVALID_ARG),
    (dict(n=-1), _lib.MM_ERR_INVALID_ARG),
    (dict(n=1 << 31), _lib.MM_ERR_INVALID_ARG),
    (dict(m=-5), _lib.MM_ERR_INVALID_ARG),
    (dict(off_type=_lib.MM_OFF_I32, m=1 << 31), _lib.MM_ERR_INVALID_ARG),
    (dict(off_type=7), _lib.MM_ERR_INVALID_ARG),
    (dict(flags=0x80), _lib.MM_ERR_INVALID_ARG),
    (dict(ws_bytes=16), _lib.MM_ERR_OUT_OF_MEMORY),
])
def test_create_argument_errors(kw, status):
    lib = _lib.load()
    st, h = _create(lib, **kw)
    assert st == status
    assert not h.value
    assert lib.mm_last_error()


def test_create_bad_tuning():
    lib = _lib.load()
    t = _lib.mm_tuning()
    lib.mm_default_tuning(ctypes.byref(t))
    t.wave_vertices = 100
    st, _ = _create(lib, tuning=ctypes.pointer(t))
    assert st == _lib.MM_ERR_INVALID_ARG
    assert b"wave_vertices" in lib.mm_last_error()
    for field, bad in (("protocol", 2), ("hint", 3), ("hint", -1), ("scan_width", 0), ("scan_width", 9),
                       ("layout", 5), ("stream_loads", 2), ("whole_graph_vertices", -1), ("relabel", 3),
                       ("relabel", -1),
                       ("hub_degree", -1), ("whole_graph_lds", 2), ("wait_release", 2),
                       ("mesh_wave_vertices", 100), ("hub_wave", 3), ("hub_wave", -1),
                       ("upper_only", 2), ("min_waves", -1), ("order_lists", 3),
                       ("order_lists", -1),
                       ("order_lists", 2),  # upper neighbours first needs upper_only = 1
                       ("probe_first", 3), ("probe_first", -1), ("occupancy", 5), ("occupancy", 8),
                       ("iter_cap", -1)):
        lib.mm_default_tuning(ctypes.byref(t))
        setattr(t, field, bad)
        st, _ = _create(lib, tuning=ctypes.pointer(t))
        assert st == _lib.MM_ERR_INVALID_ARG, field
        assert field.encode() in lib.mm_last_error(), field


def test_null_handle_calls():
    lib = _lib.load()
    assert lib.mm_run(None, None, None) == _lib.MM_ERR_INVALID_ARG
    assert lib.mm_sync(None, None) == _lib.MM_ERR_INVALID_ARG
    assert lib.mm_reset_stats(None, None) == _lib.MM_ERR_INVALID_ARG
    s = _lib.mm_stats()
    assert lib.mm_get_stats(None, None, ctypes.byref(s)) == _lib.MM_ERR_INVALID_ARG
    c = (ctypes.c_int64 * 6)()
    assert lib.mm_check(None, None, None, c) == _lib.MM_ERR_INVALID_ARG
    assert lib.mm_batch_check(None, None, None, c) == _lib.MM_ERR_INVALID_ARG
    assert lib.mm_ems_run(None, None, 1, None, 0, None, None) == _lib.MM_ERR_INVALID_ARG
    assert lib.mm_ems_scratch_bytes(-1) == 0 and lib.mm_ems_scratch_bytes(1000) >= 4000
    cnt = ctypes.c_int64()
    assert lib.mm_pairs(None, None, None, None, 0, ctypes.byref(cnt)) == _lib.MM_ERR_INVALID_ARG
    lib.mm_destroy(None)


def test_list_batch_argument_errors():
    lib = _lib.load()
    h = ctypes.c_void_p()
    t = _lib.mm_tuning()
    lib.mm_default_tuning(ctypes.byref(t))
    ws = ctypes.c_void_p(4096 * 256)  # aligned, never dereferenced: creation fails first
    n = (ctypes.c_int64 * 1)(-1)
    m = (ctypes.c_int64 * 1)(0)
    ptrs = (ctypes.c_void_p * 1)(None)
    st = lib.mm_batch_create_list(ptrs, ptrs, n, m, 1, ws, 1 << 20, 0, ctypes.byref(t), None,
                                  ctypes.byref(h))
    assert st == _lib.MM_ERR_INVALID_ARG and not h.value
    n[0], m[0] = 0, 5  # an empty graph with entries
    assert lib.mm_batch_create_list(ptrs, ptrs, n, m, 1, ws, 1 << 20, 0, ctypes.byref(t), None,
                                    ctypes.byref(h)) == _lib.MM_ERR_INVALID_ARG
    n[0], m[0] = 4, 2  # null device pointers
    assert lib.mm_batch_create_list(ptrs, ptrs, n, m, 1, ws, 1 << 20, 0, ctypes.byref(t), None,
                                    ctypes.byref(h)) == _lib.MM_ERR_INVALID_ARG
    assert lib.mm_batch_create_list(ptrs, ptrs, n, m, -1, ws, 1 << 20, 0, ctypes.byref(t), None,
                                    ctypes.byref(h)) == _lib.MM_ERR_INVALID_ARG
    assert lib.mm_batch_create_list(ptrs, ptrs, n, m, 1, ctypes.c_void_p(4096 * 256 + 8), 1 << 20,
                                    0, ctypes.byref(t), None, ctypes.byref(h)) == _lib.MM_ERR_INVALID_ARG


def test_error_raises_python_exception():
    with pytest.raises(_lib.MMError) as ei:
        _lib.check(_lib.MM_ERR_INVALID_ARG)
    assert ei.value.status == _lib.MM_ERR_INVALID_ARG


def test_stats_struct_and_conflict_row():
    import paper_2507_04420_amd as mm
    assert ctypes.sizeof(_lib.mm_stats) == 32 * 8
    s = _lib.mm_stats()
    s.reserve_conflicts, s.match_conflicts, s.conflict_max = 7, 3, 5
    s.reserve_matched, s.match_matched = 2, 1
    for b, c in enumerate([4, 1, 0, 1]):
        s.conflict_hist[b] = c
    d = _lib.stats_dict(s)
    row = mm.conflict_row(d)
    # Table II counts every failed take of u or v, whatever state it met
    assert row["total"] == 13 and row["edges"] == 6 and row["max_per_edge"] == 5
    assert row["met_reserved"] == 10 and row["met_matched"] == 3
    assert row["distribution"]["1"] == 4 and row["distribution"]["5-8"] == 1
    assert abs(row["avg_per_edge"] - 13 / 6) < 1e-12


def test_workspace_bytes_graph():
    lib = _lib.load()
    t = _lib.mm_tuning()
    lib.mm_default_tuning(ctypes.byref(t))
    base = lib.mm_workspace_bytes(1000, ctypes.byref(t))
    assert lib.mm_workspace_bytes_graph(1000, 5000, ctypes.byref(t)) == base
    t.relabel = 1
    assert lib.mm_workspace_bytes(1000, ctypes.byref(t)) == 0
    big = lib.mm_workspace_bytes_graph(1000, 5000, ctypes.byref(t))
    assert big >= base + 4 * 1000 + 8 * 1001 + 4 * 1000 + 4 * 5000
    assert lib.mm_workspace_bytes_graph(1000, -1, ctypes.byref(t)) == 0
    vtx = (ctypes.c_int64 * 2)(0, 10)
    assert lib.mm_batch_workspace_bytes(1, vtx, ctypes.byref(t)) == 0
    # the hot-vertices-last order needs the same copy, and a threshold
    t.relabel = 2
    assert lib.mm_workspace_bytes_graph(1000, 5000, ctypes.byref(t)) == big
    t.hot_degree = 0
    assert lib.mm_workspace_bytes_graph(1000, 5000, ctypes.byref(t)) == 0
    # reordered lists: a copy of the ids only, and not with a relabelled copy
    t.hot_degree = 2048
    t.order_lists = 1
    assert lib.mm_workspace_bytes_graph(1000, 5000, ctypes.byref(t)) == 0
    t.relabel = 0
    assert lib.mm_workspace_bytes(1000, ctypes.byref(t)) == 0
    assert lib.mm_workspace_bytes_graph(1000, 5000, ctypes.byref(t)) == base + 20224  # 4m to 256 B
    assert lib.mm_create_device_bytes(1000, 5000, ctypes.byref(t)) >= 1000
    assert lib.mm_batch_workspace_bytes(1, vtx, ctypes.byref(t)) == 0
    # upper neighbours first: the same copy in another order, with upper_only only
    t.order_lists = 2
    assert lib.mm_workspace_bytes_graph(1000, 5000, ctypes.byref(t)) == 0
    t.upper_only = 1
    with_upper = lib.mm_workspace_bytes_graph(1000, 5000, ctypes.byref(t))
    t.order_lists = 1
    assert with_upper == lib.mm_workspace_bytes_graph(1000, 5000, ctypes.byref(t)) > 0
    t.upper_only = 0


def _batch_bytes(lib, ns, **kw):
    t = _lib.mm_tuning()
    lib.mm_default_tuning(ctypes.byref(t))
    for k, v in kw.items():
        setattr(t, k, v)
    vtx = (ctypes.c_int64 * (len(ns) + 1))(*np.concatenate([[0], np.cumsum(ns)]).tolist())
    return lib.mm_batch_workspace_bytes(len(ns), vtx, ctypes.byref(t))


def test_batch_workspace_short_blocks_and_mesh_room():
    # host-side plan: a batch too small for 2048 wavefronts of wave_vertices
    # sources is cut into short blocks whatever wave_vertices says, so its
    # item table (16 bytes an item) does not depend on it
    lib = _lib.load()
    small = [20000, 20000]
    a = _batch_bytes(lib, small, whole_graph_vertices=0, wave_vertices=2048, min_waves=2048)
    b = _batch_bytes(lib, small, whole_graph_vertices=0, wave_vertices=64, min_waves=2048)
    assert a == b > 0
    # with about 32 wavefronts (the default) the 40000 sources take blocks of
    # 1280: 32 items instead of 626
    a32 = _batch_bytes(lib, small, whole_graph_vertices=0, wave_vertices=2048, min_waves=32)
    assert a32 == a - 256 * ((626 * 16 + 255) // 256 - (32 * 16 + 255) // 256)
    # min_waves = 0 never shortens
    z = _batch_bytes(lib, small, whole_graph_vertices=0, wave_vertices=2048, min_waves=0)
    assert z <= a32
    # a large batch keeps its blocks: longer blocks, fewer items, fewer bytes
    large = [1 << 21] * 4
    c = _batch_bytes(lib, large, whole_graph_vertices=0, wave_vertices=2048)
    d = _batch_bytes(lib, large, whole_graph_vertices=0, wave_vertices=1024)
    items_c, items_d = 4 * (1 << 21) // 2048, 4 * (1 << 21) // 1024
    assert d - c >= 16 * (items_d - items_c) - 256
    # room for mesh blocks: with mesh_wave_vertices shorter than wave_vertices
    # the plan reserves items for the shorter blocks
    e = _batch_bytes(lib, large, whole_graph_vertices=0, wave_vertices=2048, mesh_wave_vertices=128)
    assert e - c >= 16 * (4 * (1 << 21) // 128 - items_c) - 256
    # graphs swept whole are one item each, however large wave_vertices is
    f = _batch_bytes(lib, [1000] * 8, wave_vertices=64)
    g = _batch_bytes(lib, [1000] * 8, wave_vertices=4096)
    assert f == g


def test_probe_rejects_bad_arguments_without_a_device():
    lib = _lib.load()
    r, a = ctypes.c_double(), ctypes.c_double()
    assert lib.mm_probe_ceilings(100, 10, None, ctypes.byref(r), ctypes.byref(a)) == _lib.MM_ERR_INVALID_ARG
    assert lib.mm_probe_ceilings(1 << 20, 0, None, ctypes.byref(r), ctypes.byref(a)) == _lib.MM_ERR_INVALID_ARG
    assert lib.mm_probe_ceilings(1 << 20, 10, None, None, ctypes.byref(a)) == _lib.MM_ERR_INVALID_ARG
