"""Autotuner logic on the CPU: the coordinate search with a synthetic
objective (no device), rejection of candidates that fail the check, the
stored-JSON lookup and the degree-based graph classes."""
import json

import numpy as np

import graphgen
from paper_2507_04420_amd import Tuning, _lib, autotune


class FakeTarget:
    unit = "x/s"
    sample = "synthetic"

    def __init__(self, bad_layout=None):
        self.calls = 0
        self.bad_layout = bad_layout

    def measure(self, t):
        self.calls += 1
        if t.layout == self.bad_layout:
            return None  # fails the check
        # best at wave 2048, wg 128, assist 32, hint on, U8 layout
        score = 100.0
        score -= abs(np.log2(t.wave_vertices / 2048)) * 5
        score -= abs(np.log2(t.wg_size / 128)) * 3
        score -= abs(np.log2(t.assist_after / 32)) * 2
        score += 4 * (t.hint == 1)
        score += {_lib.MM_LAYOUT_U8: 6, _lib.MM_LAYOUT_U32: 0, _lib.MM_LAYOUT_U2: 1}[t.layout]
        return score


def test_search_finds_separable_optimum():
    r = autotune.search(FakeTarget(), passes=3, log=lambda s: None)
    t = r["tuning"]
    assert t["wave_vertices"] == 2048 and t["wg_size"] == 128 and t["assist_after"] == 32
    assert t["hint"] == 1 and t["layout"] == _lib.MM_LAYOUT_U8
    assert r["objective"] > r["default_objective"]
    assert r["rejected"] == 0


def test_search_never_keeps_a_rejected_candidate():
    r = autotune.search(FakeTarget(bad_layout=_lib.MM_LAYOUT_U8), passes=2, log=lambda s: None)
    assert r["tuning"]["layout"] != _lib.MM_LAYOUT_U8
    assert r["rejected"] >= 1


def test_tuned_lookup(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "TUNED_DIR", str(tmp_path))
    assert autotune.tuned("rmat", key="dev_1cu") == Tuning.default()
    t = Tuning.default().as_dict()
    t["wave_vertices"] = 512
    (tmp_path / "dev_1cu.json").write_text(json.dumps({"device": "dev_1cu", "classes": {"rmat": {"tuning": t}}}))
    assert autotune.tuned("rmat", key="dev_1cu").wave_vertices == 512
    assert autotune.tuned("grid", key="dev_1cu") == Tuning.default()


def test_classify(monkeypatch):
    # below SMALL_VERTICES every kind is "_small"
    assert autotune.classify(graphgen.grid(50, 60).off) == "grid_small"
    assert autotune.classify(graphgen.er(20000, 16, seed=1).off) == "er_small"
    assert autotune.classify(graphgen.rmat(16, seed=1).off) == "rmat_small"
    assert autotune.classify(graphgen.rmat(18, 8, seed=1).off) == "rmat_mid"
    assert autotune.classify(graphgen.grid(512, 512).off) == "grid_mid"
    # the vertex count alone decides small, mid and large
    monkeypatch.setattr(autotune, "SMALL_VERTICES", 2000)
    monkeypatch.setattr(autotune, "MID_VERTICES", 3000)
    assert autotune.classify(graphgen.grid(50, 60).off) == "grid"
    assert autotune.classify(graphgen.grid(50, 59).off) == "grid_mid"
    assert autotune.classify(graphgen.grid(40, 49).off) == "grid_small"
    assert autotune.classify(graphgen.rmat(16, seed=1).off) == "rmat"
    assert autotune.classify(graphgen.er(20000, 16, seed=1).off) == "er"
    assert autotune.classify(graphgen.er(1500, 8, seed=1).off) == "er_small"


def test_small_class_without_entry_takes_the_defaults(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "TUNED_DIR", str(tmp_path))
    doc = {"device": "dev_3cu", "classes": {"rmat": {"tuning": dict(Tuning().as_dict(), wave_vertices=64)}}}
    (tmp_path / "dev_3cu.json").write_text(json.dumps(doc))
    assert autotune.tuned("rmat_small", key="dev_3cu") == Tuning.default()


def test_search_falls_back_to_fewer_waves_in_flight():
    # a target that only accepts shapes with at most 16 wavefronts of a small
    # graph in flight: the search starts from the first conservative shape
    class Reproducible(FakeTarget):
        def measure(self, t):
            if t.min_waves == 0 or t.min_waves > 16:
                return None
            return super().measure(t)
    r = autotune.search(Reproducible(), passes=1, log=lambda s: None)
    assert r["tuning"]["min_waves"] <= 16 and r["default_objective"] is not None


def test_search_restarts_from_defaults_when_the_start_is_rejected():
    # a stored entry that fails (here: a layout the target rejects) is replaced
    # by the library defaults as the starting point
    r = autotune.search(FakeTarget(bad_layout=_lib.MM_LAYOUT_U2), start=Tuning(layout=_lib.MM_LAYOUT_U2),
                        passes=1, log=lambda s: None)
    assert r["default_objective"] is not None
    assert r["tuning"]["layout"] != _lib.MM_LAYOUT_U2


def test_spread_limit_is_a_tenth_of_the_serving_tolerance():
    # under a tenth of the 1% alone-vs-mix tolerance
    assert 0.0005 <= autotune.SPREAD_LIMIT <= 0.001
    assert set(autotune.REPRODUCIBLE) >= {"rmat_small", "grid_small", "er_small", "rmat_mid", "grid_mid"}


def test_mid_class_falls_back_to_its_kind(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "TUNED_DIR", str(tmp_path))
    doc = {"device": "dev_2cu", "classes": {"grid": {"tuning": dict(Tuning().as_dict(), wave_vertices=128)},
                                            "rmat_mid": {"tuning": dict(Tuning().as_dict(), disperse=1)}}}
    (tmp_path / "dev_2cu.json").write_text(json.dumps(doc))
    assert autotune.tuned("grid_mid", key="dev_2cu").wave_vertices == 128
    assert autotune.tuned("rmat_mid", key="dev_2cu").disperse == 1
    assert autotune.tuned("rmat", key="dev_2cu") == Tuning.default()


def test_stored_tunings_are_valid():
    # every committed tuning must be accepted by the library's own check
    import glob
    import ctypes
    lib = _lib.load()
    for path in glob.glob(autotune.TUNED_DIR + "/*.json"):
        with open(path) as f:
            doc = json.load(f)
        for cls, entry in doc["classes"].items():
            ct = Tuning(**entry["tuning"]).to_c()
            assert lib.mm_workspace_bytes_graph(1000, 5000, ctypes.byref(ct)) > 0, (path, cls)


def test_search_holds_fixed_fields():
    class Fixed(FakeTarget):
        fixed = {"relabel": 0}
        dims = ["wave_vertices", "scan_width"]
    r = autotune.search(Fixed(), start=Tuning(relabel=1), passes=1, log=lambda s: None)
    assert r["tuning"]["relabel"] == 0


def test_serving_classes_search_without_copies():
    # the classes a serving request can fall in are searched with the graph
    # as given: no relabelled or reordered copy, neither as a start nor as a
    # candidate
    class Target(FakeTarget):
        fixed = dict(autotune.COPIES)
        dims = ["wave_vertices", "scan_width"]
    r = autotune.search(Target(), start=Tuning(relabel=1, order_lists=1), passes=1,
                        log=lambda s: None)
    assert r["tuning"]["relabel"] == 0 and r["tuning"]["order_lists"] == 0
    assert set(autotune.COPIES) == {"relabel", "order_lists"}


def test_multi_target_objective():
    class Part:
        def __init__(self, m, rate):
            self.m, self.rate, self.sample = m, rate, "p"
            self.dims, self.fixed = ["hint"], {}

        def measure(self, t):
            return self.rate
    mt = autotune.MultiTarget.__new__(autotune.MultiTarget)
    mt.parts = [Part(100, 1.0), Part(300, 3.0)]  # 100e-9 s + 100e-9 s
    assert abs(mt.measure(Tuning()) - 2.0) < 1e-9
    mt.parts.append(Part(5, None))
    assert mt.measure(Tuning()) is None


def test_relabelling_must_win_by_its_premium():
    # relabelled candidates count 3% slower: a 2% gain does not buy the copy,
    # a 5% gain does, and a relabelled start gives way to a natural order
    # that measures 1% slower
    class Relabel(FakeTarget):
        dims = ["relabel"]

        def __init__(self, gain):
            super().__init__()
            self.gain = gain

        def measure(self, t):
            return 100.0 * (self.gain if t.relabel else 1.0)
    assert autotune.search(Relabel(1.02), passes=1, log=lambda s: None)["tuning"]["relabel"] == 0
    assert autotune.search(Relabel(1.05), passes=1, log=lambda s: None)["tuning"]["relabel"] == 1
    r = autotune.search(Relabel(1.01), start=Tuning(relabel=1), passes=1, log=lambda s: None)
    assert r["tuning"]["relabel"] == 0


def test_paired_dimensions_move_together():
    t = autotune._with(Tuning(), "upper_wait", (1, 1))
    assert t.upper_only == 1 and t.wait_release == 1
    assert autotune._value(t, "upper_wait") == (1, 1)
    assert autotune._value(t, "layout_protocol") == (t.layout, t.protocol)
