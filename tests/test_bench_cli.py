"""bench.py pieces that run without a GPU: the one-GPU guard and the lookup
of measured HBM traffic (only valid for the kernel sources and workload it was
taken on)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_lookup(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    cfg = {"workload": "rmat", "scale": 27, "tuning": {"layout": 1}}
    assert bench.measured_traffic(cfg) is None  # no file
    f.write_text(json.dumps({"kernel_sources_sha256": bench.kernel_sources_sha256(), "config": cfg,
                             "hbm_bytes_per_launch": 4.5e10}))
    assert bench.measured_traffic(cfg) == 4.5e10
    assert bench.measured_traffic(dict(cfg, scale=26)) is None  # other workload
    f.write_text(json.dumps({"kernel_sources_sha256": "0" * 64, "config": cfg,
                             "hbm_bytes_per_launch": 4.5e10}))
    assert bench.measured_traffic(cfg) is None  # kernel changed since


def test_variants_are_valid_tunings():
    import ctypes
    import paper_2507_04420_amd as mm
    from paper_2507_04420_amd import _lib
    lib = _lib.load()
    for name, over in bench.VARIANTS.items():
        t = mm.Tuning(**dict(mm.Tuning().as_dict(), **over)).to_c()
        assert lib.mm_workspace_bytes_graph(1000, 5000, ctypes.byref(t)) > 0, name
