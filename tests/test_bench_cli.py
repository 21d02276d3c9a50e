"""bench.py pieces that run without a GPU: the one-GPU guard, the lookup
of stored HBM traffic (only valid for the kernel sources and workload it was
taken on), the algorithmic bytes and the leg names."""
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
    assert bench.stored_traffic(cfg) == (None, None)  # no file
    rec = {"kernel_sources_sha256": bench.kernel_sources_sha256(), "config": cfg,
           "hbm_bytes_per_launch": 4.5e10}
    f.write_text(json.dumps(rec))
    traffic, stored = bench.stored_traffic(cfg)
    assert traffic == 4.5e10 and stored == rec  # the record it comes from is reported with it
    assert bench.stored_traffic(dict(cfg, scale=26)) == (None, None)  # other workload
    f.write_text(json.dumps(dict(rec, kernel_sources_sha256="0" * 64)))
    assert bench.stored_traffic(cfg) == (None, None)  # kernel changed since


def test_code_hash_ignores_comments_only():
    # the stored traffic stays valid across a change of comments, and not
    # across a change of code (string literals are code)
    a = 'int f(int x) { // one\n  return x + 1; /* two */ }\nconst char* s = "// kept";\n'
    b = '/* header */\nint f(int x) {\n\n  return x + 1;   }\nconst char* s = "// kept";  // more\n'
    assert bench.strip_comments(a) == bench.strip_comments(b)
    assert bench.strip_comments(a) != bench.strip_comments(a.replace("x + 1", "x + 2"))
    assert bench.strip_comments(a) != bench.strip_comments(a.replace('"// kept"', '"kept"'))
    assert "one" not in bench.strip_comments(a) and "two" not in bench.strip_comments(a)


def test_algorithmic_bytes():
    # per source w + 1 + 4, per id of a sequential pass 4 + 1 (the sweep's
    # units); with the states once per vertex instead: w(n+1) + 4 T + 2n + 4n
    assert bench.sweep_bytes(8, 10, 100) == 8 * 11 + 500 + 10 + 40
    assert bench.sweep_bytes_d1(8, 10, 100) == 8 * 11 + 400 + 20 + 40
    # the 16384^2 grid's closed-form T_seq (402,628,608) gives 5.37 GB
    n = 16384 * 16384
    assert abs(bench.sweep_bytes_d1(8, n, 402628608) - 5.369e9) < 1e7


def test_workload_classes_and_legs():
    assert bench.workload_class("er65536") == "er"
    assert bench.workload_class("rmat27") == "rmat" and bench.workload_class("grid16384") == "grid"
    assert set(bench.LEGS) == {"headline", "er65536", "rmat24", "grid16384", "batch", "serve"}
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--legs", "nope"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "unknown legs" in (r.stderr + r.stdout)


def test_variants_are_valid_tunings():
    import ctypes
    import paper_2507_04420_amd as mm
    from paper_2507_04420_amd import _lib
    from paper_2507_04420_amd import autotune
    lib = _lib.load()
    # over the defaults and over each single-graph workload's tuned entry,
    # which the bench's variants override
    bases = [mm.Tuning()] + [autotune.tuned(c, key="gfx950_256cu") for c in ("rmat", "er", "grid")]
    for base in bases:
        for name, over in bench.VARIANTS.items():
            t = mm.Tuning(**dict(base.as_dict(), **over)).to_c()
            assert lib.mm_workspace_bytes_graph(1000, 5000, ctypes.byref(t)) > 0, (name, base)
