"""Benchmark: single-pass maximal matching (Skipper) on one MI355X.

One step = one full matching pass (state initialisation + sweep) over a graph
resident in HBM. The default workload is R-MAT scale 27, edge factor 16,
(a, b, c) = (0.57, 0.19, 0.19), symmetrised, deduplicated, ids permuted.

value  = m / (ms_per_step) in GEdges/s, m = directed CSR entries.
roofline: the sweep kernel's algorithmic bytes per launch
          (offsets w(n+1) + source states n + mates 4n + per id read 4 B and
          its state byte, 5*T_seq, T_seq = ids SGMM reads) over its mean
          duration from HIP events
          recorded on the launch stream, against 8 TB/s.
cpu_baseline: the oracle's single-thread SGMM on the host, on the same graph.
batch: the 4096-graph mixture in one captured persistent launch against one
       launch per graph; serve: Poisson request streams over resident graphs
       (p50/p99 arrival-to-result latency, GEdges/s).
Tunings come from the package's autotuned table for this device and graph
class (library defaults where it has none).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "GEdges/s single-pass MM + % HBM roofline; batched vs per-graph graphs/s"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_kernel_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2507_04420_amd", "csrc", f)
                  for f in ("protocol.h", "sweep.h", "mm.hip", "relabel.hip", "hubs.hip")]


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(config) -> float | None:
    """HBM bytes per sweep launch from the committed rocprofv3 FETCH_SIZE and
    WRITE_SIZE runs (scaled by a plain copy of known size), if they were taken
    on the current kernel sources with this workload and tuning; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    if t.get("config") != json.loads(json.dumps(config)):
        return None
    return float(t["hbm_bytes_per_launch"])


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_workload(name: str, seed: int):
    import graphgen
    if name == "er65536":
        return graphgen.er(65536, 16, seed=seed).with_int32_offsets(), {
            "workload": "er", "n": 65536, "avg_degree": 16, "offsets": "int32", "seed": seed}
    if name.startswith("rmat"):
        scale = int(name[4:])
        return graphgen.rmat(scale, 16, seed=seed), {
            "workload": "rmat", "scale": scale, "edge_factor": 16, "abc": [0.57, 0.19, 0.19],
            "permuted": True, "offsets": "int64", "seed": seed}
    if name.startswith("grid"):
        side = int(name[4:])
        return graphgen.grid(side, side), {"workload": "grid", "rows": side, "cols": side,
                                           "offsets": "int64"}
    raise SystemExit("unknown workload %r" % name)


def host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "?")
    except OSError:
        model = "?"
    return "%s, %d logical CPUs visible" % (model, os.cpu_count() or 0)


def cpu_baseline(csr, budget_s: float = 30.0):
    """Times the oracle's single-thread SGMM (untuned) on the host."""
    import oracle
    times = []
    res = None
    while True:
        t0 = time.perf_counter()
        res = oracle.sgmm(csr)
        times.append(time.perf_counter() - t0)
        if len(times) >= 3 or sum(times) * (len(times) + 1) / len(times) > budget_s:
            break
    t = float(np.median(times))
    return res, t, len(times)


# Design-choice variants (--variants): overrides of the tuned tuning, one
# choice at a time, each timed and counted on the same resident graph.
VARIANTS = {
    "tuned": {},
    "natural_order": {"relabel": 0},
    "u8_byte_cas": {"layout": 0, "protocol": 0, "lazy_init": 0},
    "u8_byte_cas_lazy": {"layout": 0, "protocol": 0, "lazy_init": 1},
    "u2_two_phase": {"layout": 2, "protocol": 1, "lazy_init": 0},
    "u32_two_phase": {"layout": 1, "protocol": 1, "lazy_init": 0},
    "hint_bits": {"hint": 1},
    "hint_bytes": {"hint": 2},
    "no_hint": {"hint": 0},
    "assist_16": {"assist_after": 16},
    "assist_256": {"assist_after": 256},
    "no_assist": {"assist_after": 0},
    "contiguous_lanes": {"disperse": 0},
    "dispersed_lanes": {"disperse": 1},
    "wait_release": {"wait_release": 1},
}


def bench_variants(args, csr, off, nbr, base, t_seq):
    """Times each named variant (sweep mean over `steps` passes after one
    warm-up) and counts its work in a separate instrumented pass."""
    import paper_2507_04420_amd as mm
    rows = []
    w = csr.off.dtype.itemsize
    for name in args.variants.split(","):
        t = mm.Tuning(**dict(base.as_dict(), **VARIANTS[name]))
        g = mm.Graph(off, nbr, symmetric=True, timing=True, tuning=t)
        out = g.run()
        g.sync()
        g.timing()
        for _ in range(args.steps):
            g.run(out)
        g.sync()
        tm = g.timing()
        chk = g.check(out)
        g.close()
        gs = mm.Graph(off, nbr, symmetric=True, stats=True, tuning=t)
        o2 = gs.run()
        gs.sync()
        st = gs.stats()
        gs.close()
        del o2
        sweep_s = tm["mean_ms"] / 1e3
        b_sweep = w * (csr.n + 1) + 5 * t_seq + csr.n + 4 * csr.n
        row = {"variant": name, "tuning": t.as_dict(), "sweep_ms": round(tm["mean_ms"], 4),
               "gedges_per_s": round(csr.m / sweep_s / 1e9, 1),
               "alg_gbs": round(b_sweep / sweep_s / 1e9, 1),
               "violations": sum(chk[k] for k in ("out_of_range", "self_mate", "asymmetric",
                                                  "not_edge", "uncovered")),
               "size": chk["matched"] // 2,
               "t_gpu_over_m": round((st["touched"] + st["assist_reads"]) / csr.m, 5),
               "atomics": st["reserve_attempts"] + st["match_attempts"],
               "conflicts": st["reserve_conflicts"] + st["match_conflicts"],
               "word_retries": st["word_retries"], "pairs": st["pairs"],
               "launches": 1 + args.steps}
        rows.append(row)
        log("variant %-18s sweep %.4f ms  %.1f GEdges/s  T/m %.4f  atomics %d  conflicts %d  viol %d" % (
            name, row["sweep_ms"], row["gedges_per_s"], row["t_gpu_over_m"], row["atomics"],
            row["conflicts"], row["violations"]))
    return rows


def bench_serve(args, dev):
    """Serving: Poisson streams of requests over a pool of resident graphs
    whose entry counts are log-uniform in [1e4, 5e7] (ER, grid and R-MAT
    kinds); small jobs are batched continuously, large ones run alone."""
    import torch
    import graphgen
    from paper_2507_04420_amd import serve

    t0 = time.perf_counter()
    pool = graphgen.serve_pool(args.serve_pool, seed=args.seed)
    graphs = []
    for g in range(pool.num_graphs):
        sub = pool.member(g)
        off = torch.from_numpy(sub.off).to(dev)
        nbr = torch.from_numpy(sub.nbr).to(dev)
        # large jobs run with their class's serving tuning (serve.solo_tuning)
        graphs.append(serve.ResidentGraph.for_serving(off, nbr, sub.off, True, sub.name))
    torch.cuda.synchronize()
    log("serving pool: %d graphs, M=%d, generated and resident in %.1fs" % (
        pool.num_graphs, pool.m, time.perf_counter() - t0))
    free, _ = torch.cuda.mem_get_info()
    rng = np.random.default_rng(args.seed + 101)
    out = {"pool_graphs": pool.num_graphs, "pool_entries": int(pool.m), "small_edges": 2_000_000,
           "hbm_budget_bytes": int(free // 2), "rates": []}

    # the executor and tunings the serving tests check (serve.batch_tuning,
    # serve.solo_tuning)
    def scheduler():
        ex = serve.GpuExecutor.for_serving(batch_slots=2, solo_slots=2)
        return serve.Scheduler(ex, hbm_budget=free // 2, small_edges=2_000_000, max_batch=1024,
                               batch_slots=2, solo_slots=2, keep_results=False)

    # warm-up: every graph once, so the kernels are loaded and the allocator is primed
    serve.run_trace(scheduler(), [serve.Request(i, g, 0.0) for i, g in enumerate(graphs)])
    for rate in args.serve_rates:
        count = max(20, int(rate * args.serve_seconds))
        gid = rng.integers(0, len(graphs), size=count)
        arr = serve.poisson_arrivals(count, rate, seed=args.seed + int(rate))
        reqs = [serve.Request(i, graphs[g], float(arr[i])) for i, g in enumerate(gid)]
        s = scheduler()
        comps, wall = serve.run_trace(s, reqs, timeout=120)
        edges = int(sum(graphs[g].m for g in gid))
        r = serve.summarize(comps, wall, edges)
        r["rate_req_per_s"] = rate
        r["peak_in_use_bytes"] = int(s.peak_in_use)
        out["rates"].append({k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()})
        log("serve %5d req/s: p50 %.3f ms p99 %.3f ms, %.1f GEdges/s, %d batches (%.1f jobs each), %d solo" % (
            rate, r["p50_ms"], r["p99_ms"], r["gedges_per_s"], r["batch_launches"],
            r["mean_jobs_per_batch"], r["solo_launches"]))
    return out


def bench_batch(args, tun, dev):
    """Batched matching of the 4096-graph mixture: one hipGraph-captured
    persistent launch per pass, against one mm_run per graph on one stream
    (same kernels, the same tuning without the hint, caches warm)."""
    import torch
    import graphgen
    import paper_2507_04420_amd as mm

    t0 = time.perf_counter()
    mix = graphgen.mixture(args.batch_graphs, seed=args.seed)
    G = mix.num_graphs
    log("generated batch mixture: %d graphs, N=%d M=%d in %.1fs" % (G, mix.n, mix.m,
                                                                    time.perf_counter() - t0))
    off = torch.from_numpy(mix.off).to(dev)
    nbr = torch.from_numpy(mix.nbr).to(dev)
    b = mm.Batch(off, nbr, mix.vtx_off, symmetric=True, validate=True, capture=True, tuning=tun)
    out = torch.empty(mix.n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        b.run(out)
    b.sync()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(3, args.steps // 2)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(reps):
        b.run(out)
    ev1.record(stream)
    torch.cuda.synchronize()
    b.sync()
    ms_batched = ev0.elapsed_time(ev1) / reps

    # per-graph launches: one handle per member graph, outputs are views of one
    # tensor. Each launch spreads its graph over as many wavefronts as blocks of
    # 64 sources give (no whole-graph items; min_waves = 2048 shortens every
    # block of a small graph to 64) and runs no hint (its fill would be one more
    # launch per graph): its fastest form alone.
    tun_pg = mm.Tuning(**dict(tun.as_dict(), whole_graph_vertices=0, hint=0, min_waves=2048))
    vtx = mix.vtx_off
    offs, handles = [], []
    out2 = torch.empty(mix.n, dtype=torch.int32, device=dev)
    views = []
    for g in range(G):
        v0, v1 = int(vtx[g]), int(vtx[g + 1])
        e0, e1 = int(mix.off[v0]), int(mix.off[v1])
        og = (off[v0:v1 + 1] - e0).contiguous()
        offs.append(og)
        handles.append(mm.Graph(og, nbr[e0:e1], symmetric=True, tuning=tun_pg))
        views.append(out2[v0:v1])
    for h, o in zip(handles, views):
        h.run(o)
    torch.cuda.synchronize()
    rounds = 3
    ev0.record(stream)
    for _ in range(rounds):
        for h, o in zip(handles, views):
            h.run(o)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_per_graph_total = ev0.elapsed_time(ev1) / rounds

    # untimed: the library's device check of both outputs (every member graph)
    def violations(r):
        return sum(r[k] for k in ("out_of_range", "self_mate", "asymmetric", "not_edge", "uncovered"))
    bad_b = violations(b.check(out))
    bad_p = violations(b.check(out2))
    items = b.items
    for h in handles:
        h.close()
    b.close()
    res = {
        "graphs": G,
        "N": int(mix.n),
        "M": int(mix.m),
        "work_items": int(items),
        "ms_batched": round(ms_batched, 4),
        "graphs_per_s_batched": round(G / (ms_batched / 1e3), 1),
        "ms_per_graph_launches": round(ms_per_graph_total, 4),
        "tuning_per_graph": tun_pg.as_dict(),
        "graphs_per_s_per_graph": round(G / (ms_per_graph_total / 1e3), 1),
        "ratio": round(ms_per_graph_total / ms_batched, 3),
        "gedges_per_s_batched": round(mix.m / (ms_batched / 1e3) / 1e9, 2),
        "checker_violations_batched": int(bad_b),
        "checker_violations_per_graph": int(bad_p),
    }
    log("batch: %.3f ms batched vs %.3f ms per-graph launches (x%.2f), violations %d/%d" % (
        ms_batched, ms_per_graph_total, res["ratio"], bad_b, bad_p))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat27")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--layout", default=None, choices=["u8", "u32", "u2"])
    ap.add_argument("--lazy", type=int, default=None)
    ap.add_argument("--wave-vertices", type=int, default=None)
    ap.add_argument("--wg-size", type=int, default=None)
    ap.add_argument("--disperse", type=int, default=None)
    ap.add_argument("--assist-after", type=int, default=None)
    ap.add_argument("--no-stats", action="store_true")
    ap.add_argument("--batch-graphs", type=int, default=4096)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[200.0, 500.0, 1000.0, 2000.0])
    ap.add_argument("--serve-seconds", type=float, default=1.5)
    ap.add_argument("--serve-pool", type=int, default=96)
    ap.add_argument("--variants", default=None,
                    help="comma-separated design-choice variants (%s): time and count each on the "
                         "workload and print one JSON line of rows instead of the benchmark line"
                         % ",".join(VARIANTS))
    ap.add_argument("--untuned", action="store_true",
                    help="library default tunings instead of the autotuned table")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (read + write of known size), so that "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE can be scaled")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the matching pass of one graph runs on a single "
              "MI355X (no multi-GPU path is built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2507_04420_amd as mm
    from paper_2507_04420_amd import _lib

    t0 = time.perf_counter()
    csr, config = make_workload(args.workload, args.seed)
    log("generated %s: n=%d m=%d in %.1fs" % (args.workload, csr.n, csr.m, time.perf_counter() - t0))

    # CPU baseline: the oracle's SGMM, single thread; also yields T_seq.
    ref, t_sgmm, reps = cpu_baseline(csr)
    t_seq = ref.touched
    log("SGMM (oracle, 1 thread): %.3fs x%d, pairs=%d, T_seq=%d (%.4f m)" % (
        t_sgmm, reps, ref.pairs, t_seq, t_seq / max(csr.m, 1)))

    dev = torch.device("cuda:0")
    off = torch.from_numpy(csr.off).to(dev)
    nbr = torch.from_numpy(csr.nbr).to(dev)
    torch.cuda.synchronize()

    from paper_2507_04420_amd import autotune
    tun = mm.Tuning.default() if args.untuned else autotune.tuned(config["workload"])
    if args.layout is not None:
        tun.layout = {"u8": _lib.MM_LAYOUT_U8, "u32": _lib.MM_LAYOUT_U32, "u2": _lib.MM_LAYOUT_U2}[args.layout]
    if args.lazy is not None:
        tun.lazy_init = args.lazy
    if args.wave_vertices:
        tun.wave_vertices = args.wave_vertices
    if args.wg_size:
        tun.wg_size = args.wg_size
    if args.disperse is not None:
        tun.disperse = args.disperse
    if args.assist_after is not None:
        tun.assist_after = args.assist_after

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.int32, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.add(src, 0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 x (1 GiB read + 1 GiB write) with torch.add(src, 0, out=dst)")

    if args.variants:
        rows = bench_variants(args, csr, off, nbr, tun, t_seq)
        print(json.dumps({"mode": "variants", "config": config, "n": csr.n, "m": csr.m,
                          "t_seq": t_seq, "size_sgmm": ref.pairs, "steps": args.steps,
                          "rows": rows}), flush=True)
        return

    g = mm.Graph(off, nbr, symmetric=True, validate=True, timing=True, tuning=tun)
    out = torch.empty(csr.n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        g.run(out)
    g.sync()
    g.timing()  # drop warm-up launches

    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        g.run(out)
    ev1.record(stream)
    torch.cuda.synchronize()
    g.sync()
    total_ms = ev0.elapsed_time(ev1)
    ms_per_step = total_ms / args.steps
    sweep = g.timing()
    log("timed %d steps: %.4f ms/step; sweep kernel mean %.4f ms (min %.4f, max %.4f, n=%d)" % (
        args.steps, ms_per_step, sweep["mean_ms"], sweep["min_ms"], sweep["max_ms"], sweep["count"]))

    # Untimed: the library's device check of the last output (the exact
    # checker of Section II-B, counted on the GPU; the test suite pins it
    # against the oracle's).
    chk = g.check(out)
    chk_viol = sum(chk[k] for k in ("out_of_range", "self_mate", "asymmetric", "not_edge", "uncovered"))
    chk_size = chk["matched"] // 2
    log("check: violations=%d size=%d (SGMM %d)" % (chk_viol, chk_size, ref.pairs))

    counters = conflicts = None
    if not args.no_stats:
        gs = mm.Graph(off, nbr, symmetric=True, stats=True, tuning=tun)
        o2 = gs.run()
        gs.sync()
        counters = gs.stats()
        c2 = gs.check(o2)
        counters["checker_violations"] = sum(
            c2[k] for k in ("out_of_range", "self_mate", "asymmetric", "not_edge", "uncovered"))
        gs.close()
        log("counters: %s" % counters)
        # Table II on this graph: worst (most conflicting edges) of five passes
        conflicts = mm.conflict_table(off, nbr, runs=5, tuning=tun)
        log("conflicts (Table II): %s" % conflicts)

    del g
    batch = None
    if not args.no_batch:
        tb = mm.Tuning.default() if args.untuned else autotune.tuned("batch")
        batch = bench_batch(args, tb, dev)
        batch["tuning"] = tb.as_dict()
    serving = None if args.no_serve else bench_serve(args, dev)

    n, m = csr.n, csr.m
    w = csr.off.dtype.itemsize
    # Algorithmic bytes of one sweep launch: per source its offset w, its
    # state byte and its mate (4 B); per id a sequential pass must read (T_seq)
    # the id (4 B) and that neighbour's state byte. The pass adds the state
    # initialisation n.
    b_sweep = w * (n + 1) + 5 * t_seq + n + 4 * n
    b_pass = b_sweep + n
    csr_bytes = w * (n + 1) + 4 * m
    sweep_s = sweep["mean_ms"] / 1e3
    achieved = b_sweep / sweep_s / 1e9 if sweep_s > 0 else 0.0
    value = m / (ms_per_step / 1e3) / 1e9
    cfg_out = dict(config, n=n, m=m, tuning={k: int(v) for k, v in vars(tun).items()})
    traffic = measured_traffic(cfg_out)
    result = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GEdges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": cfg_out,
        "roofline": {
            "bound": "hbm",
            "kernel": "sweep_kernel",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": traffic,
            # measured HBM bytes per launch over the same duration: how close the
            # kernel's real traffic comes to the peak
            "traffic_frac": (round(traffic / sweep_s / 1e9 / HBM_PEAK_GBS, 5)
                             if traffic and sweep_s > 0 else None),
            "alg_bytes_per_launch": int(b_sweep),
            "sweep_ms": round(sweep["mean_ms"], 5),
            "pass_alg_bytes": int(b_pass),
            "pass_frac": round(b_pass / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 5),
            # the edge rate a pass that streams the whole CSR once (offsets and
            # ids, w(n+1) + 4m bytes) would reach at the peak, and the value as
            # a fraction of it: the roofline of a method without early exit
            "csr_stream_gedges_per_s": round(m / (csr_bytes / (HBM_PEAK_GBS * 1e9)) / 1e9, 1),
            "csr_stream_frac": round(value / (m / (csr_bytes / (HBM_PEAK_GBS * 1e9)) / 1e9), 5),
        },
        "cpu_baseline": {
            "value": round(m / t_sgmm / 1e9, 4),
            "unit": "GEdges/s",
            "cores": 1,
            "kind": "oracle",
            "sample": "full graph, SGMM single thread, median of %d run(s), %.3f s each" % (reps, t_sgmm),
            "host": host_cpu(),
        },
        "checker": {"kind": "device check (mm_check)", "violations": int(chk_viol),
                    "size": int(chk_size), "size_sgmm": ref.pairs, "t_seq": t_seq},
        "counters": counters,
        "conflicts": conflicts,
        "batch": batch,
        "serve": serving,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
