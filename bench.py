"""Benchmark: single-pass maximal matching (Skipper) on one MI355X.

One step = one full matching pass (state initialisation + sweep) over a graph
resident in HBM. The headline workload is R-MAT scale 27, edge factor 16,
(a, b, c) = (0.57, 0.19, 0.19), symmetrised, deduplicated, ids permuted.

value  = m / (ms_per_step) in GEdges/s, m = directed CSR entries.
roofline: the sweep kernel's algorithmic bytes per launch (per source its
          offset w, its state byte and its mate 4 B; per id a sequential pass
          must read, T_seq = ids SGMM reads, the id 4 B and its state byte)
          over its mean duration from HIP events recorded on the launch
          stream, against 8 TB/s; beside it the same bytes with the state
          bytes counted once per vertex (frac_d1), and the two ceilings that
          bind a pass of random accesses (random line reads, random atomics),
          each measured live on the box with plain torch operations.
cpu_baseline: the oracle's single-thread SGMM, pinned to one host core, on
          the same graph (it also gives T_seq).
legs: every single-graph configuration (ER n=65536 with int32 offsets,
      R-MAT-24, R-MAT-27, the 16384^2 grid) with create time, the sweep of the
      graph as given beside one on a create-time copy (relabelled or with
      reordered lists), B_alg, frac, T_gpu/m and its SGMM baseline, and for
      ER and R-MAT-24 the multi-pass mutual-selection baseline (time, passes,
      ids read); batch: the 4096-graph mixture in one captured persistent
      launch against one launch per graph, with its algorithmic bytes from
      every member's T_seq; serve: Poisson request streams over resident
      graphs (p50/p99 arrival-to-result latency, GEdges/s).
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
                  for f in ("protocol.h", "sweep.h", "pieces.h", "internal.h", "mm.hip", "relabel.hip",
                            "hubs.hip", "order.hip")]
VIOLATION_KEYS = ("out_of_range", "self_mate", "asymmetric", "not_edge", "uncovered")
LEGS = ("headline", "er65536", "rmat24", "grid16384", "batch", "serve")


def strip_comments(src: str) -> str:
    """C/C++ source without its comments and with runs of whitespace
    collapsed (string and character literals kept as they are), so that a
    change of comments alone leaves the code's hash unchanged."""
    out = []
    i, n = 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return "\n".join(" ".join(line.split()) for line in "".join(out).splitlines() if line.strip())


def kernel_sources_sha256() -> str:
    """SHA-256 of the code (comments stripped) of the sources that decide
    what the sweep kernel does and which graph it reads."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, encoding="utf-8") as fh:
            h.update(strip_comments(fh.read()).encode())
    return h.hexdigest()


def stored_traffic(config):
    """The HBM bytes per sweep launch that the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs measured (scaled by a plain copy of known
    size), with the record they come from, if that record was taken on the
    current kernel sources with this workload and tuning; else (None, None).
    This run does not measure them itself."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None, None
    if t.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None, None
    if t.get("config") != json.loads(json.dumps(config)):
        return None, None
    return float(t["hbm_bytes_per_launch"]), t


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


def workload_class(name: str) -> str:
    """The tuned-table class of a workload name (er65536 -> er, rmat27 -> rmat)."""
    return "er" if name.startswith("er") else name.rstrip("0123456789")


def host_record() -> dict:
    model = "?"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "?")
    except OSError:
        pass
    ram = None
    try:
        with open("/proc/meminfo") as f:
            kb = next(int(l.split()[1]) for l in f if l.startswith("MemTotal"))
            ram = round(kb / 1024 / 1024, 1)
    except (OSError, StopIteration):
        pass
    return {"cpu": model, "logical_cpus": os.cpu_count() or 0, "ram_gib": ram}


def cpu_baseline(csr, budget_s: float = 30.0):
    """Times the oracle's single-thread SGMM (untuned) on the host, pinned to
    one core (the first the process may use; the equivalent of taskset -c)."""
    import oracle
    old = os.sched_getaffinity(0)
    core = min(old)
    os.sched_setaffinity(0, {core})
    times = []
    res = None
    try:
        while True:
            t0 = time.perf_counter()
            res = oracle.sgmm(csr)
            times.append(time.perf_counter() - t0)
            if len(times) >= 3 or sum(times) * (len(times) + 1) / len(times) > budget_s:
                break
    finally:
        os.sched_setaffinity(0, old)
    return res, float(np.median(times)), len(times), core


def sweep_bytes(w: int, n: int, t_seq: int) -> int:
    """Algorithmic bytes of one sweep launch, per unit: per source its offset
    (w), its state byte (1) and its mate (4); per id a sequential pass must
    read (T_seq) the id (4) and that neighbour's state byte (1)."""
    return w * (n + 1) + 5 * t_seq + n + 4 * n


def sweep_bytes_d1(w: int, n: int, t_seq: int) -> int:
    """The same with the states counted once per vertex: w(n+1) + 4 T_seq +
    2n (state init written, then read) + 4n (mates)."""
    return w * (n + 1) + 4 * t_seq + 2 * n + 4 * n


def live_ceilings(dev) -> dict:
    """The ceilings of a pass of random accesses, measured on this GPU: the
    library's probe (mm_probe_ceilings: plain kernels of independent random
    4-byte reads, and of random 4-byte atomic adds, over 1 GiB, 2^26 of each,
    no other memory traffic), and a device-to-device copy of 1 GiB with torch
    (bytes read + written) as a measured counterpart of the nominal 8 TB/s."""
    import ctypes
    import torch
    from paper_2507_04420_amd import _lib
    lib = _lib.load()
    reads, atomics = ctypes.c_double(), ctypes.c_double()
    stream = torch.cuda.current_stream(dev)
    _lib.check(lib.mm_probe_ceilings(1 << 30, 1 << 26, ctypes.c_void_p(stream.cuda_stream),
                                     ctypes.byref(reads), ctypes.byref(atomics)))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    src = torch.ones(1 << 28, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(5):
        dst.copy_(src)
    ev[1].record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * src.numel() * 4 / (ev[0].elapsed_time(ev[1]) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"random_reads_per_s": round(reads.value, -6), "random_atomics_per_s": round(atomics.value, -6),
            "copy_gbs": round(copy_gbs, 1),
            "how": "mm_probe_ceilings: 2^26 independent random 4-byte reads, then 2^26 random "
                   "4-byte atomic adds, over 1 GiB (plain kernels, two timed launches each); "
                   "torch copy_ of 1 GiB (read + write bytes), 5 timed repeats"}


def timed_passes(g, out, steps, warmup):
    """Warm-up passes, then `steps` timed passes on the current stream:
    returns (ms per pass by events around all of them, sweep timing)."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        g.run(out)
    g.sync()
    g.timing()  # drop warm-up launches
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        g.run(out)
    ev1.record(stream)
    torch.cuda.synchronize()
    g.sync()
    return ev0.elapsed_time(ev1) / steps, g.timing()


def bench_single(args, name, tun, dev, *, natural=False, conflicts=False, ceilings=None,
                 ems=False):
    """One single-graph configuration: the oracle baseline (T_seq), the
    handle's create time, `steps` timed passes, the device check, an
    instrumented pass (T_gpu, atomics, conflicts), and, for a tuning that
    builds a copy of the graph (relabelled or with reordered lists), the same
    passes on the graph as given on a second handle."""
    import torch
    import paper_2507_04420_amd as mm

    t0 = time.perf_counter()
    csr, config = make_workload(name, args.seed)
    log("generated %s: n=%d m=%d in %.1fs" % (name, csr.n, csr.m, time.perf_counter() - t0))
    ref, t_sgmm, reps, core = cpu_baseline(csr)
    t_seq = ref.touched
    log("SGMM (oracle, core %d): %.3fs x%d, pairs=%d, T_seq=%d (%.4f m)" % (
        core, t_sgmm, reps, ref.pairs, t_seq, t_seq / max(csr.m, 1)))
    off = torch.from_numpy(csr.off).to(dev)
    nbr = torch.from_numpy(csr.nbr).to(dev)
    torch.cuda.synchronize()
    n, m = csr.n, csr.m
    w = csr.off.dtype.itemsize
    del csr

    tc = time.perf_counter()
    g = mm.Graph(off, nbr, symmetric=True, timing=True, tuning=tun)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - tc) * 1e3
    out = torch.empty(n, dtype=torch.int32, device=dev)
    ms_per_step, sweep = timed_passes(g, out, args.steps, args.warmup)
    chk = g.check(out)
    viol = sum(chk[k] for k in VIOLATION_KEYS)
    size = chk["matched"] // 2
    g.close()
    del g
    log("%s: create %.1f ms; %.4f ms/pass, sweep %.4f ms (min %.4f max %.4f); %.1f GEdges/s; "
        "violations %d, size %d (SGMM %d)" % (
            name, create_ms, ms_per_step, sweep["mean_ms"], sweep["min_ms"], sweep["max_ms"],
            m / ms_per_step / 1e6, viol, size, ref.pairs))

    ems_leg = None
    if ems:
        # the multi-pass baseline the paper compares with (Section II-C), on
        # the same resident graph: time, passes and ids read against the sweep
        ge = mm.Graph(off, nbr, symmetric=True, tuning=tun)
        o_e, st_e = ge.ems(seed=args.seed)
        torch.cuda.synchronize()
        times = []
        for _ in range(3):
            t_e = time.perf_counter()
            o_e, st_e = ge.ems(seed=args.seed, out=o_e)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t_e) * 1e3)
        chk_e = ge.check(o_e)
        ge.close()
        ems_leg = {"ms": round(float(np.median(times)), 3), "iterations": int(st_e["iterations"]),
                   "touched_over_m": round(st_e["touched"] / m, 4), "pairs": int(st_e["pairs"]),
                   "violations": int(sum(chk_e[k] for k in VIOLATION_KEYS)),
                   "sweep_speedup": round(float(np.median(times)) / ms_per_step, 1)}
        log("%s mutual selection: %.3f ms, %d passes, ids read %.3f m, %d pairs (sweep %.4f ms)" % (
            name, ems_leg["ms"], ems_leg["iterations"], ems_leg["touched_over_m"], ems_leg["pairs"],
            ms_per_step))

    counters = conflict_row = None
    if not args.no_stats:
        gs = mm.Graph(off, nbr, symmetric=True, stats=True, tuning=tun)
        o2 = gs.run()
        gs.sync()
        counters = gs.stats()
        c2 = gs.check(o2)
        counters["checker_violations"] = sum(c2[k] for k in VIOLATION_KEYS)
        gs.close()
        del o2
        if conflicts:
            # Table II on this graph: worst (most conflicting edges) of five passes
            conflict_row = mm.conflict_table(off, nbr, runs=5, tuning=tun)
            log("conflicts (Table II): %s" % conflict_row)

    natural_leg = None
    change = {k: v for k, v in COPIES.items() if getattr(tun, k) != v}
    if natural and change:
        # the same passes on the graph as given: no relabelled or reordered copy
        tn = mm.Tuning(**dict(tun.as_dict(), **change))
        tc = time.perf_counter()
        gn = mm.Graph(off, nbr, symmetric=True, timing=True, tuning=tn)
        torch.cuda.synchronize()
        create_n = (time.perf_counter() - tc) * 1e3
        ms_n, sweep_n = timed_passes(gn, out, args.steps, args.warmup)
        chk_n = gn.check(out)
        gn.close()
        natural_leg = {"tuning_change": change, "create_ms": round(create_n, 2),
                       "ms_per_step": round(ms_n, 5), "sweep_ms": round(sweep_n["mean_ms"], 5),
                       "gedges_per_s": round(m / ms_n / 1e6, 2),
                       "frac": round(sweep_bytes(w, n, t_seq) / (sweep_n["mean_ms"] / 1e3) / 1e9
                                     / HBM_PEAK_GBS, 5),
                       "violations": int(sum(chk_n[k] for k in VIOLATION_KEYS)),
                       "size": chk_n["matched"] // 2}
        log("%s without the copy: create %.1f ms; %.4f ms/pass, sweep %.4f ms; %.1f GEdges/s" % (
            name, create_n, ms_n, sweep_n["mean_ms"], m / ms_n / 1e6))
    del off, nbr, out
    torch.cuda.empty_cache()

    sweep_s = sweep["mean_ms"] / 1e3
    b_sweep = sweep_bytes(w, n, t_seq)
    b_d1 = sweep_bytes_d1(w, n, t_seq)
    leg = {
        "config": dict(config, n=n, m=m, tuning=tun.as_dict()),
        "create_ms": round(create_ms, 2),
        "relabel_copy_bytes": (8 * (n + 1) + 4 * n + 4 * m + 4 * n) if tun.relabel else 0,
        "ordered_copy_bytes": 4 * m if tun.order_lists else 0,
        "ms_per_step": round(ms_per_step, 5),
        "us_per_step": round(ms_per_step * 1e3, 2),
        "sweep_ms": round(sweep["mean_ms"], 5),
        "gedges_per_s": round(m / ms_per_step / 1e6, 3),
        "alg_bytes_per_launch": int(b_sweep),
        "frac": round(b_sweep / sweep_s / 1e9 / HBM_PEAK_GBS, 5),
        "alg_bytes_d1": int(b_d1),
        "frac_d1": round(b_d1 / sweep_s / 1e9 / HBM_PEAK_GBS, 5),
        "t_seq": int(t_seq),
        "t_gpu_over_m": (round((counters["touched"] + counters["assist_reads"]) / m, 5)
                         if counters else None),
        "violations": int(viol),
        "size": int(size),
        "size_sgmm": int(ref.pairs),
        "cpu_baseline": {"value": round(m / t_sgmm / 1e9, 4), "unit": "GEdges/s", "cores": 1,
                         "kind": "oracle", "pinned_core": core, "t_sgmm_s": round(t_sgmm, 4),
                         "sample": "full graph, SGMM single thread, median of %d run(s)" % reps,
                         "gain_over_sgmm": round(t_sgmm / (ms_per_step / 1e3), 1)},
    }
    if counters:
        atomics = counters["reserve_attempts"] + counters["match_attempts"]
        leg["atomics_per_launch"] = int(atomics)
        if ceilings:
            leg["atomic_frac"] = round(atomics / sweep_s / ceilings["random_atomics_per_s"], 4)
    if natural_leg:
        leg["without_copy"] = natural_leg
    if ems_leg:
        leg["mutual_selection"] = ems_leg
    return leg, counters, conflict_row, sweep


# Tuning fields that build a copy of the graph at create time, and their
# values without it (the headline also times the graph as given).
COPIES = {"relabel": 0, "order_lists": 0}

# Design-choice variants (--variants): overrides of the tuned tuning, one
# choice at a time, each timed and counted on the same resident graph.
VARIANTS = {
    "tuned": {},
    "natural_order": {"relabel": 0},
    # the relabelled copies replace a reordered one (the two do not combine)
    "relabelled": {"relabel": 1, "order_lists": 0},
    "order_lists": {"order_lists": 1},
    "upper_first": {"order_lists": 2, "upper_only": 1},
    "probe_first": {"probe_first": 1},
    "probe_each": {"probe_first": 2},
    "probe_first_upper_first": {"probe_first": 1, "order_lists": 2, "upper_only": 1},
    "probe_first_given_lists": {"probe_first": 1, "order_lists": 0},
    "probe_none": {"probe_first": 0},
    "occ6": {"occupancy": 6},
    "occ0": {"occupancy": 0},
    "chunk_256": {"hub_chunk": 256},
    "assist_chunk_256": {"assist_after": 256, "hub_chunk": 256},
    "probe_first_w2": {"probe_first": 1, "scan_width": 2},
    "probe_first_w3": {"probe_first": 1, "scan_width": 3},
    "given_lists": {"order_lists": 0},
    "relabel_hot": {"relabel": 2, "order_lists": 0},
    "relabel_hot_512": {"relabel": 2, "hot_degree": 512, "order_lists": 0},
    "relabel_hot_1024": {"relabel": 2, "hot_degree": 1024, "order_lists": 0},
    "relabel_hot_4096": {"relabel": 2, "hot_degree": 4096, "order_lists": 0},
    "relabel_hot_8192": {"relabel": 2, "hot_degree": 8192, "order_lists": 0},
    # (the upper-first copy needs upper_only: the degree-ordered one instead)
    "all_entries": {"upper_only": 0, "order_lists": 1},
    "all_entries_relabelled": {"upper_only": 0, "relabel": 1, "order_lists": 0},
    "u8_byte_cas": {"layout": 0, "protocol": 0, "lazy_init": 0},
    "u8_byte_cas_lazy": {"layout": 0, "protocol": 0, "lazy_init": 1},
    "lazy": {"lazy_init": 1},
    "eager": {"lazy_init": 0},
    "u2_two_phase": {"layout": 2, "protocol": 1, "lazy_init": 0},
    "u32_two_phase": {"layout": 1, "protocol": 1, "lazy_init": 0},
    "hint_bits": {"hint": 1},
    "hint_bytes": {"hint": 2},
    "no_hint": {"hint": 0},
    "assist_16": {"assist_after": 16},
    "assist_32": {"assist_after": 32},
    "assist_256": {"assist_after": 256},
    "assist_64": {"assist_after": 64},
    "wg_128": {"wg_size": 128},
    "no_assist": {"assist_after": 0},
    "contiguous_lanes": {"disperse": 0},
    "dispersed_lanes": {"disperse": 1},
    "wait_release": {"wait_release": 1},
    "upper_only": {"upper_only": 1},
    "upper_only_hint_bytes": {"upper_only": 1, "hint": 2},
    "upper_only_u8": {"upper_only": 1, "layout": 0, "protocol": 0, "lazy_init": 0},
    "upper_only_natural": {"upper_only": 1, "relabel": 0, "order_lists": 0},
    "upper_wait": {"upper_only": 1, "wait_release": 1},
    "hub_wave": {"hub_wave": 1},
    "hub_wave_1024": {"hub_wave": 1, "hub_chunk": 1024},
    "hub_group": {"hub_wave": 2},
    "hub_group_1024": {"hub_wave": 2, "hub_chunk": 1024},
    "hub_group_wg256": {"hub_wave": 2, "wg_size": 256},
    "hub_lane_64": {"hub_chunk": 64, "hub_wave": 0},
    "hub_lane": {"hub_wave": 0},
    "no_hub_tier": {"hub_degree": 0},
    "stream_loads": {"stream_loads": 1},
    "scan_2": {"scan_width": 2},
    "scan_3": {"scan_width": 3},
    "hub_2048": {"hub_degree": 2048},
    "hub_16384": {"hub_degree": 16384},
    "wg_256": {"wg_size": 256},
    "wv_64": {"wave_vertices": 64},
    "wv_256": {"wave_vertices": 256},
    "wv_1024": {"wave_vertices": 1024},
    "wg_64": {"wg_size": 64},
    "mw_2048": {"min_waves": 2048},
    "mw_32": {"min_waves": 32},
    "scan_1": {"scan_width": 1},
    "wv_4096": {"wave_vertices": 4096},
    "u32": {"layout": 1, "protocol": 0, "lazy_init": 0},
    "u8": {"layout": 0, "protocol": 0, "lazy_init": 0},
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
        b_sweep = sweep_bytes(w, csr.n, t_seq)
        row = {"variant": name, "tuning": t.as_dict(), "sweep_ms": round(tm["mean_ms"], 4),
               "gedges_per_s": round(csr.m / sweep_s / 1e9, 1),
               "alg_gbs": round(b_sweep / sweep_s / 1e9, 1),
               "violations": sum(chk[k] for k in VIOLATION_KEYS),
               "size": chk["matched"] // 2,
               "t_gpu_over_m": round((st["touched"] + st["assist_reads"]) / csr.m, 5),
               "atomics": st["reserve_attempts"] + st["match_attempts"],
               "conflicts": (st["reserve_conflicts"] + st["match_conflicts"] + st["reserve_matched"]
                             + st["match_matched"]),
               "word_retries": st["word_retries"], "pairs": st["pairs"],
               "launches": 1 + args.steps}
        rows.append(row)
        log("variant %-18s sweep %.4f ms  %.1f GEdges/s  T/m %.4f  atomics %d  conflicts %d  viol %d" % (
            name, row["sweep_ms"], row["gedges_per_s"], row["t_gpu_over_m"], row["atomics"],
            row["conflicts"], row["violations"]))
    return rows


def bench_ab(args, csr, off, nbr, base):
    """Interleaved A/B of two variants: one handle each, created once and
    kept; rounds alternate A then B (then B then A) so that neither gains
    from its position; every round times `steps` passes of each by the
    handles' sweep events. Reports per variant the median and spread of the
    round means, and the median of the paired differences B - A."""
    import paper_2507_04420_amd as mm
    names = args.ab.split(",")
    if len(names) != 2:
        raise SystemExit("--ab takes two variant names")
    tun = [mm.Tuning(**dict(base.as_dict(), **VARIANTS[nm])) for nm in names]
    hs = [mm.Graph(off, nbr, symmetric=True, timing=True, tuning=t) for t in tun]
    outs = [h.run() for h in hs]
    for h in hs:
        h.sync()
        h.timing()
    means = [[], []]
    for r in range(args.ab_rounds):
        order = (0, 1) if r % 2 == 0 else (1, 0)
        for k in order:
            for _ in range(args.steps):
                hs[k].run(outs[k])
            hs[k].sync()
            means[k].append(hs[k].timing()["mean_ms"])
    viol = [sum(h.check(o)[k] for k in VIOLATION_KEYS) for h, o in zip(hs, outs)]
    for h in hs:
        h.close()
    diff = [b - a for a, b in zip(means[0], means[1])]
    rows = []
    for k in range(2):
        v = np.array(means[k])
        rows.append({"variant": names[k], "tuning": tun[k].as_dict(),
                     "median_ms": round(float(np.median(v)), 4), "min_ms": round(float(v.min()), 4),
                     "max_ms": round(float(v.max()), 4), "sd_ms": round(float(v.std()), 4),
                     "gedges_per_s": round(csr.m / float(np.median(v)) / 1e6, 1),
                     "violations": int(viol[k]), "round_means_ms": [round(x, 4) for x in v]})
        log("ab %-20s median %.4f ms (min %.4f max %.4f sd %.4f) over %d rounds" % (
            names[k], rows[-1]["median_ms"], rows[-1]["min_ms"], rows[-1]["max_ms"],
            rows[-1]["sd_ms"], args.ab_rounds))
    d = np.array(diff)
    res = {"rows": rows, "median_diff_ms": round(float(np.median(d)), 4),
           "diff_min_ms": round(float(d.min()), 4), "diff_max_ms": round(float(d.max()), 4),
           "b_faster_rounds": int((d < 0).sum()), "rounds": args.ab_rounds, "steps": args.steps}
    log("ab %s - %s: median %.4f ms, range %.4f .. %.4f, %s faster in %d of %d rounds" % (
        names[1], names[0], res["median_diff_ms"], res["diff_min_ms"], res["diff_max_ms"], names[1],
        res["b_faster_rounds"], args.ab_rounds))
    return res


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
        count = max(args.serve_requests, int(rate * args.serve_seconds))
        gid = rng.integers(0, len(graphs), size=count)
        arr = serve.poisson_arrivals(count, rate, seed=args.seed + int(rate))
        reqs = [serve.Request(i, graphs[g], float(arr[i])) for i, g in enumerate(gid)]
        s = scheduler()
        comps, wall = serve.run_trace(s, reqs, timeout=120)
        edges = int(sum(graphs[g].m for g in gid))
        r = serve.summarize(comps, wall, edges)
        r["rate_req_per_s"] = rate
        r["peak_in_use_bytes"] = int(s.peak_in_use)
        r["memory_waits"] = int(s.memory_waits)
        out["rates"].append({k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()})
        log("serve %5d req/s: %d requests, p50 %.3f ms p99 %.3f ms, %.1f GEdges/s, %d batches "
            "(%.2f jobs each), %d solo" % (
                rate, count, r["p50_ms"], r["p99_ms"], r["gedges_per_s"], r["batch_launches"],
                r["mean_jobs_per_batch"], r["solo_launches"]))

    # admission by HBM footprint under a budget that binds: 1.25 times the
    # largest request's footprint (two of the largest jobs never run at
    # once), at the highest rate up to 2000 req/s
    probe = scheduler()
    fps = [probe.executor.footprint(serve.Request(0, g, 0.0), probe.route(serve.Request(0, g, 0.0)))
           for g in graphs]
    budget = int(1.25 * max(fps))
    rate = max([r for r in args.serve_rates if r <= 2000.0] or [min(args.serve_rates)])
    count = max(args.serve_requests, int(rate * args.serve_seconds))
    gid = rng.integers(0, len(graphs), size=count)
    arr = serve.poisson_arrivals(count, rate, seed=args.seed + 7 * int(rate))
    reqs = [serve.Request(i, graphs[g], float(arr[i])) for i, g in enumerate(gid)]
    ex = serve.GpuExecutor.for_serving(batch_slots=2, solo_slots=2)
    s = serve.Scheduler(ex, hbm_budget=budget, small_edges=2_000_000, max_batch=1024, batch_slots=2,
                        solo_slots=2, keep_results=False)
    comps, wall = serve.run_trace(s, reqs, timeout=120)
    r = serve.summarize(comps, wall, int(sum(graphs[g].m for g in gid)))
    r.update(rate_req_per_s=rate, hbm_budget_bytes=int(budget), peak_in_use_bytes=int(s.peak_in_use),
             largest_footprint_bytes=int(max(fps)), memory_waits=int(s.memory_waits))
    out["budget_bound"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
    log("serve %5d req/s under a %.1f MB budget: p50 %.3f ms p99 %.3f ms, peak in use %.1f MB, "
        "%d requests waited for memory" % (rate, budget / 1e6, r["p50_ms"], r["p99_ms"],
                                           s.peak_in_use / 1e6, s.memory_waits))
    return out


def bench_batch(args, tun, dev):
    """Batched matching of the 4096-graph mixture: one hipGraph-captured
    persistent launch per pass, against one mm_run per graph on one stream
    (same kernels, the same tuning without the hint, caches warm). The
    oracle's SGMM over every member (one core) is the CPU baseline and gives
    the members' T_seq for the algorithmic bytes."""
    import torch
    import graphgen
    import oracle
    import paper_2507_04420_amd as mm

    t0 = time.perf_counter()
    mix = graphgen.mixture(args.batch_graphs, seed=args.seed)
    G = mix.num_graphs
    log("generated batch mixture: %d graphs, N=%d M=%d in %.1fs" % (G, mix.n, mix.m,
                                                                    time.perf_counter() - t0))
    # CPU baseline over every member (pinned to one core), and T_seq
    old = os.sched_getaffinity(0)
    core = min(old)
    os.sched_setaffinity(0, {core})
    t_seq = 0
    pairs_sgmm = 0
    t_cpu = 0.0
    try:
        for g in range(G):
            sub = mix.member(g)
            tc = time.perf_counter()
            r = oracle.sgmm(sub)
            t_cpu += time.perf_counter() - tc
            t_seq += r.touched
            pairs_sgmm += r.pairs
    finally:
        os.sched_setaffinity(0, old)
    log("batch SGMM (oracle, core %d): %.3f s over %d graphs, T_seq=%d" % (core, t_cpu, G, t_seq))

    off = torch.from_numpy(mix.off).to(dev)
    nbr = torch.from_numpy(mix.nbr).to(dev)
    tc = time.perf_counter()
    b = mm.Batch(off, nbr, mix.vtx_off, symmetric=True, validate=True, capture=True, tuning=tun)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - tc) * 1e3
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
    # block of a small graph to 64), runs no hint (its fill would be one more
    # launch per graph) and examines both entries of an edge (one side only
    # doubles the time of the small meshes spread this way: 1561 against
    # 709 ms for the 4096 members): its fastest form alone.
    tun_pg = mm.Tuning(**dict(tun.as_dict(), whole_graph_vertices=0, hint=0, min_waves=2048,
                              upper_only=0))
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
        return sum(r[k] for k in VIOLATION_KEYS)
    cb = b.check(out)
    bad_b = violations(cb)
    bad_p = violations(b.check(out2))
    items = b.items
    for h in handles:
        h.close()
    b.close()
    # algorithmic bytes of a pass over all members, as for one graph summed
    # over them (each member's offsets have one entry more than its vertices)
    b_alg = sweep_bytes(8, mix.n, t_seq) + 8 * (G - 1)
    res = {
        "graphs": G,
        "N": int(mix.n),
        "M": int(mix.m),
        "work_items": int(items),
        "create_ms": round(create_ms, 2),
        "ms_batched": round(ms_batched, 4),
        "graphs_per_s_batched": round(G / (ms_batched / 1e3), 1),
        "ms_per_graph_launches": round(ms_per_graph_total, 4),
        "tuning_per_graph": tun_pg.as_dict(),
        "graphs_per_s_per_graph": round(G / (ms_per_graph_total / 1e3), 1),
        "ratio": round(ms_per_graph_total / ms_batched, 3),
        "gedges_per_s_batched": round(mix.m / (ms_batched / 1e3) / 1e9, 2),
        "t_seq": int(t_seq),
        "alg_bytes_per_pass": int(b_alg),
        # over the whole captured pass (fills, LDS kernel, persistent sweep);
        # the sweep kernel's own duration is in the profiles
        "frac_of_pass": round(b_alg / (ms_batched / 1e3) / 1e9 / HBM_PEAK_GBS, 5),
        "size": int(cb["matched"] // 2),
        "size_sgmm": int(pairs_sgmm),
        "checker_violations_batched": int(bad_b),
        "checker_violations_per_graph": int(bad_p),
        "cpu_baseline": {"value": round(G / t_cpu, 1), "unit": "graphs/s", "cores": 1,
                         "kind": "oracle", "pinned_core": core, "t_sgmm_s": round(t_cpu, 3),
                         "sample": "SGMM over all %d members, one after the other" % G},
    }
    log("batch: %.3f ms batched vs %.3f ms per-graph launches (x%.2f), violations %d/%d, "
        "alg %.2f GB per pass" % (ms_batched, ms_per_graph_total, res["ratio"], bad_b, bad_p,
                                  b_alg / 1e9))
    del off, nbr, out, out2, offs, views
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat27", help="the headline workload")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated subset of %s (default: all; without the headline "
                         "the line holds only the legs asked for)" % ",".join(LEGS))
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
    ap.add_argument("--serve-rates", type=float, nargs="+",
                    default=[200.0, 500.0, 1000.0, 2000.0, 20000.0])
    ap.add_argument("--serve-seconds", type=float, default=1.5)
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests per rate at least (the default 10000 puts 100 samples above the p99)")
    ap.add_argument("--serve-pool", type=int, default=256)
    ap.add_argument("--variants", default=None,
                    help="comma-separated design-choice variants (%s): time and count each on the "
                         "workload and print one JSON line of rows instead of the benchmark line"
                         % ",".join(VARIANTS))
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the live random-read and random-atomic probes (profiling runs)")
    ap.add_argument("--ab", default=None,
                    help="two variants (names as for --variants): interleaved A/B rounds on one "
                         "handle each; prints one JSON line of the comparison")
    ap.add_argument("--ab-rounds", type=int, default=20)
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
    legs = set(args.legs.split(","))
    unknown = legs - set(LEGS)
    if unknown:
        raise SystemExit("unknown legs %s" % sorted(unknown))
    if args.no_batch:
        legs.discard("batch")
    if args.no_serve:
        legs.discard("serve")

    import torch
    import paper_2507_04420_amd as mm
    from paper_2507_04420_amd import _lib, autotune

    dev = torch.device("cuda:0")

    def tuning_for(graph_class):
        t = mm.Tuning.default() if args.untuned else autotune.tuned(graph_class)
        if args.layout is not None:
            t.layout = {"u8": _lib.MM_LAYOUT_U8, "u32": _lib.MM_LAYOUT_U32, "u2": _lib.MM_LAYOUT_U2}[args.layout]
        if args.lazy is not None:
            t.lazy_init = args.lazy
        if args.wave_vertices:
            t.wave_vertices = args.wave_vertices
        if args.wg_size:
            t.wg_size = args.wg_size
        if args.disperse is not None:
            t.disperse = args.disperse
        if args.assist_after is not None:
            t.assist_after = args.assist_after
        return t

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.int32, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.add(src, 0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 x (1 GiB read + 1 GiB write) with torch.add(src, 0, out=dst)")

    if args.ab:
        csr, config = make_workload(args.workload, args.seed)
        off = torch.from_numpy(csr.off).to(dev)
        nbr = torch.from_numpy(csr.nbr).to(dev)
        res = bench_ab(args, csr, off, nbr, tuning_for(workload_class(args.workload)))
        print(json.dumps(dict({"mode": "ab", "config": config, "n": csr.n, "m": csr.m}, **res)),
              flush=True)
        return

    if args.variants:
        csr, config = make_workload(args.workload, args.seed)
        ref, t_sgmm, reps, core = cpu_baseline(csr)
        off = torch.from_numpy(csr.off).to(dev)
        nbr = torch.from_numpy(csr.nbr).to(dev)
        rows = bench_variants(args, csr, off, nbr, tuning_for(workload_class(args.workload)),
                              ref.touched)
        print(json.dumps({"mode": "variants", "config": config, "n": csr.n, "m": csr.m,
                          "t_seq": ref.touched, "size_sgmm": ref.pairs, "steps": args.steps,
                          "rows": rows}), flush=True)
        return

    ceilings = None if args.no_ceilings else live_ceilings(dev)
    if ceilings:
        log("live ceilings: %.3g random reads/s, %.3g random atomics/s" % (
            ceilings["random_reads_per_s"], ceilings["random_atomics_per_s"]))

    if "headline" not in legs:
        # a subset of the legs (profiling runs): one JSON line of those
        out = {"mode": "legs", "ceilings": ceilings}
        for name in ("er65536", "rmat24", "grid16384"):
            if name in legs:
                out[name] = bench_single(args, name, tuning_for(workload_class(name)), dev,
                                         natural=True, ceilings=ceilings,
                                         ems=name in ("er65536", "rmat24"))[0]
        if "batch" in legs:
            tb = mm.Tuning.default() if args.untuned else autotune.tuned("batch")
            out["batch"] = dict(bench_batch(args, tb, dev), tuning=tb.as_dict())
        if "serve" in legs:
            out["serve"] = bench_serve(args, dev)
        print(json.dumps(out), flush=True)
        return

    # the headline graph first, while the device is empty
    head, counters, conflicts, sweep = bench_single(
        args, args.workload, tuning_for(workload_class(args.workload)), dev, natural=True,
        conflicts=not args.no_stats, ceilings=ceilings)
    others = {}
    for name in ("er65536", "rmat24", "grid16384"):
        if name in legs and name != args.workload:
            others[name] = bench_single(args, name, tuning_for(workload_class(name)), dev,
                                        natural=True, ceilings=ceilings,
                                        ems=name in ("er65536", "rmat24"))[0]
    batch = None
    if "batch" in legs:
        tb = mm.Tuning.default() if args.untuned else autotune.tuned("batch")
        batch = bench_batch(args, tb, dev)
        batch["tuning"] = tb.as_dict()
    serving = bench_serve(args, dev) if "serve" in legs else None

    cfg = head["config"]
    m = cfg["m"]
    sweep_s = sweep["mean_ms"] / 1e3
    ms_per_step = head["ms_per_step"]
    value = m / (ms_per_step / 1e3) / 1e9
    b_sweep = head["alg_bytes_per_launch"]
    achieved = b_sweep / sweep_s / 1e9
    cfg_traffic = dict(cfg, tuning={k: int(v) for k, v in cfg["tuning"].items()})
    traffic, traffic_rec = stored_traffic(cfg_traffic)
    secondary = dict(ceilings or {})
    if counters:
        secondary["atomics_per_launch"] = head.get("atomics_per_launch")
        secondary["atomic_frac"] = head.get("atomic_frac")
    if traffic_rec and traffic_rec.get("l2_miss_read_requests_per_launch"):
        req = float(traffic_rec["l2_miss_read_requests_per_launch"])
        secondary["l2_miss_read_requests_per_launch_stored"] = req
        if ceilings:
            secondary["request_frac"] = round(req / sweep_s / ceilings["random_reads_per_s"], 4)
    # the same roof with other byte counts (states once per vertex, as in
    # frac_d1): every entry's id read once (B_full, 4m for 4 T_seq), the ids
    # this pass read (T_gpu for T_seq); the measured copy bandwidth instead
    # of the nominal peak; the stored traffic over B_sweep
    n_, w_ = cfg["n"], (8 if cfg.get("offsets") == "int64" else 4)
    b_full = sweep_bytes_d1(w_, n_, m)
    secondary["alg_bytes_full_d1"] = int(b_full)
    secondary["frac_full_d1"] = round(b_full / sweep_s / 1e9 / HBM_PEAK_GBS, 5)
    if counters:
        t_gpu = counters["touched"] + counters["assist_reads"]
        secondary["alg_bytes_t_gpu_d1"] = int(sweep_bytes_d1(w_, n_, t_gpu))
        secondary["frac_t_gpu_d1"] = round(secondary["alg_bytes_t_gpu_d1"] / sweep_s / 1e9
                                           / HBM_PEAK_GBS, 5)
    if ceilings and ceilings.get("copy_gbs"):
        secondary["frac_of_copy_bw"] = round(achieved / ceilings["copy_gbs"], 5)
    if traffic:
        secondary["traffic_over_alg_bytes"] = round(traffic / b_sweep, 3)
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
        "config": cfg,
        "roofline": {
            "bound": "hbm",
            # the six-wave build with occupancy = 6 (the same code)
            "kernel": "sweep_kernel_w6" if cfg["tuning"].get("occupancy") == 6 else "sweep_kernel",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            # HBM bytes per launch from the committed counter runs (rocprofv3
            # FETCH_SIZE and WRITE_SIZE on this kernel source, workload and
            # tuning), not measured in this run; null when they no longer apply
            "traffic": traffic,
            "traffic_source": (("stored: profiles/sweep_kernel_traffic.json, kernel sources "
                                "sha256 %s" % traffic_rec["kernel_sources_sha256"][:16])
                               if traffic_rec else None),
            "traffic_frac": (round(traffic / sweep_s / 1e9 / HBM_PEAK_GBS, 5)
                             if traffic and sweep_s > 0 else None),
            "alg_bytes_per_launch": int(b_sweep),
            "frac_d1": head["frac_d1"],
            "sweep_ms": round(sweep["mean_ms"], 5),
            "secondary": secondary,
        },
        "cpu_baseline": dict(head["cpu_baseline"], host=host_record()),
        "checker": {"kind": "device check (mm_check)", "violations": head["violations"],
                    "size": head["size"], "size_sgmm": head["size_sgmm"], "t_seq": head["t_seq"]},
        "create_ms": head["create_ms"],
        "relabel_copy_bytes": head["relabel_copy_bytes"],
        "ordered_copy_bytes": head["ordered_copy_bytes"],
        "without_copy": head.get("without_copy"),
        "counters": counters,
        "conflicts": conflicts,
        "legs": others,
        "batch": batch,
        "serve": serving,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
