#!/usr/bin/env python3
"""Benchmark: exact-count pair throughput of the angular 2pcf hot path.

One step = the whole hot path over the large single-GPU workload (1e6
clustered data points, 2e6 uniform randoms over the octant, 40 log bins over
[0.0005, 30] deg): DD, DR and RR histograms on the GPU, copied to the host,
then Landy-Szalay w(theta).  Catalogs are resident in HBM before the timed
region starts.  The two exact paths (FP32 chord, FP64 vector) are each timed
and checked against each other; the fastest is the headline value.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "exact-count Gpairs/s, FP32-chord vs FP64 path; p50/p99 job latency"
# ALU roofline of the FP32 angular kernel: 256 CUs x 4 SIMDs x 32 FP32 lanes
# x 2.4 GHz = 78.6e12 FP32 lane operations per second (157.3 TFLOP/s counting
# an FMA as two).  The kernel decides a pair from the dot product of the FP32
# copies where that suffices, so a pair needs at least 4 of them: one
# multiply and two FMAs for p, one to bin it.  Chord-only kernels (pruned
# launches) and the 3-D squared distance need at least 7: 3 subtractions,
# one multiply and two FMAs, and the table key.
FP32_LANE_OPS = 256 * 4 * 32 * 2.4e9
OPS_PER_PAIR_FP32 = 4
OPS_PER_PAIR_CHORD = 7
# FP64 vector path: 78.6e12 FP64 lane operations per second; a pair needs 6
# (three products, two sums, 1 - d) plus the key.
FP64_LANE_OPS = 256 * 4 * 16 * 2.4e9
OPS_PER_PAIR_FP64 = 7
PATH_NAMES = {0: "fp32_chord", 1: "fp64"}
# the FP32 angular kernel decides steps from the dot product first and forms
# the chord where that does not settle them
KERNEL_NAMES = {0: "pairs_kernel<6> (FP32, dot product first, chord where needed)",
                1: "pairs_kernel<1> (FP64 vector)"}
HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(HERE, "profiles", "hbm_traffic_octant_1e6x2e6.txt")


def kernel_source_hash() -> str:
    """SHA-256 of the kernel sources with comments and layout removed, so that
    an edit of a comment does not orphan counters taken on the same code."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("kernels.hip", "internal.h"):
        with open(os.path.join(HERE, "paper_1204_6630_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic(path: str):
    """HBM bytes per launch of a pair kernel on the octant workload, from the
    committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when the
    kernel sources changed since those counters were taken."""
    try:
        rows = dict(line.split()[:2] for line in open(TRAFFIC_FILE)
                    if line.strip() and not line.startswith("#"))
    except (OSError, ValueError):
        return None
    if rows.get("kernels_sha256") != kernel_source_hash() or path not in rows:
        return None
    return int(float(rows[path]))


def roofline(prec: int, kernel_gpairs: float, ms_per_launch: float, traffic=None, kernel=None,
             ops_per_pair=None) -> dict:
    if prec == 0:
        peak = FP32_LANE_OPS / (ops_per_pair or OPS_PER_PAIR_FP32) / 1e9
    else:
        peak = FP64_LANE_OPS / (ops_per_pair or OPS_PER_PAIR_FP64) / 1e9
    roof = {"bound": "alu", "achieved": round(kernel_gpairs, 1), "peak": round(peak, 1),
            "unit": "Gpairs/s", "frac": round(kernel_gpairs / peak, 4)}
    roof.update({"traffic": traffic, "kernel": kernel or KERNEL_NAMES[prec],
                 "kernel_ms_per_launch": round(ms_per_launch, 3)})
    return roof


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["octant", "batched", "serving"], default="octant",
                    help="octant: 1e6 x 2e6 DD+DR+RR (default); batched: 64 uneven catalogs "
                         "against one 1e6 random in one launch; serving: Poisson job stream")
    ap.add_argument("--jobs", type=int, default=300, help="serving: number of jobs")
    ap.add_argument("--defer-release-mb", type=int, default=1024,
                    help="serving: finished jobs' catalogs are released in batches of up to "
                         "this many MiB (0 releases each at its job's completion)")
    ap.add_argument("--autotune", action="store_true",
                    help="tune each path's launch shape on a sample first (default: the "
                         "library's defaults, which are the tuned shapes for this workload)")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=float, default=1.0,
                    help="catalog size factor (1.0 = the full workload)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-prune", action="store_true",
                    help="skip the extra run with exact tile pruning (never the headline)")
    ap.add_argument("--no-jackknife", action="store_true",
                    help="skip the jackknife-region step (8 x 8 regions over the octant)")
    ap.add_argument("--no-3d", action="store_true",
                    help="skip the 3-D xi(r) step (1e6 x 2e6 points in a box of side 1000)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--theta-max", type=float, default=0.0,
                    help="octant workload: last edge in degrees (0: the workload's 30 deg)")
    ap.add_argument("--batched-steps", type=int, default=2,
                    help="default line: timed steps of the batched 64-catalog leg (0 skips it)")
    ap.add_argument("--serving-jobs", type=int, default=120,
                    help="octant workload: jobs of the bounded serving leg (p50/p99 latency "
                         "in the same line); 0 skips it")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-size "
                         "reference for profiler byte counters)")
    return ap.parse_args()


def cpu_baseline(xd, xr, edges, seconds):
    """The oracle on the host cores over a bounded sample: DR rows [0, R) of
    the data catalog against the whole random catalog."""
    import oracle
    threads = oracle.default_threads()
    rows = max(8, 2 * threads)
    while True:     # grow the sample until it takes a quarter of the budget
        t = time.perf_counter()
        oracle.count(oracle.DR, xd, edges, b_xyz=xr, row_begin=0, row_end=rows, nthreads=threads)
        dt = time.perf_counter() - t
        if dt >= seconds / 4 or rows >= xd[0].size:
            break
        rows = min(xd[0].size, rows * 4)
    rows = int(min(xd[0].size, max(rows, rows * seconds / max(dt, 1e-3))))
    t = time.perf_counter()
    oracle.count(oracle.DR, xd, edges, b_xyz=xr, row_begin=0, row_end=rows, nthreads=threads)
    dt = time.perf_counter() - t
    pairs = rows * xr[0].size
    return {"value": pairs / dt / 1e9, "unit": "Gpairs/s", "cores": threads, "kind": "oracle",
            "sample": f"DR, data rows [0,{rows}) x {xr[0].size} randoms = {pairs:.3e} pairs "
                      f"in {dt:.1f} s"}


def bench_batched(args, tp, torch):
    """64 data catalogs of uneven size (each in a 20x20 deg sub-patch) and one
    resident 1e6-point uniform random catalog: 64 DD + 64 DR + 1 RR jobs.
    Timed: the whole batch as one hipGraph-replayed launch, and beside it the
    same jobs as 129 separate launches."""
    import synthcat
    wl = synthcat.batched_64(scale=args.scale)
    e = wl.edges_deg
    ctx = tp.Context(0)
    cats = [ctx.upload_catalog(c.ra, c.dec) for c in wl.data]
    r = wl.randoms[0]
    cr = ctx.upload_catalog(r.ra, r.dec)
    jobs = [(tp.DD, c, -1) for c in cats] + [(tp.DR, c, cr) for c in cats] + [(tp.RR, cr, -1)]
    sizes = [c.n for c in wl.data]
    pairs = sum(n * (n - 1) // 2 for n in sizes) + sum(n * r.n for n in sizes) + r.n * (r.n - 1) // 2
    print(f"# batched: {len(jobs)} jobs, {pairs:.4e} pairs", file=sys.stderr, flush=True)
    tuning = {"autotuned": False}
    if args.autotune:
        # the launch shape for this workload: a sample of DR row blocks of the
        # two largest catalogs against the randoms and a DD block
        from paper_1204_6630_amd.autotune import autotune
        big = sorted(range(len(cats)), key=lambda k: -sizes[k])[:2]
        sample = [(tp.DR, cats[k], cr, 0, min(sizes[k], 8192)) for k in big]
        sample.append((tp.DD, cats[big[0]], -1, 0, min(sizes[big[0]], 8192)))
        t = autotune(ctx, sample, e, tp.FP32_CHORD)
        tuning = dict(t["tuning"], autotuned=True, cached=t["cached"])
        print(f"# batched tuning: {tuning}", file=sys.stderr, flush=True)
    ref = ctx.count_batch(jobs, e, graph=True)          # capture + warm-up
    for _ in range(args.warmup):
        ctx.count_batch(jobs, e, graph=True)
    ctx.kernel_time(reset=True)
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        got = ctx.count_batch(jobs, e, graph=True)
    t1 = time.perf_counter()
    ctx.set_timing(False)
    kms, launches = ctx.kernel_time(reset=True)
    if not np.array_equal(got, ref):
        sys.exit("graph replay differs from the first batch")
    # the same jobs as separate plain launches (the library's default shape)
    ctx.set_tuning()
    out = torch.zeros((len(jobs), e.size + 1), dtype=torch.int64, device="cuda:0")
    for k, (kind, a, b) in enumerate(jobs):
        ctx.count_async(kind, a, e, out[k].data_ptr(), cat_b=b)
    ctx.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        for k, (kind, a, b) in enumerate(jobs):
            ctx.count_async(kind, a, e, out[k].data_ptr(), cat_b=b)
        ctx.synchronize()       # the library's stream, not torch's
        sep = out.cpu().numpy().astype(np.uint64)
    t3 = time.perf_counter()
    if not np.array_equal(sep, ref):
        sys.exit("separate launches differ from the batch")
    value = pairs * args.steps / (t1 - t0) / 1e9
    sep_value = pairs * args.steps / (t3 - t2) / 1e9
    kg = pairs * args.steps / (kms / 1e3) / 1e9
    ctx.close()
    return {
        "metric": METRIC, "value": round(value, 2), "unit": "Gpairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round((t1 - t0) / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": wl.name, "catalogs": len(cats), "n_random": r.n,
                   "nbins": int(e.size - 1), "pairs_per_step": pairs, "jobs": len(jobs),
                   "parallelism": "single-gpu"},
        "roofline": roofline(tp.FP32_CHORD, kg, kms / max(1, launches),
                             kernel=KERNEL_NAMES[0] + ", one launch for all jobs"),
        "separate_launches_gpairs_s": round(sep_value, 2),
        "batched_over_separate": round(value / sep_value, 3),
        "tuning": tuning,
    }


def bench_serving(args, tp):
    """Poisson arrivals of DD/DR/RR jobs (40/40/20), catalog sizes log-uniform
    in [1e3, 1e6], clustered or uniform over the octant, three resident 2e6
    random catalogs, HBM budget 1 GiB for the jobs' memory.  The arrival rate is
    0.7 x the measured sustained rate / the mean pairs per job."""
    import synthcat
    from paper_1204_6630_amd.serving import Job, LibraryBackend, Server, poisson_arrivals
    e = synthcat.log_edges(0.001, 20.0, 30)
    ctx = tp.Context(0)
    n_random = int(round(2_000_000 * args.scale))
    rnd = [ctx.upload_catalog(c.ra, c.dec) for c in synthcat.serving_randoms(n_random)]
    spec = synthcat.serving_jobs(n_jobs=args.jobs, size_hi=int(1_000_000 * args.scale))
    print(f"# serving: generating {len(spec)} job catalogs", file=sys.stderr, flush=True)
    jobs = []
    for k, s in enumerate(spec):
        j = Job(id=s["id"], kind=s["kind"], arrival=0.0, random=s["random"])
        if s["kind"] != "RR":
            c = synthcat.serving_catalog(s)
            j.ra, j.dec, j.n = c.ra, c.dec, c.n
        jobs.append(j)
        if (k + 1) % 250 == 0:
            print(f"# serving: {k + 1} job catalogs generated", file=sys.stderr, flush=True)
    # sustained rate: one DR of a 1e5 catalog against a resident random
    g = synthcat.rng_for(5, 999)
    probe = ctx.upload_catalog(*synthcat.uniform_patch(100_000, synthcat.OCTANT, g))
    ctx.count(tp.DR, probe, e, cat_b=rnd[0])
    t = time.perf_counter()
    ctx.count(tp.DR, probe, e, cat_b=rnd[0])
    rate = 100_000 * n_random / (time.perf_counter() - t)
    ctx.release_catalog(probe)
    mean_pairs = np.mean([j.pairs(n_random) if j.kind != "RR" else 0 for j in jobs])
    lam = 0.7 * rate / mean_pairs
    arr = poisson_arrivals(len(jobs), lam, synthcat.rng_for(5, 1000))
    for j, a in zip(jobs, arr):
        j.arrival = float(a)
    used0, _ = ctx.hbm_usage()
    ctx.set_hbm_budget(used0 + (1 << 30))
    srv = Server(LibraryBackend(ctx, e), randoms=rnd, n_random=n_random, max_inflight=8,
                 max_deferred_bytes=args.defer_release_mb << 20)
    print(f"# serving: rate {rate/1e9:.0f} Gpairs/s, lambda {lam:.2f}/s, {len(jobs)} jobs",
          file=sys.stderr, flush=True)
    ctx.stats(reset=True)
    rep = srv.run(jobs)
    computed = ctx.stats(reset=True).pairs     # launched pairs: cached RR results excluded
    ctx.set_hbm_budget(0)
    # alone-vs-mix spot check: three completed jobs recounted alone
    for j in [x for x in jobs if x.kind == "DD"][:3]:
        c = ctx.upload_catalog(j.ra, j.dec)
        alone = ctx.count(tp.DD, c, e)
        ctx.release_catalog(c)
        if not np.array_equal(alone, rep.results[j.id]):
            sys.exit(f"job {j.id}: result in the mix differs from the result alone")
    value = computed / rep.makespan / 1e9
    ctx.close()
    return {
        "metric": METRIC, "value": round(value, 2), "unit": "Gpairs/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": round(rep.makespan * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "serving_stream", "jobs": len(jobs), "n_random": n_random,
                   "randoms": 3, "nbins": int(e.size - 1), "arrival_rate_per_s": round(lam, 3),
                   "hbm_budget_bytes": 1 << 30, "defer_release_mb": args.defer_release_mb,
                   "parallelism": "single-gpu"},
        "latency_ms": {"p50": round(rep.percentile(50) * 1e3, 2),
                       "p99": round(rep.percentile(99) * 1e3, 2)},
        "computed_pairs": computed, "served_pairs": rep.pairs,
        "served_gpairs_s_with_rr_cache": round(rep.pairs / rep.makespan / 1e9, 2),
        "max_inflight": rep.max_inflight, "max_bytes": rep.max_bytes,
    }


def main():
    args = parse()
    if args.gpus != 1:
        sys.exit("bench.py runs on one GPU only: the library has no multi-GPU path "
                 f"(asked for --gpus {args.gpus})")
    import torch
    import paper_1204_6630_amd as tp
    import synthcat

    if not torch.cuda.is_available():
        sys.exit("bench.py needs a GPU")
    tp.lib()    # fails loudly if the HIP library is not built
    if args.workload == "batched":
        print(json.dumps(bench_batched(args, tp, torch)), flush=True)
        return
    if args.workload == "serving":
        print(json.dumps(bench_serving(args, tp)), flush=True)
        return
    dev = torch.device("cuda:0")
    if args.copy_probe_mb:
        src = torch.ones(args.copy_probe_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wl = synthcat.octant_1e6x2e6(scale=args.scale)
    d, r = wl.data[0], wl.randoms[0]
    nd, nr = d.n, r.n
    edges = wl.edges_deg
    if args.theta_max:
        # the same catalogs with the 40 log bins reaching theta_max (edges to
        # 120 deg leave no wavefront step wholly beyond the last edge)
        edges = synthcat.log_edges(float(edges[0]), args.theta_max, edges.size - 1)
    nslots = edges.size + 1
    pairs_step = nd * (nd - 1) // 2 + nd * nr + nr * (nr - 1) // 2

    ctx = tp.Context(0)
    t_up = time.perf_counter()
    cd = ctx.upload_catalog(d.ra, d.dec)
    cr = ctx.upload_catalog(r.ra, r.dec)
    t_up = time.perf_counter() - t_up
    out = torch.zeros((3, nslots), dtype=torch.int64, device=dev)
    torch.cuda.synchronize()    # torch's stream is not the context's
    rows = min(nd, 32768)
    tune_sample = [(tp.DR, cd, cr, 0, rows), (tp.DD, cd, -1, 0, rows)]

    def tune(prec):
        if not args.autotune:
            ctx.set_tuning()
            return None
        from paper_1204_6630_amd.autotune import autotune
        t = autotune(ctx, tune_sample, edges, prec)
        print(f"# tuning {PATH_NAMES[prec]}: {t['tuning']} (cached: {t['cached']})",
              file=sys.stderr, flush=True)
        return t["tuning"]

    def step(prec):
        ctx.count_async(tp.DD, cd, edges, out[0].data_ptr(), precision=prec)
        ctx.count_async(tp.DR, cd, edges, out[1].data_ptr(), cat_b=cr, precision=prec)
        ctx.count_async(tp.RR, cr, edges, out[2].data_ptr(), precision=prec)
        ctx.synchronize()       # the context's own stream, not torch's
        h = out.cpu().numpy().astype(np.uint64)
        w = tp.landy_szalay(h[0], h[1], h[2], nd, nr)
        return h, w

    first_step = {}

    def run(prec, k, w):
        tuning = tune(prec)
        for i in range(w):
            t = time.perf_counter()
            h, _ = step(prec)
            if i == 0:      # includes the edge compiler, plans and operand packs
                first_step[prec] = time.perf_counter() - t
        torch.cuda.synchronize()
        ctx.kernel_time(reset=True)
        ctx.stats(reset=True)
        ctx.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(k):
            h, ws = step(prec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.set_timing(False)
        kms, launches = ctx.kernel_time(reset=True)
        st = ctx.stats(reset=True)
        # per kind: one more launch of each, timed alone with HIP events
        per_kind = {}
        for name, kind, a, b, npairs in (("DD", tp.DD, cd, -1, nd * (nd - 1) // 2),
                                         ("DR", tp.DR, cd, cr, nd * nr),
                                         ("RR", tp.RR, cr, -1, nr * (nr - 1) // 2)):
            ctx.set_timing(True)
            ctx.count_async(kind, a, edges, out[0].data_ptr(), cat_b=b, precision=prec)
            ctx.synchronize()
            ctx.set_timing(False)
            ms, _ = ctx.kernel_time(reset=True)
            per_kind[name] = round(npairs / (ms / 1e3) / 1e9, 1)
        ctx.stats(reset=True)
        tot = [int(x.sum()) for x in h]
        ok = tot == [nd * (nd - 1) // 2, nd * nr, nr * (nr - 1) // 2]
        t = ctx.get_tuning()     # 0 = the library's default
        rpl = t["rows_per_lane"] or 4
        tuning = dict(t, rows_per_lane=rpl, autotuned=tuning is not None)
        rows_per_step = rpl * 64
        cols_per_step = {tp.FP32_CHORD: 4, tp.FP64: 2}[prec]
        return {"s": t1 - t0, "kernel_ms": kms, "launches": launches, "hist": h, "w": ws,
                "totals_ok": ok, "flagged": st.flagged, "exact": st.exact, "pairs": st.pairs,
                "rare": st.rare_steps, "beyond": st.beyond_steps, "one_slot": st.one_slot_steps,
                "two_slot": st.two_slot_steps, "chord": st.chord_steps, "per_kind": per_kind,
                "tuning": tuning, "pairs_per_wave_step": rows_per_step * cols_per_step}

    print(f"# workload {wl.name}: N_D={nd} N_R={nr} nbins={edges.size - 1} "
          f"pairs/step={pairs_step:.4e}", file=sys.stderr, flush=True)
    paths = [tp.FP32_CHORD]
    if not args.no_fp64:
        paths.append(tp.FP64)
    runs = {}
    for prec in paths:
        runs[prec] = run(prec, args.steps, args.warmup)
        print(f"# {PATH_NAMES[prec]}: {args.steps} steps in {runs[prec]['s']:.3f} s",
              file=sys.stderr, flush=True)
        if not runs[prec]["totals_ok"]:
            sys.exit(f"{PATH_NAMES[prec]}: slot totals do not match the pair counts")
        if not all(np.array_equal(a, b) for a, b in zip(runs[paths[0]]["hist"], runs[prec]["hist"])):
            sys.exit(f"{PATH_NAMES[paths[0]]} and {PATH_NAMES[prec]} histograms differ")

    def summary(prec):
        r = runs[prec]
        v = pairs_step * args.steps / r["s"] / 1e9
        kv = pairs_step * args.steps / (r["kernel_ms"] / 1e3) / 1e9
        return {"gpairs_s": round(v, 2), "kernel_gpairs_s": round(kv, 1),
                "kernel_gpairs_s_per_kind": r["per_kind"],
                "ms_per_step": round(r["s"] / args.steps * 1e3, 3),
                "kernel_ms_per_launch": round(r["kernel_ms"] / max(1, r["launches"]), 3),
                "tuning": r["tuning"],
                "flagged_rate": r["flagged"] / max(1, r["pairs"]),
                "exact_rate": r["exact"] / max(1, r["pairs"]),
                "rare_step_rate": r["rare"] * r["pairs_per_wave_step"] / max(1, r["pairs"]),
                "beyond_last_edge_rate": r["beyond"] * r["pairs_per_wave_step"] / max(1, r["pairs"]),
                "one_slot_rate": r["one_slot"] * r["pairs_per_wave_step"] / max(1, r["pairs"]),
                "two_slot_rate": r["two_slot"] * r["pairs_per_wave_step"] / max(1, r["pairs"]),
                "chord_step_rate": r["chord"] * r["pairs_per_wave_step"] / max(1, r["pairs"])}

    sums = {prec: summary(prec) for prec in paths}
    pruned = None
    if not args.no_prune:
        # exact tile pruning (FP32 chord): whole blocks are binned without
        # evaluating their pairs, so this is not the brute-force rate and is
        # never the headline; same histograms required
        ctx.set_tuning(prune=1)
        step(tp.FP32_CHORD)
        torch.cuda.synchronize()
        ctx.stats(reset=True)
        ctx.kernel_time(reset=True)
        ctx.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            hp, _ = step(tp.FP32_CHORD)
        t1 = time.perf_counter()
        ctx.set_timing(False)
        kms, _ = ctx.kernel_time(reset=True)
        st = ctx.stats(reset=True)
        ctx.set_tuning()
        if not all(np.array_equal(a, b) for a, b in zip(runs[paths[0]]["hist"], hp)):
            sys.exit("pruned and brute-force histograms differ")
        evaluated = st.pairs - st.pruned_pairs
        pruned = {"gpairs_s_algorithmic": round(pairs_step * args.steps / (t1 - t0) / 1e9, 2),
                  "ms_per_step": round((t1 - t0) / args.steps * 1e3, 3),
                  "kernel_ms_per_step": round(kms / args.steps, 3),
                  "pruned_fraction": round(st.pruned_pairs / max(1, st.pairs), 4),
                  # the roofline of the pairs the kernel still evaluated
                  "roofline_evaluated_pairs": roofline(
                      tp.FP32_CHORD, evaluated / (kms / 1e3) / 1e9, kms / (3 * args.steps),
                      kernel="pairs_kernel<0> with pruning (FP32 chord)", ops_per_pair=OPS_PER_PAIR_CHORD),
                  "note": "exact tile pruning (tuning prune=1): same counts; pairs of pruned "
                          "blocks are not evaluated, so not comparable to value"}
    jack = None
    if not args.no_jackknife:
        # jackknife regions: the same catalogs labelled with an 8 x 8 RA/Dec
        # grid (64 regions); one step = DD, DR, RR with per-region counts
        # (FP32 chord path) and the host delete-one jackknife of w
        nreg = 64
        lab_d = synthcat.grid_regions(d.ra, d.dec, synthcat.OCTANT, 8, 8)
        lab_r = synthcat.grid_regions(r.ra, r.dec, synthcat.OCTANT, 8, 8)
        jd = ctx.upload_catalog_regions(d.ra, d.dec, lab_d, nreg)
        jr = ctx.upload_catalog_regions(r.ra, r.dec, lab_r, nreg)
        nd_reg, nr_reg = ctx.catalog_regions(jd), ctx.catalog_regions(jr)

        def jstep():
            a = ctx.count_regions(tp.DD, jd, edges)
            b = ctx.count_regions(tp.DR, jd, edges, cat_b=jr)
            c = ctx.count_regions(tp.RR, jr, edges)
            tp.jackknife(a[0], a[1], b[0], b[1], c[0], c[1], nd, nd_reg, nr, nr_reg)
            return a, b, c

        jstep()
        ctx.kernel_time(reset=True)
        ctx.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ja, jb_, jc = jstep()
        t1 = time.perf_counter()
        ctx.set_timing(False)
        kms, _ = ctx.kernel_time(reset=True)
        ctx.stats(reset=True)
        if not all(np.array_equal(x[0], y) for x, y in zip((ja, jb_, jc), runs[paths[0]]["hist"])):
            sys.exit("jackknife-region totals and brute-force histograms differ")
        ms = (t1 - t0) / args.steps * 1e3
        jack = {"nreg": nreg, "gpairs_s": round(pairs_step * args.steps / (t1 - t0) / 1e9, 2),
                "ms_per_step": round(ms, 3), "kernel_ms_per_step": round(kms / args.steps, 3),
                "roofline": roofline(tp.FP32_CHORD, pairs_step * args.steps / (kms / 1e3) / 1e9,
                                     kms / (3 * args.steps),
                                     kernel="pairs_kernel<6> with region copies (FP32)"),
                "over_plain_step": round(ms / sums[tp.FP32_CHORD]["ms_per_step"], 3),
                "note": "DD+DR+RR with per-region counts (FP32 chord) + host jackknife of w; "
                        "same totals as the plain step"}
        ctx.release_catalog(jd)
        ctx.release_catalog(jr)
    xi3d = None
    if not args.no_3d:
        # the 3-D variant xi(r): same kernels keyed on squared distances; one
        # step = DD + DR + RR + Landy-Szalay on a 1e6 x 2e6 box workload
        w3 = synthcat.box_1e6x2e6(scale=args.scale)
        b_d = ctx.upload_catalog_3d(*w3.data.xyz())
        b_r = ctx.upload_catalog_3d(*w3.randoms.xyz())
        n3d, n3r = w3.data.n, w3.randoms.n
        pairs3 = n3d * (n3d - 1) // 2 + n3d * n3r + n3r * (n3r - 1) // 2
        out3 = torch.zeros((3, w3.edges.size + 1), dtype=torch.int64, device=dev)
        torch.cuda.synchronize()
        xi3d = {"workload": w3.name, "n_d": n3d, "n_r": n3r, "nbins": int(w3.edges.size - 1),
                "r_range": [float(w3.edges[0]), float(w3.edges[-1])], "pairs_per_step": pairs3}
        hist3 = {}
        for prec in (tp.FP32_CHORD, tp.FP64):
            def step3():
                ctx.count_async(tp.DD, b_d, w3.edges, out3[0].data_ptr(), precision=prec)
                ctx.count_async(tp.DR, b_d, w3.edges, out3[1].data_ptr(), cat_b=b_r, precision=prec)
                ctx.count_async(tp.RR, b_r, w3.edges, out3[2].data_ptr(), precision=prec)
                ctx.synchronize()
                h = out3.cpu().numpy().astype(np.uint64)
                tp.landy_szalay(h[0], h[1], h[2], n3d, n3r)
                return h
            step3()
            ctx.kernel_time(reset=True)
            ctx.stats(reset=True)
            ctx.set_timing(True)
            t0 = time.perf_counter()
            for _ in range(args.steps):
                h3 = step3()
            t1 = time.perf_counter()
            ctx.set_timing(False)
            kms, nl = ctx.kernel_time(reset=True)
            st = ctx.stats(reset=True)
            if [int(x.sum()) for x in h3] != [n3d * (n3d - 1) // 2, n3d * n3r, n3r * (n3r - 1) // 2]:
                sys.exit("3-D slot totals do not match the pair counts")
            hist3[prec] = h3
            xi3d[PATH_NAMES[prec]] = {
                "gpairs_s": round(pairs3 * args.steps / (t1 - t0) / 1e9, 2),
                "kernel_gpairs_s": round(pairs3 * args.steps / (kms / 1e3) / 1e9, 1),
                "ms_per_step": round((t1 - t0) / args.steps * 1e3, 3),
                "kernel_ms_per_launch": round(kms / max(1, nl), 3),
                "exact_rate": st.exact / max(1, st.pairs),
                # FP32: 3 differences, a square, 2 FMAs and the key (as for
                # angles); FP64: 3 differences, 3 squares, 2 sums (the key
                # is the high word of r^2)
                "roofline": roofline(prec, pairs3 * args.steps / (kms / 1e3) / 1e9, kms / max(1, nl),
                                     kernel={tp.FP32_CHORD: "pairs_kernel<5> (3-D FP32)",
                                             tp.FP64: "pairs_kernel<4> (3-D FP64)"}[prec],
                                     ops_per_pair=OPS_PER_PAIR_CHORD if prec == tp.FP32_CHORD else 8)}
        for other in (tp.FP64,):
            if not all(np.array_equal(a, b) for a, b in zip(hist3[tp.FP32_CHORD], hist3[other])):
                sys.exit("3-D histograms differ between precisions")
        if not args.no_prune:
            # the same 3-D step with exact tile pruning (bounding balls), FP32
            ctx.set_tuning(prune=1)
            prec = tp.FP32_CHORD
            step3()
            ctx.kernel_time(reset=True)
            ctx.stats(reset=True)
            ctx.set_timing(True)
            t0 = time.perf_counter()
            for _ in range(args.steps):
                h3p = step3()
            t1 = time.perf_counter()
            ctx.set_timing(False)
            kms, _ = ctx.kernel_time(reset=True)
            st = ctx.stats(reset=True)
            ctx.set_tuning()
            if not all(np.array_equal(a, b) for a, b in zip(hist3[tp.FP32_CHORD], h3p)):
                sys.exit("3-D pruned and brute-force histograms differ")
            xi3d["fp32_pruned"] = {"gpairs_s_algorithmic": round(pairs3 * args.steps / (t1 - t0) / 1e9, 2),
                                   "kernel_ms_per_step": round(kms / args.steps, 3),
                                   "pruned_fraction": round(st.pruned_pairs / max(1, st.pairs), 4)}
        ctx.release_catalog(b_d)
        ctx.release_catalog(b_r)
        del out3
    head = max(paths, key=lambda p: sums[p]["gpairs_s"])
    hs = sums[head]
    roof = roofline(head, hs["kernel_gpairs_s"], hs["kernel_ms_per_launch"],
                    measured_traffic(PATH_NAMES[head]) if args.scale == 1.0 and not args.theta_max else None)
    res = {
        "metric": METRIC,
        "value": hs["gpairs_s"],
        "unit": "Gpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hs["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head != tp.FP32_CHORD else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_d": nd, "n_r": nr, "nbins": int(edges.size - 1),
                   "theta_deg": [float(edges[0]), float(edges[-1])],
                   "pairs_per_step": pairs_step, "kinds": "DD+DR+RR+LS",
                   "parallelism": "single-gpu"},
        "headline_path": PATH_NAMES[head],
        "roofline": roof,
        "end_to_end": {"upload_s": round(t_up, 3),
                       "first_step_s": round(first_step.get(head, float("nan")), 3),
                       "note": "catalog upload (host RA/Dec to resident FP64/FP32 SoA) and the "
                               "first step with the edge compiler and plans; not in value"},
    }
    for prec in paths:
        res[PATH_NAMES[prec]] = sums[prec]
    if pruned is not None:
        res["fp32_chord_pruned"] = pruned
    if jack is not None:
        res["jackknife_regions"] = jack
    if xi3d is not None:
        res["xi_r_3d"] = xi3d
    if tp.FP64 in sums:
        res["fp32_over_fp64"] = round(sums[tp.FP32_CHORD]["gpairs_s"] / sums[tp.FP64]["gpairs_s"], 3)
    if not args.no_cpu_baseline:
        import oracle
        xd = oracle.radec_to_xyz(d.ra, d.dec)
        xr = oracle.radec_to_xyz(r.ra, r.dec)
        cb = cpu_baseline(xd, xr, edges, args.cpu_seconds)
        cb["extrapolated_full_step_s"] = round(pairs_step / (cb["value"] * 1e9), 1)
        res["cpu_baseline"] = cb
    ctx.close()
    if args.serving_jobs > 0:
        # the metric's latency half: a bounded Poisson job stream on a context
        # of its own (the serving workload's recipe with fewer jobs)
        sv = bench_serving(argparse.Namespace(**{**vars(args), "jobs": args.serving_jobs}), tp)
        res["serving_stream"] = {
            "jobs": sv["config"]["jobs"], "n_random": sv["config"]["n_random"],
            "arrival_rate_per_s": sv["config"]["arrival_rate_per_s"],
            "latency_ms": sv["latency_ms"], "gpairs_s_launched": sv["value"],
            "served_gpairs_s_with_rr_cache": sv["served_gpairs_s_with_rr_cache"],
            "makespan_s": round(sv["ms_per_step"] / 1e3, 3), "max_inflight": sv["max_inflight"],
            "note": "DD/DR/RR jobs 40/40/20, sizes log-uniform [1e3, 1e6], 3 resident 2e6 "
                    "randoms with cached RR, 1 GiB HBM budget; latency = arrival to result "
                    "on the host; not in value"}
    if args.batched_steps > 0:
        # the batched workload's leg: 129 jobs in one graph-replayed launch
        # (autotuned launch shape) against the same jobs as separate launches
        bt = bench_batched(argparse.Namespace(**{**vars(args), "steps": args.batched_steps, "warmup": 1,
                                                 "autotune": True}), tp, torch)
        res["batched_64"] = {
            "workload": bt["config"]["workload"], "jobs": bt["config"]["jobs"],
            "pairs_per_step": bt["config"]["pairs_per_step"], "steps": bt["steps"],
            "gpairs_s_one_launch": bt["value"], "ms_per_step": bt["ms_per_step"],
            "separate_launches_gpairs_s": bt["separate_launches_gpairs_s"],
            "batched_over_separate": bt["batched_over_separate"], "roofline": bt["roofline"],
            "tuning": bt["tuning"],
            "note": "64 data catalogs (5e3..5e5 points, 20x20 deg sub-patches) + one 1e6 random "
                    "catalog: 64 DD + 64 DR + 1 RR jobs in one hipGraph-replayed launch; not in value"}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
