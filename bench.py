#!/usr/bin/env python3
"""Benchmark: exact-count pair throughput of the angular 2pcf hot path.

One step = the whole hot path over the large single-GPU workload (1e6
clustered data points, 2e6 uniform randoms over the octant, 40 log bins over
[0.0005, 30] deg): DD, DR and RR histograms on the GPU, copied to the host,
then Landy-Szalay w(theta).  Catalogs are resident in HBM before the timed
region starts.  The FP32-chord path is the headline value; the all-FP64 path
is timed beside it.  Prints one JSON line.

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
# FP32-VALU pair roofline: 256 CUs x 64 lanes x 2.4 GHz = 39.32e12 VALU lane
# issue slots per second, 4 slots per pair (chord^2 as packed FP32 plus one
# for the bin decision) -> 9.83e12 pairs/s.
PEAK_GPAIRS = 256 * 64 * 2.4e9 / 4 / 1e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["octant", "batched", "serving"], default="octant",
                    help="octant: 1e6 x 2e6 DD+DR+RR (default); batched: 64 uneven catalogs "
                         "against one 1e6 random in one launch; serving: Poisson job stream")
    ap.add_argument("--jobs", type=int, default=300, help="serving: number of jobs")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shape instead of tuning on a sample")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=float, default=1.0,
                    help="catalog size factor (1.0 = the full workload)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-matrix", action="store_true", help="skip the FP64 matrix-core path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    wl = synthcat.config4(scale=args.scale)
    e = wl.edges_deg
    ctx = tp.Context(0)
    cats = [ctx.upload_catalog(c.ra, c.dec) for c in wl.data]
    r = wl.randoms[0]
    cr = ctx.upload_catalog(r.ra, r.dec)
    jobs = [(tp.DD, c, -1) for c in cats] + [(tp.DR, c, cr) for c in cats] + [(tp.RR, cr, -1)]
    sizes = [c.n for c in wl.data]
    pairs = sum(n * (n - 1) // 2 for n in sizes) + sum(n * r.n for n in sizes) + r.n * (r.n - 1) // 2
    print(f"# batched: {len(jobs)} jobs, {pairs:.4e} pairs", file=sys.stderr, flush=True)
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
    # the same jobs as separate launches
    out = torch.zeros((len(jobs), e.size + 1), dtype=torch.int64, device="cuda:0")
    for k, (kind, a, b) in enumerate(jobs):
        ctx.count_async(kind, a, e, out[k].data_ptr(), cat_b=b)
    ctx.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        for k, (kind, a, b) in enumerate(jobs):
            ctx.count_async(kind, a, e, out[k].data_ptr(), cat_b=b)
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
        "roofline": {"bound": "alu", "achieved": round(kg, 1), "peak": round(PEAK_GPAIRS, 1),
                     "unit": "Gpairs/s", "frac": round(kg / PEAK_GPAIRS, 4), "traffic": None,
                     "kernel": "pairs_kernel<0> (FP32 chord), one launch per batch"},
        "separate_launches_gpairs_s": round(sep_value, 2),
        "batched_over_separate": round(value / sep_value, 3),
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
    rnd = [ctx.upload_catalog(c.ra, c.dec) for c in synthcat.config5_randoms(n_random)]
    spec = synthcat.config5_jobs(n_jobs=args.jobs, size_hi=int(1_000_000 * args.scale))
    print(f"# serving: generating {len(spec)} job catalogs", file=sys.stderr, flush=True)
    jobs = []
    for s in spec:
        j = Job(id=s["id"], kind=s["kind"], arrival=0.0, random=s["random"])
        if s["kind"] != "RR":
            c = synthcat.config5_catalog(s)
            j.ra, j.dec, j.n = c.ra, c.dec, c.n
        jobs.append(j)
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
    srv = Server(LibraryBackend(ctx, e), randoms=rnd, n_random=n_random, max_inflight=8)
    print(f"# serving: rate {rate/1e9:.0f} Gpairs/s, lambda {lam:.2f}/s, {len(jobs)} jobs",
          file=sys.stderr, flush=True)
    rep = srv.run(jobs)
    ctx.set_hbm_budget(0)
    # alone-vs-mix spot check: three completed jobs recounted alone
    for j in [x for x in jobs if x.kind == "DD"][:3]:
        c = ctx.upload_catalog(j.ra, j.dec)
        alone = ctx.count(tp.DD, c, e)
        ctx.release_catalog(c)
        if not np.array_equal(alone, rep.results[j.id]):
            sys.exit(f"job {j.id}: result in the mix differs from the result alone")
    value = rep.pairs / rep.makespan / 1e9
    ctx.close()
    return {
        "metric": METRIC, "value": round(value, 2), "unit": "Gpairs/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": round(rep.makespan * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "config5_serving", "jobs": len(jobs), "n_random": n_random,
                   "randoms": 3, "nbins": int(e.size - 1), "arrival_rate_per_s": round(lam, 3),
                   "hbm_budget_bytes": 1 << 30, "parallelism": "single-gpu"},
        "latency_ms": {"p50": round(rep.percentile(50) * 1e3, 2),
                       "p99": round(rep.percentile(99) * 1e3, 2)},
        "max_inflight": rep.max_inflight, "max_bytes": rep.max_bytes,
    }


def main():
    args = parse()
    if args.gpus != 1:
        sys.exit("bench.py runs on one GPU only: this build has no multi-GPU path "
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
    wl = synthcat.config3(scale=args.scale)
    d, r = wl.data[0], wl.randoms[0]
    nd, nr = d.n, r.n
    edges = wl.edges_deg
    nslots = edges.size + 1
    pairs_step = nd * (nd - 1) // 2 + nd * nr + nr * (nr - 1) // 2

    stream = torch.cuda.current_stream(dev)
    ctx = tp.Context(0, stream=stream.cuda_stream)
    cd = ctx.upload_catalog(d.ra, d.dec)
    cr = ctx.upload_catalog(r.ra, r.dec)
    out = torch.zeros((3, nslots), dtype=torch.int64, device=dev)
    tuning = None
    if not args.no_autotune:
        from paper_1204_6630_amd.autotune import autotune
        rows = min(nd, 32768)
        sample = [(tp.DR, cd, cr, 0, rows), (tp.DD, cd, -1, 0, rows)]
        tuning = autotune(ctx, sample, edges, tp.FP32_CHORD)
        print(f"# tuning: {tuning['tuning']} (cached: {tuning['cached']})", file=sys.stderr,
              flush=True)

    def step(prec):
        ctx.count_async(tp.DD, cd, edges, out[0].data_ptr(), precision=prec)
        ctx.count_async(tp.DR, cd, edges, out[1].data_ptr(), cat_b=cr, precision=prec)
        ctx.count_async(tp.RR, cr, edges, out[2].data_ptr(), precision=prec)
        h = out.cpu().numpy().astype(np.uint64)
        w = tp.landy_szalay(h[0], h[1], h[2], nd, nr)
        return h, w

    def run(prec, k, w):
        for _ in range(w):
            h, _ = step(prec)
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
        pairs, flagged, exact, rare = ctx.stats(reset=True)
        tot = [int(x.sum()) for x in h]
        ok = tot == [nd * (nd - 1) // 2, nd * nr, nr * (nr - 1) // 2]
        return {"s": t1 - t0, "kernel_ms": kms, "launches": launches, "hist": h, "w": ws,
                "totals_ok": ok, "flagged": flagged, "exact": exact, "pairs": pairs, "rare": rare}

    print(f"# workload {wl.name}: N_D={nd} N_R={nr} nbins={edges.size - 1} "
          f"pairs/step={pairs_step:.4e}", file=sys.stderr, flush=True)
    f32 = run(tp.FP32_CHORD, args.steps, args.warmup)
    print(f"# fp32-chord: {args.steps} steps in {f32['s']:.3f} s", file=sys.stderr, flush=True)
    f64 = None
    if not args.no_fp64:
        f64 = run(tp.FP64, args.steps, args.warmup)
        print(f"# fp64: {args.steps} steps in {f64['s']:.3f} s", file=sys.stderr, flush=True)
        if not all(np.array_equal(a, b) for a, b in zip(f32["hist"], f64["hist"])):
            sys.exit("FP32-chord and FP64 histograms differ")
    fmx = None
    if not args.no_matrix:
        fmx = run(tp.FP64_MATRIX, args.steps, args.warmup)
        print(f"# fp64-matrix: {args.steps} steps in {fmx['s']:.3f} s", file=sys.stderr, flush=True)
        if not all(np.array_equal(a, b) for a, b in zip(f32["hist"], fmx["hist"])):
            sys.exit("FP32-chord and FP64-matrix histograms differ")
    if not f32["totals_ok"]:
        sys.exit("slot totals do not match the pair counts")

    ms_step = f32["s"] / args.steps * 1e3
    value = pairs_step * args.steps / f32["s"] / 1e9
    k_gpairs = pairs_step * args.steps / (f32["kernel_ms"] / 1e3) / 1e9
    res = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Gpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_d": nd, "n_r": nr, "nbins": int(edges.size - 1),
                   "theta_deg": [float(edges[0]), float(edges[-1])],
                   "pairs_per_step": pairs_step, "kinds": "DD+DR+RR+LS",
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "alu", "achieved": round(k_gpairs, 1), "peak": round(PEAK_GPAIRS, 1),
                     "unit": "Gpairs/s", "frac": round(k_gpairs / PEAK_GPAIRS, 4),
                     "traffic": None, "kernel": "pairs_kernel<0> (FP32 chord)",
                     "kernel_ms_per_launch": round(f32["kernel_ms"] / max(1, f32["launches"]), 3)},
        "tuning": tuning["tuning"] if tuning else None,
        "fp32_chord": {"gpairs_s": round(value, 2), "kernel_gpairs_s": round(k_gpairs, 1),
                       "flagged_rate": f32["flagged"] / max(1, f32["pairs"]),
                       "recheck_rate": f32["exact"] / max(1, f32["pairs"]),
                       "rare_step_rate": f32["rare"] * 64 * 2 * ctx.get_tuning()["rows_per_lane"]
                       / max(1, f32["pairs"])},
    }
    if f64 is not None:
        v64 = pairs_step * args.steps / f64["s"] / 1e9
        k64 = pairs_step * args.steps / (f64["kernel_ms"] / 1e3) / 1e9
        res["fp64"] = {"gpairs_s": round(v64, 2), "kernel_gpairs_s": round(k64, 1),
                       "ms_per_step": round(f64["s"] / args.steps * 1e3, 3),
                       "flagged_rate": f64["flagged"] / max(1, f64["pairs"]),
                       "exact_rate": f64["exact"] / max(1, f64["pairs"])}
        res["fp32_over_fp64"] = round(value / v64, 3)
    if fmx is not None:
        vmx = pairs_step * args.steps / fmx["s"] / 1e9
        kmx = pairs_step * args.steps / (fmx["kernel_ms"] / 1e3) / 1e9
        res["fp64_matrix"] = {"gpairs_s": round(vmx, 2), "kernel_gpairs_s": round(kmx, 1),
                              "ms_per_step": round(fmx["s"] / args.steps * 1e3, 3),
                              "flagged_rate": fmx["flagged"] / max(1, fmx["pairs"]),
                              "exact_rate": fmx["exact"] / max(1, fmx["pairs"])}
    if not args.no_cpu_baseline:
        import oracle
        xd = oracle.radec_to_xyz(d.ra, d.dec)
        xr = oracle.radec_to_xyz(r.ra, r.dec)
        res["cpu_baseline"] = cpu_baseline(xd, xr, edges, args.cpu_seconds)
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
