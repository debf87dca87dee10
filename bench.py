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
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=float, default=1.0,
                    help="catalog size factor (1.0 = the full workload)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
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
    dev = torch.device("cuda:0")
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
        pairs, flagged, exact = ctx.stats(reset=True)
        tot = [int(x.sum()) for x in h]
        ok = tot == [nd * (nd - 1) // 2, nd * nr, nr * (nr - 1) // 2]
        return {"s": t1 - t0, "kernel_ms": kms, "launches": launches, "hist": h, "w": ws,
                "totals_ok": ok, "flagged": flagged, "exact": exact, "pairs": pairs}

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
        "fp32_chord": {"gpairs_s": round(value, 2), "kernel_gpairs_s": round(k_gpairs, 1),
                       "flagged_rate": f32["flagged"] / max(1, f32["pairs"]),
                       "recheck_rate": f32["exact"] / max(1, f32["pairs"])},
    }
    if f64 is not None:
        v64 = pairs_step * args.steps / f64["s"] / 1e9
        k64 = pairs_step * args.steps / (f64["kernel_ms"] / 1e3) / 1e9
        res["fp64"] = {"gpairs_s": round(v64, 2), "kernel_gpairs_s": round(k64, 1),
                       "ms_per_step": round(f64["s"] / args.steps * 1e3, 3),
                       "flagged_rate": f64["flagged"] / max(1, f64["pairs"]),
                       "exact_rate": f64["exact"] / max(1, f64["pairs"])}
        res["fp32_over_fp64"] = round(value / v64, 3)
    if not args.no_cpu_baseline:
        import oracle
        xd = oracle.radec_to_xyz(d.ra, d.dec)
        xr = oracle.radec_to_xyz(r.ra, r.dec)
        res["cpu_baseline"] = cpu_baseline(xd, xr, edges, args.cpu_seconds)
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
