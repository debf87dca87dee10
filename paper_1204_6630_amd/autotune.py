"""Autotuner for the pair kernels' launch shape.

Knobs: rows held per lane, LDS
histogram copies per wavefront, the largest column range of a work unit, the
grid size, the cell-table budget and, for FP32 byte tables, the wrapped or the
clamped table layout.  The search is a coordinate descent from the library's
defaults: each knob in turn is swept over its candidates with the others held
at the best values so far, on a sample of the caller's workload (a block of
rows against the full column catalog) timed with the library's HIP-event
kernel timer.  The best shape is applied to the context and cached on disk,
keyed by device, HIP runtime, precision and bin count.  Counts never depend
on the choice.
"""

from __future__ import annotations

import json
import os
import time

from . import FP32_CHORD, Context

# 0 is the library's default for every knob
CANDIDATES = {
    "rows_per_lane": (0, 2, 4),
    "hist_copies": (0, 32, 8),
    "max_cols": (0, 16384),
    "blocks_per_cu": (0, 12),
    "lut_direct": (0, 1),
    "lut_bytes": (0, 16896),
}


def _cache_path() -> str:
    return os.environ.get("TPCF_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "tpcf", "autotune.json"))


def _device_key(precision: int, nbins: int) -> str:
    try:
        import torch
        name = torch.cuda.get_device_name(0)
        hip = getattr(torch.version, "hip", "") or ""
    except Exception:  # pragma: no cover
        name, hip = "unknown", ""
    # the version part changes whenever the kernels' trade-offs do
    return f"v4|{name}|hip{hip}|prec{precision}|nbins{nbins}"


def _load_cache() -> dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(cache: dict):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def time_sample(ctx: Context, sample, edges, precision: int, repeats: int = 2) -> float:
    """Best summed pair-kernel time (ms) of the sample requests."""
    best = float("inf")
    for _ in range(repeats):
        ctx.kernel_time(reset=True)
        ctx.set_timing(True)
        for kind, a, b, rb, re in sample:
            ctx.count(kind, a, edges, cat_b=b, precision=precision, row_begin=rb, row_end=re)
        ctx.set_timing(False)
        ms, _ = ctx.kernel_time(reset=True)
        best = min(best, ms)
    return best


def autotune(ctx: Context, sample, edges, precision: int = FP32_CHORD, use_cache: bool = True,
             candidates: dict | None = None) -> dict:
    """Pick and apply the fastest launch shape for `sample`, a list of
    (kind, cat_a, cat_b, row_begin, row_end) requests representative of the
    workload.  Returns {"tuning": ..., "timings_ms": ..., "cached": bool}."""
    nbins = len(edges) - 1
    key = _device_key(precision, nbins)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        t = cache[key]["tuning"]
        ctx.set_tuning(**t)
        return {"tuning": t, "timings_ms": cache[key].get("timings_ms", {}), "cached": True}
    cand = candidates or CANDIDATES
    timings = {}
    t0 = time.perf_counter()
    # warm the tables and plans once with the defaults
    ctx.set_tuning()
    time_sample(ctx, sample, edges, precision, repeats=1)

    def measure(t):
        tk = json.dumps(t, sort_keys=True)
        if tk not in timings:
            ctx.set_tuning(**t)
            timings[tk] = round(time_sample(ctx, sample, edges, precision), 3)
        return timings[tk]

    best = {name: 0 for name in cand}
    best_ms = measure(best)
    for name, values in cand.items():
        for v in values:
            if v == best[name]:
                continue
            t = dict(best, **{name: v})
            ms = measure(t)
            if ms < 0.99 * best_ms:       # keep a change only for a clear gain
                best, best_ms = t, ms
    ctx.set_tuning(**best)
    if use_cache:
        cache[key] = {"tuning": best, "timings_ms": timings,
                      "seconds": round(time.perf_counter() - t0, 2)}
        _store_cache(cache)
    return {"tuning": best, "timings_ms": timings, "cached": False}
