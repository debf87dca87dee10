"""Autotuner for the pair kernels' launch shape.

Candidates: rows held per lane (2 or 4), LDS histogram copies per wavefront
(32 or 16), the largest column range of a work unit, and the grid size.  Each
candidate is timed on a sample of the caller's workload (a block of rows
against the full column catalog) with the library's HIP-event kernel timer;
the fastest is applied to the context and cached on disk, keyed by device,
HIP runtime, precision and bin count.  Counts never depend on the choice.
"""

from __future__ import annotations

import itertools
import json
import os
import time

from . import FP32_CHORD, Context

CANDIDATES = {
    "rows_per_lane": (2, 4),
    "hist_copies": (32, 16),
    "max_cols": (4096, 16384),
    "blocks_per_cu": (0, 12),
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
    return f"{name}|hip{hip}|prec{precision}|nbins{nbins}"


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
    names = list(cand)
    timings = {}
    t0 = time.perf_counter()
    # warm the tables and plans once with the defaults
    ctx.set_tuning()
    time_sample(ctx, sample, edges, precision, repeats=1)
    best, best_ms = None, float("inf")
    for values in itertools.product(*(cand[n] for n in names)):
        t = dict(zip(names, values))
        ctx.set_tuning(**t)
        ms = time_sample(ctx, sample, edges, precision)
        timings[json.dumps(t, sort_keys=True)] = round(ms, 3)
        if ms < best_ms:
            best, best_ms = t, ms
    ctx.set_tuning(**best)
    if use_cache:
        cache[key] = {"tuning": best, "timings_ms": timings,
                      "seconds": round(time.perf_counter() - t0, 2)}
        _store_cache(cache)
    return {"tuning": best, "timings_ms": timings, "cached": False}
