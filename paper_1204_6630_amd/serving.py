"""Request loop for pair-count jobs: continuous batching over libtpcf.

Jobs (DD on the job's own catalog, DR of the job's catalog against a resident
random catalog, RR of a resident random catalog) arrive over time.  The loop

  * admits arrived jobs in arrival order while a slot is free and the job's
    device memory fits the HBM budget (catalog upload, then ``tpcf_submit``);
    a job that does not fit waits until completed jobs release memory;
  * polls in-flight jobs, which run concurrently on the library's streams,
    records each result and its latency (arrival to result on the host);
  * releases finished jobs' catalogs in batches: when nothing is in flight,
    when admission needs the memory, or past ``max_deferred_bytes``.  Freeing
    device memory waits for the whole device, so a release at every
    completion would stall the loop behind the longest running job;
  * serves repeated RR requests from the library's result cache, and an RR
    request for a random catalog whose RR count is still running waits for
    that count and takes its result instead of launching a second one.

The device side is the C library; this module only sequences calls.  The
backend is injectable so the admission logic can be exercised without a GPU.
"""

from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import DD, DR, FP32_CHORD, RR, TpcfError

KINDS = {"DD": DD, "DR": DR, "RR": RR}
BYTES_PER_POINT = 36          # FP64 + FP32 structure-of-arrays copies
BYTES_PER_JOB = 1 << 20       # unit plan and tables, generous


@dataclass
class Job:
    id: int
    kind: str                 # "DD", "DR" or "RR"
    arrival: float            # seconds after the start of the run
    ra: np.ndarray | None = None
    dec: np.ndarray | None = None
    random: int = 0           # index of the resident random catalog
    n: int = 0

    def pairs(self, n_random: int) -> int:
        if self.kind == "DD":
            return self.n * (self.n - 1) // 2
        if self.kind == "DR":
            return self.n * n_random
        return n_random * (n_random - 1) // 2


@dataclass
class Report:
    results: dict = field(default_factory=dict)      # job id -> histogram
    latency: dict = field(default_factory=dict)      # job id -> seconds
    admitted_at: dict = field(default_factory=dict)
    max_inflight: int = 0
    max_bytes: int = 0
    makespan: float = 0.0
    pairs: int = 0

    def percentile(self, q: float) -> float:
        v = np.array(sorted(self.latency.values()))
        return float(np.percentile(v, q)) if v.size else float("nan")


class LibraryBackend:
    """The libtpcf context behind the loop."""

    def __init__(self, ctx, edges_deg, precision=FP32_CHORD):
        self.ctx = ctx
        self.edges = np.ascontiguousarray(edges_deg, dtype=np.float64)
        self.precision = precision
        self.nslots = self.edges.size + 1

    def usage(self):
        return self.ctx.hbm_usage()

    def upload(self, job: Job) -> int:
        return self.ctx.upload_catalog(job.ra, job.dec)

    def submit(self, kind: int, cat_a: int, cat_b: int) -> int:
        return self.ctx.submit(kind, cat_a, self.edges, cat_b=cat_b, precision=self.precision)

    def poll(self, jid: int):
        return self.ctx.poll(jid, self.nslots)

    def release(self, cat: int):
        self.ctx.release_catalog(cat)


class Server:
    def __init__(self, backend, randoms: list, n_random: int, max_inflight: int = 8,
                 clock=time.perf_counter, idle=lambda: time.sleep(0.0002),
                 max_deferred_bytes: int = 1 << 30):
        self.b = backend
        self.randoms = randoms          # resident random catalog ids
        self.n_random = n_random
        self.max_inflight = max_inflight
        self.clock = clock
        self.idle = idle
        self.max_deferred_bytes = max_deferred_bytes

    def bytes_needed(self, job: Job) -> int:
        own = job.n * BYTES_PER_POINT if job.kind != "RR" else 0
        return own + BYTES_PER_JOB

    def run(self, jobs: list) -> Report:
        rep = Report()
        pending = collections.deque(sorted(jobs, key=lambda j: j.arrival))
        waiting = collections.deque()
        inflight = {}                  # job handle -> (job, own catalog or None)
        deferred = []                  # catalogs of finished jobs, not yet released
        rr_leader = {}                 # random index -> handle of its running RR count
        followers = collections.defaultdict(list)   # handle -> RR jobs waiting on it
        deferred_bytes = 0

        def release_deferred():
            nonlocal deferred_bytes
            for c in deferred:
                self.b.release(c)
            deferred.clear()
            deferred_bytes = 0

        t0 = self.clock()
        while pending or waiting or inflight:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            progressed = False
            # admission, in arrival order
            while waiting:
                job = waiting[0]
                if job.kind == "RR" and job.random in rr_leader:
                    # needs no slot: it waits on the running count
                    waiting.popleft()
                    followers[rr_leader[job.random]].append(job)
                    rep.admitted_at[job.id] = self.clock() - t0
                    progressed = True
                    continue
                if len(inflight) >= self.max_inflight:
                    break
                used, budget = self.b.usage()
                if budget and used + self.bytes_needed(job) > budget and inflight:
                    if deferred:
                        release_deferred()
                        continue    # check again with that memory back
                    break           # wait for memory to be released
                cat = None
                try:
                    if job.kind != "RR":
                        cat = self.b.upload(job)
                    rnd = self.randoms[job.random]
                    if job.kind == "DD":
                        h = self.b.submit(DD, cat, -1)
                    elif job.kind == "DR":
                        h = self.b.submit(DR, cat, rnd)
                    else:
                        h = self.b.submit(RR, rnd, -1)
                except TpcfError as e:
                    if cat is not None:
                        self.b.release(cat)
                    if e.code == -5 and inflight:
                        if deferred:
                            release_deferred()
                            continue
                        break       # over budget: retry once something completes
                    raise
                waiting.popleft()
                inflight[h] = (job, cat)
                if job.kind == "RR":
                    rr_leader[job.random] = h
                rep.admitted_at[job.id] = self.clock() - t0
                rep.max_inflight = max(rep.max_inflight, len(inflight))
                rep.max_bytes = max(rep.max_bytes, self.b.usage()[0])
                progressed = True
            # completions
            for h in list(inflight):
                res = self.b.poll(h)
                if res is None:
                    continue
                job, cat = inflight.pop(h)
                t = self.clock() - t0
                rep.results[job.id] = res
                rep.latency[job.id] = t - job.arrival
                rep.pairs += job.pairs(self.n_random)
                if job.kind == "RR" and rr_leader.get(job.random) == h:
                    del rr_leader[job.random]
                for f in followers.pop(h, []):
                    rep.results[f.id] = res.copy()
                    rep.latency[f.id] = t - f.arrival
                    rep.pairs += f.pairs(self.n_random)
                if cat is not None:
                    deferred.append(cat)
                    deferred_bytes += self.bytes_needed(job)
                progressed = True
            if deferred and (not inflight or deferred_bytes > self.max_deferred_bytes):
                release_deferred()
            if not progressed:
                self.idle()
        rep.makespan = self.clock() - t0
        release_deferred()
        return rep


def poisson_arrivals(n: int, rate: float, rng: np.random.Generator) -> np.ndarray:
    """Arrival times of a Poisson process of the given rate (per second)."""
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
