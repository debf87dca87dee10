"""CPU tests of the request loop's scheduling (fake device, fake clock).

The fake backend mimics the library's contract: uploads count against an HBM
budget and fail with TPCF_E_BUDGET beyond it, submitted jobs finish after a
time proportional to their pairs, poll returns None until then.
"""

import numpy as np
import pytest

import paper_1204_6630_amd as tp
from paper_1204_6630_amd.serving import BYTES_PER_POINT, Job, Server, poisson_arrivals


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance(self, dt=1e-3):
        self.t += dt


class FakeBackend:
    def __init__(self, clock, budget, rate=1e9, n_random=1000):
        self.clock = clock
        self.budget = budget
        self.used = 10_000
        self.rate = rate
        self.n_random = n_random
        self.cats = {}
        self.jobs = {}
        self.next = 1
        self.uploads = 0
        self.peak = self.used

    def usage(self):
        return self.used, self.budget

    def upload(self, job):
        need = job.n * BYTES_PER_POINT
        if self.budget and self.used + need > self.budget:
            raise tp.TpcfError(-5, "over budget")
        self.used += need
        self.peak = max(self.peak, self.used)
        cid = self.next
        self.next += 1
        self.cats[cid] = (need, job.n)
        self.uploads += 1
        return cid

    def submit(self, kind, a, b):
        if kind == tp.DD:
            pairs = self.cats[a][1] ** 2 // 2
        elif kind == tp.DR:
            pairs = self.cats[a][1] * self.n_random
        else:
            pairs = self.n_random ** 2 // 2
        jid = self.next
        self.next += 1
        self.jobs[jid] = (self.clock() + pairs / self.rate, kind)
        return jid

    def poll(self, jid):
        done_at, kind = self.jobs[jid]
        if self.clock() >= done_at:
            del self.jobs[jid]
            return np.array([kind], dtype=np.uint64)
        return None

    def release(self, cat):
        self.used -= self.cats.pop(cat)[0]


def _jobs(n, seed=0, rate=50.0):
    g = np.random.default_rng(seed)
    arr = poisson_arrivals(n, rate, g)
    out = []
    for k in range(n):
        u = g.uniform()
        kind = "DD" if u < 0.4 else ("DR" if u < 0.8 else "RR")
        size = int(np.exp(g.uniform(np.log(1e3), np.log(1e5))))
        out.append(Job(id=k, kind=kind, arrival=float(arr[k]), n=size if kind != "RR" else 0,
                       random=int(g.integers(0, 3))))
    return out


def _run(jobs, budget, max_inflight=4):
    clock = FakeClock()
    be = FakeBackend(clock, budget)
    srv = Server(be, randoms=[101, 102, 103], n_random=1000, max_inflight=max_inflight,
                 clock=clock, idle=clock.advance)
    return srv.run(jobs), be


def test_every_job_completes_in_arrival_order_admission():
    jobs = _jobs(200)
    rep, be = _run(jobs, budget=0)
    assert set(rep.results) == {j.id for j in jobs}
    order = [j.id for j in sorted(jobs, key=lambda j: j.arrival)]
    adm = [rep.admitted_at[i] for i in order]
    assert all(a <= b for a, b in zip(adm, adm[1:]))
    assert all(rep.latency[j.id] >= 0 for j in jobs)
    assert all(rep.admitted_at[j.id] >= j.arrival - 1e-12 for j in jobs)
    # results belong to their jobs
    for j in jobs:
        assert int(rep.results[j.id][0]) == tp.__dict__[j.kind]


def test_budget_is_never_exceeded_and_memory_returns():
    jobs = _jobs(150, seed=1)
    budget = 10_000 + 3 * 100_000 * BYTES_PER_POINT
    rep, be = _run(jobs, budget=budget)
    assert set(rep.results) == {j.id for j in jobs}
    assert be.peak <= budget
    assert rep.max_bytes <= budget
    assert be.used == 10_000


def test_slot_limit_and_rr_needs_no_upload():
    jobs = _jobs(120, seed=2)
    rep, be = _run(jobs, budget=0, max_inflight=3)
    assert rep.max_inflight <= 3
    assert be.uploads == sum(1 for j in jobs if j.kind != "RR")


def test_a_job_larger_than_the_budget_alone_raises():
    jobs = [Job(id=0, kind="DD", arrival=0.0, n=10**6)]
    with pytest.raises(tp.TpcfError):
        _run(jobs, budget=1_000_000)


def test_poisson_arrivals_rate():
    g = np.random.default_rng(5)
    a = poisson_arrivals(20000, 40.0, g)
    assert np.all(np.diff(a) > 0)
    assert abs(a[-1] / 20000 - 1 / 40.0) < 0.05 / 40.0 * 5


class ReleaseWatch(FakeBackend):
    """Records, at each release, how many jobs are still running and whether
    the loop was blocked on memory (an upload would not have fit)."""

    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        self.release_log = []

    def release(self, cat):
        self.release_log.append(len(self.jobs))
        super().release(cat)


def test_catalogs_are_released_in_batches_when_the_device_is_idle():
    # no budget: a release (a device-wide wait on the GPU) only happens
    # once nothing is in flight, or past the deferred-bytes cap
    jobs = _jobs(150, seed=3, rate=400.0)
    clock = FakeClock()
    be = ReleaseWatch(clock, budget=0)
    srv = Server(be, randoms=[101, 102, 103], n_random=1000, max_inflight=4,
                 clock=clock, idle=clock.advance)
    rep = srv.run(jobs)
    assert set(rep.results) == {j.id for j in jobs}
    assert be.used == 10_000 and not be.cats
    assert len(be.release_log) == sum(1 for j in jobs if j.kind != "RR")
    assert all(n == 0 for n in be.release_log)
    # a small cap forces releases while jobs run; everything still completes
    clock = FakeClock()
    be = ReleaseWatch(clock, budget=0)
    srv = Server(be, randoms=[101, 102, 103], n_random=1000, max_inflight=4,
                 clock=clock, idle=clock.advance, max_deferred_bytes=1)
    rep = srv.run(jobs)
    assert set(rep.results) == {j.id for j in jobs}
    assert be.used == 10_000
    assert any(n > 0 for n in be.release_log)


def test_deferred_catalogs_are_released_when_admission_needs_memory():
    # a tight budget: admission frees the deferred catalogs rather than wait
    jobs = _jobs(150, seed=4, rate=400.0)
    budget = 10_000 + 3 * 100_000 * BYTES_PER_POINT
    clock = FakeClock()
    be = ReleaseWatch(clock, budget=budget)
    srv = Server(be, randoms=[101, 102, 103], n_random=1000, max_inflight=4,
                 clock=clock, idle=clock.advance)
    rep = srv.run(jobs)
    assert set(rep.results) == {j.id for j in jobs}
    assert be.peak <= budget and be.used == 10_000
    assert any(n > 0 for n in be.release_log)


class RRWatch(FakeBackend):
    """Flags a second RR count of one random catalog while the first runs."""

    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        self.rr_running = {}        # job id -> random catalog id
        self.rr_submits = 0
        self.overlap = False

    def submit(self, kind, a, b):
        jid = super().submit(kind, a, b)
        if kind == tp.RR:
            self.rr_submits += 1
            self.overlap |= a in self.rr_running.values()
            self.rr_running[jid] = a
        return jid

    def poll(self, jid):
        res = super().poll(jid)
        if res is not None:
            self.rr_running.pop(jid, None)
        return res


def test_rr_requests_share_a_running_rr_count():
    # RR requests 1 ms apart over three random catalogs (an RR count takes
    # 25 ms here), with small DR jobs between them: later requests arrive
    # while their random catalog's RR count runs and take its result
    jobs = []
    for k in range(90):
        if k % 3 == 2:
            jobs.append(Job(id=k, kind="DR", arrival=k * 1e-3, n=20, random=k % 3))
        else:
            jobs.append(Job(id=k, kind="RR", arrival=k * 1e-3, random=(k // 3) % 3))
    clock = FakeClock()
    be = RRWatch(clock, budget=0, rate=2e7)
    srv = Server(be, randoms=[101, 102, 103], n_random=1000, max_inflight=4,
                 clock=clock, idle=clock.advance)
    rep = srv.run(jobs)
    assert set(rep.results) == {j.id for j in jobs}
    assert not be.overlap
    n_rr = sum(1 for j in jobs if j.kind == "RR")
    assert be.rr_submits < n_rr // 4
    for j in jobs:
        assert int(rep.results[j.id][0]) == tp.__dict__[j.kind]
        assert rep.latency[j.id] >= 0
