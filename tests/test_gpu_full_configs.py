"""GPU parity at the full sizes of the batched and serving workloads (needs
an MI355X).

* Batched: the 64 uneven data catalogs (5e3 .. 5e5 points, each in a
  20 x 20 deg sub-patch) and the 1e6-point random catalog, as the benchmark
  runs them: 129 jobs in one graph-replayed launch.  Every job's totals
  close, three jobs equal their separate launches, and sampled stored row
  blocks of two catalogs (DD and DR) equal the oracle.
* Serving: the first jobs of the job stream at their full sizes (up to 1e6
  points against 2e6 randoms) through submit/wait, each also submitted for a
  sampled row block whose returned histogram equals the oracle.
"""

import numpy as np
import pytest

import oracle
import paper_1204_6630_amd as tp
import synthcat

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tp.Context(0)
    yield c
    c.close()


def _rows(n, size, seed):
    g = np.random.default_rng(seed)
    r0 = int(g.integers(0, max(1, n - size)))
    return r0, min(n, r0 + size)


def _stored(ctx, cid, xyz):
    order = ctx.catalog_order(cid)
    return tuple(c[order] for c in xyz)


def test_batched_64_full_batch(ctx):
    wl = synthcat.batched_64()
    e = wl.edges_deg
    cats = [ctx.upload_catalog(c.ra, c.dec) for c in wl.data]
    r = wl.randoms[0]
    cr = ctx.upload_catalog(r.ra, r.dec)
    try:
        jobs = [(tp.DD, c, -1) for c in cats] + [(tp.DR, c, cr) for c in cats] + [(tp.RR, cr, -1)]
        got = ctx.count_batch(jobs, e, graph=True)
        again = ctx.count_batch(jobs, e, graph=True)          # a replay of the captured graph
        assert np.array_equal(got, again)
        sizes = [c.n for c in wl.data]
        totals = [n * (n - 1) // 2 for n in sizes] + [n * r.n for n in sizes] + [r.n * (r.n - 1) // 2]
        assert [int(h.sum()) for h in got] == totals
        big = int(np.argmax(sizes))
        for k in (0, big, 64 + big):
            kind, a, b = jobs[k]
            assert np.array_equal(got[k], ctx.count(kind, a, e, cat_b=b)), k
        xr = oracle.radec_to_xyz(r.ra, r.dec)
        for c in (big, int(np.argmin(sizes))):
            xs = _stored(ctx, cats[c], oracle.radec_to_xyz(wl.data[c].ra, wl.data[c].dec))
            r0, r1 = _rows(sizes[c], 256, c)
            dd = ctx.count(tp.DD, cats[c], e, row_begin=r0, row_end=r1)
            assert np.array_equal(dd, oracle.count(oracle.DD, xs, e, row_begin=r0, row_end=r1))
            dr = ctx.count(tp.DR, cats[c], e, cat_b=cr, row_begin=r0, row_end=r1)
            assert np.array_equal(dr, oracle.count(oracle.DR, xs, e, b_xyz=xr, row_begin=r0, row_end=r1))
    finally:
        for c in cats:
            ctx.release_catalog(c)
        ctx.release_catalog(cr)


def test_serving_jobs_at_full_size(ctx):
    e = synthcat.log_edges(0.001, 20.0, 30)
    randoms = synthcat.serving_randoms()
    rids = [ctx.upload_catalog(c.ra, c.dec) for c in randoms]
    jobs = synthcat.serving_jobs(n_jobs=6)
    try:
        for job in jobs:
            cat = randoms[job["random"]] if job["kind"] == "RR" else synthcat.serving_catalog(job)
            cid = rids[job["random"]] if job["kind"] == "RR" else ctx.upload_catalog(cat.ra, cat.dec)
            kind = {"DD": tp.DD, "DR": tp.DR, "RR": tp.RR}[job["kind"]]
            other = rids[job["random"]] if kind == tp.DR else -1
            jid = ctx.submit(kind, cid, e, cat_b=other)
            got = ctx.wait(jid, e.size + 1)
            n = cat.n
            nb = randoms[job["random"]].n
            assert int(got.sum()) == (n * nb if kind == tp.DR else n * (n - 1) // 2), job
            xs = _stored(ctx, cid, oracle.radec_to_xyz(cat.ra, cat.dec))
            r0, r1 = _rows(n, 96, job["id"])
            # the job's own result for a row range, through submit and wait
            part = ctx.wait(ctx.submit(kind, cid, e, cat_b=other, row_begin=r0, row_end=r1), e.size + 1)
            if kind == tp.DR:
                xr = oracle.radec_to_xyz(randoms[job["random"]].ra, randoms[job["random"]].dec)
                ref = oracle.count(oracle.DR, xs, e, b_xyz=xr, row_begin=r0, row_end=r1)
            else:
                ref = oracle.count(oracle.DD, xs, e, row_begin=r0, row_end=r1)
            assert np.array_equal(part, ref), job
            if kind != tp.RR:
                ctx.release_catalog(cid)
    finally:
        for c in rids:
            ctx.release_catalog(c)
