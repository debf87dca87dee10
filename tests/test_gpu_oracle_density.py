"""Oracle parity at the density of the measurement plan (needs an MI355X).

Paper, Section 4: the GPU histograms are judged against the C code on the
CPU.  Here every comparison is with the FP64 oracle, bit for bit:

* octant 1e5 (1e5 clustered + 1e5 uniform points, 30 bins): DD, DR and RR
  in full, both precisions (2e10 pairs of oracle work);
* octant 1e6 x 2e6 (40 bins): 16 seeded blocks of 1000 stored rows per kind
  (DD, DR, RR), both precisions;
* batched (64 uneven catalogs + 1e6 randoms): the batch's own histograms of
  its smallest catalogs in full (DD of the four smallest, DR of the two
  smallest against the randoms), and 16 seeded blocks of 1000 stored rows
  per kind over the catalogs;
* serving: submitted jobs restricted to 1000 stored rows, their own results
  (through submit and wait) against the oracle.

The oracle runs on the host cores (OMP_NUM_THREADS of them at most), a few
minutes in all.
"""

import numpy as np
import pytest

import oracle
import paper_1204_6630_amd as tp
import synthcat

pytestmark = pytest.mark.gpu

PRECS = [tp.FP32_CHORD, tp.FP64]
BLOCK = 1000
NBLOCKS = 16


@pytest.fixture(scope="module")
def ctx():
    c = tp.Context(0)
    yield c
    c.close()


def _xyz(cat):
    return oracle.radec_to_xyz(cat.ra, cat.dec)


def _stored(ctx, cid, xyz):
    order = ctx.catalog_order(cid)
    return tuple(c[order] for c in xyz)


def _blocks(n, seed, count=NBLOCKS, size=BLOCK):
    """`count` seeded, non-overlapping blocks of `size` stored rows."""
    g = np.random.default_rng(seed)
    slots = max(1, n // size)
    picks = np.sort(g.choice(slots, size=min(count, slots), replace=False))
    return [(int(s) * size, int(min(n, (int(s) + 1) * size))) for s in picks]


def test_octant_1e5_in_full_against_the_oracle(ctx):
    wl = synthcat.octant_1e5()
    d, r = wl.data[0], wl.randoms[0]
    e = wl.edges_deg
    xd, xr = _xyz(d), _xyz(r)
    ref = (oracle.count(oracle.DD, xd, e), oracle.count(oracle.DR, xd, e, b_xyz=xr),
           oracle.count(oracle.RR, xr, e))
    cd = ctx.upload_catalog(d.ra, d.dec)
    cr = ctx.upload_catalog(r.ra, r.dec)
    try:
        for prec in PRECS:
            got = (ctx.count(tp.DD, cd, e, precision=prec), ctx.count(tp.DR, cd, e, cat_b=cr, precision=prec),
                   ctx.count(tp.RR, cr, e, precision=prec))
            for kind, g, f in zip(("DD", "DR", "RR"), got, ref):
                assert np.array_equal(g, f), (kind, prec)
    finally:
        ctx.release_catalog(cd)
        ctx.release_catalog(cr)


def test_octant_1e6x2e6_sixteen_row_blocks_per_kind(ctx):
    wl = synthcat.octant_1e6x2e6()
    d, r = wl.data[0], wl.randoms[0]
    e = wl.edges_deg
    cd = ctx.upload_catalog(d.ra, d.dec)
    cr = ctx.upload_catalog(r.ra, r.dec)
    try:
        xd, xr = _stored(ctx, cd, _xyz(d)), _stored(ctx, cr, _xyz(r))
        cases = [("DD", tp.DD, oracle.DD, cd, -1, xd, None, _blocks(d.n, 301)),
                 ("DR", tp.DR, oracle.DR, cd, cr, xd, xr, _blocks(d.n, 302)),
                 ("RR", tp.RR, oracle.RR, cr, -1, xr, None, _blocks(r.n, 303))]
        for name, kind, okind, a, b, xa, xb, blocks in cases:
            assert len(blocks) == NBLOCKS
            for rb, re in blocks:
                ref = oracle.count(okind, xa, e, b_xyz=xb, row_begin=rb, row_end=re)
                for prec in PRECS:
                    got = ctx.count(kind, a, e, cat_b=b, precision=prec, row_begin=rb, row_end=re)
                    assert np.array_equal(got, ref), (name, rb, prec)
    finally:
        ctx.release_catalog(cd)
        ctx.release_catalog(cr)


def test_batched_64_own_results_and_row_blocks(ctx):
    wl = synthcat.batched_64()
    e = wl.edges_deg
    cats = [ctx.upload_catalog(c.ra, c.dec) for c in wl.data]
    r = wl.randoms[0]
    cr = ctx.upload_catalog(r.ra, r.dec)
    try:
        jobs = [(tp.DD, c, -1) for c in cats] + [(tp.DR, c, cr) for c in cats] + [(tp.RR, cr, -1)]
        got = ctx.count_batch(jobs, e, graph=True)
        sizes = np.array([c.n for c in wl.data])
        by_size = np.argsort(sizes)
        xr = _xyz(r)
        # the batch's own histograms of its smallest catalogs, in full
        for c in by_size[:4]:
            assert np.array_equal(got[c], oracle.count(oracle.DD, _xyz(wl.data[c]), e)), ("DD", c)
        for c in by_size[:2]:
            assert np.array_equal(got[64 + c], oracle.count(oracle.DR, _xyz(wl.data[c]), e, b_xyz=xr)), ("DR", c)
        # 16 seeded blocks of 1000 stored rows per kind: DD and DR in the
        # catalogs (one block each in 16 catalogs drawn by size rank), RR in
        # the randoms
        g = np.random.default_rng(304)
        picks = g.choice(64, size=NBLOCKS, replace=False)
        xs_r = _stored(ctx, cr, xr)
        for c in picks:
            xs = _stored(ctx, cats[c], _xyz(wl.data[c]))
            (rb, re), = _blocks(int(sizes[c]), 305 + int(c), count=1)
            dd = ctx.count(tp.DD, cats[c], e, row_begin=rb, row_end=re)
            assert np.array_equal(dd, oracle.count(oracle.DD, xs, e, row_begin=rb, row_end=re)), ("DD", c)
            dr = ctx.count(tp.DR, cats[c], e, cat_b=cr, row_begin=rb, row_end=re)
            assert np.array_equal(dr, oracle.count(oracle.DR, xs, e, b_xyz=xr, row_begin=rb,
                                                   row_end=re)), ("DR", c)
        for rb, re in _blocks(r.n, 306):
            # DD kind on the random catalog: the same pairs as RR, never cached
            rr = ctx.count(tp.DD, cr, e, row_begin=rb, row_end=re)
            assert np.array_equal(rr, oracle.count(oracle.RR, xs_r, e, row_begin=rb, row_end=re)), ("RR", rb)
    finally:
        for c in cats:
            ctx.release_catalog(c)
        ctx.release_catalog(cr)


def test_serving_jobs_own_results_on_row_blocks(ctx):
    """Jobs of the serving stream submitted with a 1000-row range: the result
    each job hands back (submit, then wait) equals the oracle."""
    e = synthcat.log_edges(0.001, 20.0, 30)
    randoms = synthcat.serving_randoms()
    rids = [ctx.upload_catalog(c.ra, c.dec) for c in randoms]
    xr = [_stored(ctx, rid, _xyz(c)) for rid, c in zip(rids, randoms)]
    spec = synthcat.serving_jobs(n_jobs=10)
    try:
        pending = []
        for job in spec:
            kind = {"DD": tp.DD, "DR": tp.DR, "RR": tp.RR}[job["kind"]]
            if kind == tp.RR:
                cid, cat, xs = rids[job["random"]], randoms[job["random"]], xr[job["random"]]
            else:
                cat = synthcat.serving_catalog(job)
                cid = ctx.upload_catalog(cat.ra, cat.dec)
                xs = _stored(ctx, cid, _xyz(cat))
            (rb, re), = _blocks(cat.n, 400 + job["id"], count=1)
            other = rids[job["random"]] if kind == tp.DR else -1
            jid = ctx.submit(kind, cid, e, cat_b=other, row_begin=rb, row_end=re)
            pending.append((job, kind, cid, xs, rb, re, jid))
        for job, kind, cid, xs, rb, re, jid in pending:
            got = ctx.wait(jid, e.size + 1)
            okind = {tp.DD: oracle.DD, tp.DR: oracle.DR, tp.RR: oracle.RR}[kind]
            xb = xr[job["random"]] if kind == tp.DR else None
            ref = oracle.count(okind, xs, e, b_xyz=xb, row_begin=rb, row_end=re)
            assert np.array_equal(got, ref), job
        for job, kind, cid, *_ in pending:
            if kind != tp.RR:
                ctx.release_catalog(cid)
    finally:
        for c in rids:
            ctx.release_catalog(c)
