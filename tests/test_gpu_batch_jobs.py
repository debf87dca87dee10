"""GPU tests of batched launches and asynchronous jobs (needs an MI355X).

* a batch of uneven catalogs counted in one launch equals the same counts
  made one by one, and the oracle on the small ones;
* a hipGraph-captured batch, replayed several times with eager work and
  synchronisations in between, returns the eager result on every replay;
* submitted jobs overlapping on four streams return the same counts alone and
  in the mix; RR results come from the cache on resubmission; a cancelled job
  reports cancellation while the other jobs stay exact;
* the HBM budget refuses allocations beyond it and the accounting returns to
  its start when catalogs are released.
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


@pytest.fixture(scope="module")
def small_batch(ctx):
    """Eight catalogs of uneven size in 20 x 20 deg sub-patches (the batched
    workload's recipe, scaled down) and one uniform random catalog."""
    wl = synthcat.batched_64(n_catalogs=8, scale=0.02)
    cats = [ctx.upload_catalog(c.ra, c.dec) for c in wl.data]
    r = wl.randoms[0]
    cr = ctx.upload_catalog(r.ra, r.dec)
    return wl, cats, cr


@pytest.mark.parametrize("prec", [tp.FP32_CHORD, tp.FP64])
def test_batch_equals_single_counts_and_oracle(ctx, small_batch, prec):
    wl, cats, cr = small_batch
    e = wl.edges_deg
    jobs = [(tp.DD, c, -1) for c in cats] + [(tp.DR, c, cr) for c in cats] + [(tp.RR, cr, -1)]
    got = ctx.count_batch(jobs, e, precision=prec)
    for k, (kind, a, b) in enumerate(jobs):
        single = ctx.count(kind, a, e, cat_b=b, precision=prec)
        assert np.array_equal(got[k], single), k
    # the oracle on the smallest catalogs
    sizes = [c.n for c in wl.data]
    for k in np.argsort(sizes)[:2]:
        x = oracle.radec_to_xyz(wl.data[k].ra, wl.data[k].dec)
        assert np.array_equal(got[k], oracle.count(oracle.DD, x, e))


def test_batch_graph_replays_match_eager(ctx, small_batch):
    wl, cats, cr = small_batch
    e = wl.edges_deg
    jobs = [(tp.DD, c, -1) for c in cats] + [(tp.DR, c, cr) for c in cats]
    eager = ctx.count_batch(jobs, e)
    for rep in range(4):
        g = ctx.count_batch(jobs, e, graph=True)
        assert np.array_equal(g, eager), rep
        # eager work and a synchronisation between replays
        one = ctx.count(tp.DR, cats[0], e, cat_b=cr)
        assert np.array_equal(one, eager[len(cats)])
        ctx.synchronize()


def test_batch_rejects_mixed_edges(ctx, small_batch):
    wl, cats, cr = small_batch
    e = wl.edges_deg
    arr = (tp.JobDesc * 2)()
    e2 = e.copy()
    e2[-1] = 25.0
    arr[0] = tp.Context._desc(tp.DD, cats[0], e)
    arr[1] = tp.Context._desc(tp.DD, cats[1], e2)
    out = np.zeros((2, e.size + 1), dtype=np.uint64)
    rc = tp.lib().tpcf_count_batch(ctx.handle, arr, 2, 0, out.ctypes.data)
    assert rc == -1


def test_jobs_alone_and_in_the_mix(ctx, small_batch):
    wl, cats, cr = small_batch
    e = wl.edges_deg
    ns = e.size + 1
    reqs = [(tp.DD, c, -1) for c in cats] + [(tp.DR, c, cr) for c in cats]
    alone = [ctx.count(k, a, e, cat_b=b) for k, a, b in reqs]
    ids = [ctx.submit(k, a, e, cat_b=b) for k, a, b in reqs]
    results = {}
    while len(results) < len(ids):
        for i, jid in enumerate(ids):
            if i in results:
                continue
            h = ctx.poll(jid, ns)
            if h is not None:
                results[i] = h
    for i in range(len(ids)):
        assert np.array_equal(results[i], alone[i]), i


def test_rr_result_cache(ctx, small_batch):
    wl, cats, cr = small_batch
    e = wl.edges_deg
    ns = e.size + 1
    first = ctx.wait(ctx.submit(tp.RR, cr, e), ns)
    jid = ctx.submit(tp.RR, cr, e)
    h = ctx.poll(jid, ns)          # served at submit: done on the first poll
    assert h is not None and np.array_equal(h, first)
    assert np.array_equal(ctx.count(tp.RR, cr, e), first)


def test_cancel_leaves_other_jobs_exact(ctx):
    g = synthcat.rng_for(96, 0)
    big = ctx.upload_catalog(*synthcat.uniform_patch(200_000, synthcat.OCTANT, g))
    small = ctx.upload_catalog(*synthcat.uniform_patch(3000, synthcat.PATCH_30, g))
    e = synthcat.log_edges(0.01, 10.0, 20)
    ns = e.size + 1
    ref = ctx.count(tp.DD, small, e)
    victim = ctx.submit(tp.DD, big, e)
    other = ctx.submit(tp.DD, small, e)
    ctx.cancel(victim)
    with pytest.raises(tp.TpcfError) as ei:
        ctx.wait(victim, ns)
    assert ei.value.code == -6
    assert np.array_equal(ctx.wait(other, ns), ref)
    with pytest.raises(tp.TpcfError) as ei:
        ctx.poll(victim, ns)       # retired
    assert ei.value.code == -4
    ctx.release_catalog(big)
    ctx.release_catalog(small)


def test_release_refused_while_job_unretired(ctx):
    g = synthcat.rng_for(96, 1)
    c = ctx.upload_catalog(*synthcat.uniform_patch(2000, synthcat.PATCH_30, g))
    e = synthcat.log_edges(0.01, 10.0, 20)
    jid = ctx.submit(tp.DD, c, e)
    with pytest.raises(tp.TpcfError):
        ctx.release_catalog(c)
    ctx.wait(jid, e.size + 1)
    ctx.release_catalog(c)


def test_hbm_budget_and_accounting():
    with tp.Context(0) as c:
        used0, _ = c.hbm_usage()
        g = synthcat.rng_for(96, 2)
        ra, dec = synthcat.uniform_patch(100_000, synthcat.OCTANT, g)
        cid = c.upload_catalog(ra, dec)
        used1, _ = c.hbm_usage()
        assert used1 - used0 >= 100_000 * 36
        c.set_hbm_budget(used1 + 1_000_000)
        with pytest.raises(tp.TpcfError) as ei:
            c.upload_catalog(ra, dec)
        assert ei.value.code == -5
        assert c.hbm_usage()[0] == used1
        c.release_catalog(cid)
        assert c.hbm_usage()[0] == used0
        c.set_hbm_budget(0)
