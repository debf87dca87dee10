"""tpcf_count_noalloc (needs an MI355X): the entry point that allocates no
device memory, called through the C ABI, against tpcf_count on the same
catalogs: bit-identical histograms on two calls in a row, the second with a
smaller input, for both precisions; the context's device memory does not
grow; errors leave the output untouched."""

import ctypes

import numpy as np
import pytest

import oracle
import paper_1204_6630_amd as tp
import synthcat

pytestmark = pytest.mark.gpu


def _noalloc(ctx, kind, cat_a, edges, cat_b=-1, precision=tp.FP32_CHORD, row_begin=-1, row_end=-1):
    e = np.ascontiguousarray(edges, dtype=np.float64)
    out = np.zeros(e.size + 1, dtype=np.uint64)
    rc = tp.lib().tpcf_count_noalloc(ctx.handle, kind, cat_a, cat_b, e.ctypes.data, e.size - 1, precision,
                                     row_begin, row_end, out.ctypes.data)
    return rc, out


@pytest.fixture(scope="module")
def ctx():
    c = tp.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec", [tp.FP32_CHORD, tp.FP64])
def test_noalloc_equals_count_on_two_calls(ctx, prec):
    wl = synthcat.patch30_1e4()
    d, r = wl.data[0], wl.randoms[0]
    e = wl.edges_deg
    cd = ctx.upload_catalog(d.ra, d.dec)
    cr = ctx.upload_catalog(r.ra, r.dec)
    small = ctx.upload_catalog(d.ra[:1500], d.dec[:1500])
    try:
        used0 = ctx.hbm_usage()[0]
        # first call: the whole DR request
        rc, got = _noalloc(ctx, tp.DR, cd, e, cat_b=cr, precision=prec)
        assert rc == 0, tp.lib().tpcf_last_error(None)
        assert ctx.hbm_usage()[0] == used0          # nothing allocated
        ref = ctx.count(tp.DR, cd, e, cat_b=cr, precision=prec)
        assert np.array_equal(got, ref)
        # second call, smaller: DD of a 1500-point catalog (the work area
        # keeps the first call's contents; what must start at zero is cleared)
        rc, got2 = _noalloc(ctx, tp.DD, small, e, precision=prec)
        assert rc == 0, tp.lib().tpcf_last_error(None)
        ref2 = ctx.count(tp.DD, small, e, precision=prec)
        assert np.array_equal(got2, ref2)
        assert int(got2.sum()) == 1500 * 1499 // 2
        # the oracle agrees too (stored order does not matter for whole catalogs)
        xs = oracle.radec_to_xyz(d.ra[:1500], d.dec[:1500])
        assert np.array_equal(got2, oracle.count(oracle.DD, xs, e))
        # a row range and RR (never taken from the result cache here)
        rc, got3 = _noalloc(ctx, tp.RR, cr, e, precision=prec, row_begin=17, row_end=2100)
        assert rc == 0
        assert np.array_equal(got3, ctx.count(tp.RR, cr, e, precision=prec, row_begin=17, row_end=2100))
    finally:
        for c in (cd, cr, small):
            ctx.release_catalog(c)


def test_noalloc_octant_size_dr_fits(ctx):
    """A request of the large single-GPU workload's size (1e6 x 2e6 DR, here
    on a 3000-row range of the data so it stays quick) plans into the fixed
    work area and equals tpcf_count."""
    wl = synthcat.octant_1e6x2e6()
    d, r = wl.data[0], wl.randoms[0]
    cd = ctx.upload_catalog(d.ra, d.dec)
    cr = ctx.upload_catalog(r.ra, r.dec)
    try:
        rc, got = _noalloc(ctx, tp.DR, cd, wl.edges_deg, cat_b=cr, row_begin=5000, row_end=8000)
        assert rc == 0, tp.lib().tpcf_last_error(None)
        assert np.array_equal(got, ctx.count(tp.DR, cd, wl.edges_deg, cat_b=cr, row_begin=5000, row_end=8000))
        rc, got = _noalloc(ctx, tp.DD, cd, wl.edges_deg, row_begin=0, row_end=2048)
        assert rc == 0, tp.lib().tpcf_last_error(None)
        assert np.array_equal(got, ctx.count(tp.DD, cd, wl.edges_deg, row_begin=0, row_end=2048))
    finally:
        ctx.release_catalog(cd)
        ctx.release_catalog(cr)


def test_noalloc_errors_leave_output_untouched(ctx):
    wl = synthcat.patch30_1e4(scale=0.1)
    d = wl.data[0]
    cd = ctx.upload_catalog(d.ra, d.dec)
    try:
        e = np.ascontiguousarray(wl.edges_deg)
        out = np.full(e.size + 1, 7, dtype=np.uint64)
        L = tp.lib()
        assert L.tpcf_count_noalloc(ctx.handle, 9, cd, -1, e.ctypes.data, e.size - 1, 0, -1, -1,
                                    out.ctypes.data) == -1          # bad kind
        assert L.tpcf_count_noalloc(ctx.handle, tp.DD, 12345, -1, e.ctypes.data, e.size - 1, 0, -1, -1,
                                    out.ctypes.data) == -4          # unknown catalog
        assert L.tpcf_count_noalloc(ctx.handle, tp.DD, cd, -1, e.ctypes.data, e.size - 1, 0, 5, 2,
                                    out.ctypes.data) == -1          # bad row range
        assert L.tpcf_count_noalloc(ctx.handle, tp.DD, cd, -1, e.ctypes.data, e.size - 1, 0, -1, -1,
                                    None) == -1                     # no output
        assert (out == 7).all()
    finally:
        ctx.release_catalog(cd)
