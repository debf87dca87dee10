"""GPU parity of the jackknife region counts (needs an MI355X).

tpcf_count_regions against the oracle's per-region counts, bit-exact, for
every precision: a clustered patch cut into a grid of regions; ragged label
sets with empty regions, one-point regions and region sizes off every tile
and 16-row boundary; pruning on; and at the full octant size (1e6 x 2e6) the
property that the counts with one region deleted equal plain counts of the
reduced catalogs.  The jackknife built on the GPU counts matches the oracle's
recount-based jackknife.
"""

import numpy as np
import pytest

import oracle
import paper_1204_6630_amd as tp
import synthcat

pytestmark = pytest.mark.gpu

PRECS = [tp.FP32_CHORD, tp.FP64]
_cache = {}


@pytest.fixture(scope="module")
def ctx():
    c = tp.Context(0)
    yield c
    c.close()


def _cached(key, fn):
    if key not in _cache:
        _cache[key] = fn()
    return _cache[key]


@pytest.fixture(scope="module")
def grid_case(ctx):
    """patch30_1e4's catalogs (1e4 + 1e4 on a 30x30 deg patch), 4 x 3 regions."""
    wl = synthcat.patch30_1e4()
    d, r = wl.data[0], wl.randoms[0]
    fp = synthcat.PATCH_30
    nreg = 12
    rd = synthcat.grid_regions(d.ra, d.dec, fp, 4, 3)
    rr = synthcat.grid_regions(r.ra, r.dec, fp, 4, 3)
    cd = ctx.upload_catalog_regions(d.ra, d.dec, rd, nreg)
    cr = ctx.upload_catalog_regions(r.ra, r.dec, rr, nreg)
    xd = oracle.radec_to_xyz(d.ra, d.dec)
    xr = oracle.radec_to_xyz(r.ra, r.dec)
    ref = _cached("grid", lambda: {
        "DD": oracle.count_regions(oracle.DD, xd, rd, wl.edges_deg, nreg),
        "DR": oracle.count_regions(oracle.DR, xd, rd, wl.edges_deg, nreg, b_xyz=xr, b_region=rr),
        "RR": oracle.count_regions(oracle.RR, xr, rr, wl.edges_deg, nreg),
    })
    return wl, cd, cr, rd, rr, nreg, xd, xr, ref


def _check(got, ref):
    assert np.array_equal(got[0], ref[0])
    assert got[1].shape == ref[1].shape
    assert np.array_equal(got[1], ref[1])


@pytest.mark.parametrize("prec", PRECS)
def test_grid_regions_bit_exact(ctx, grid_case, prec):
    wl, cd, cr, rd, rr, nreg, _, _, ref = grid_case
    assert np.array_equal(ctx.catalog_regions(cd), np.bincount(rd, minlength=nreg))
    _check(ctx.count_regions(tp.DD, cd, wl.edges_deg, precision=prec), ref["DD"])
    _check(ctx.count_regions(tp.DR, cd, wl.edges_deg, cat_b=cr, precision=prec), ref["DR"])
    _check(ctx.count_regions(tp.RR, cr, wl.edges_deg, precision=prec), ref["RR"])
    # the total equals the plain count of the same catalog
    assert np.array_equal(ctx.count(tp.DD, cd, wl.edges_deg, precision=prec), ref["DD"][0])


def test_stored_order_groups_regions(ctx, grid_case):
    _, cd, _, rd, _, _, _, _, _ = grid_case
    lab = rd[ctx.catalog_order(cd)]
    assert np.all(np.diff(lab) >= 0)


def test_jackknife_from_gpu_counts_equals_oracle_recount(ctx, grid_case):
    wl, cd, cr, rd, rr, nreg, xd, xr, _ = grid_case
    dd = ctx.count_regions(tp.DD, cd, wl.edges_deg)
    dr = ctx.count_regions(tp.DR, cd, wl.edges_deg, cat_b=cr)
    rrc = ctx.count_regions(tp.RR, cr, wl.edges_deg)
    nd_reg, nr_reg = ctx.catalog_regions(cd), ctx.catalog_regions(cr)
    s, m, c = tp.jackknife(dd[0], dd[1], dr[0], dr[1], rrc[0], rrc[1],
                           wl.data[0].n, nd_reg, wl.randoms[0].n, nr_reg)
    so, mo, co = _cached("jk", lambda: oracle.jackknife(xd, rd, xr, rr, wl.edges_deg, nreg))
    assert np.array_equal(np.isnan(s), np.isnan(so))
    np.testing.assert_allclose(s, so, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(m, mo, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(c, co, rtol=1e-10, atol=1e-18)


def _ragged_labels(n, nreg, seed):
    """Skewed labels: two empty regions, one region of one point, the rest of
    random sizes (none a multiple of the tile sizes by design)."""
    g = synthcat.rng_for(95, seed)
    w = g.uniform(0.2, 1.0, size=nreg)
    w[1] = 0.0
    w[nreg - 2] = 0.0
    lab = g.choice(nreg, size=n, p=w / w.sum()).astype(np.int32)
    lab[lab == 3] = 0
    lab[n // 2] = 3     # region 3 holds exactly one point
    return lab


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("na,nb,nreg", [(1537, 2049, 9), (1300, 1, 7), (35, 4100, 11)])
def test_ragged_regions_bit_exact(ctx, prec, na, nb, nreg):
    g = synthcat.rng_for(95, 100 + na)
    fp = (0.0, 12.0, 0.0, 12.0)
    ra, dec = synthcat.uniform_patch(na, fp, g)
    rb_ra, rb_dec = synthcat.uniform_patch(nb, fp, g)
    la = _ragged_labels(na, nreg, na)
    lb = _ragged_labels(nb, nreg, nb) if nb > 1 else np.zeros(nb, np.int32)
    e = synthcat.log_edges(0.02, 8.0, 17)
    ca = ctx.upload_catalog_regions(ra, dec, la, nreg)
    cb = ctx.upload_catalog_regions(rb_ra, rb_dec, lb, nreg)
    xa = oracle.radec_to_xyz(ra, dec)
    xb = oracle.radec_to_xyz(rb_ra, rb_dec)
    try:
        ref_dd = _cached(("rdd", na, nreg), lambda: oracle.count_regions(oracle.DD, xa, la, e, nreg))
        ref_dr = _cached(("rdr", na, nb, nreg),
                         lambda: oracle.count_regions(oracle.DR, xa, la, e, nreg, b_xyz=xb, b_region=lb))
        _check(ctx.count_regions(tp.DD, ca, e, precision=prec), ref_dd)
        _check(ctx.count_regions(tp.DR, ca, e, cat_b=cb, precision=prec), ref_dr)
    finally:
        ctx.release_catalog(ca)
        ctx.release_catalog(cb)


@pytest.mark.parametrize("prec", PRECS)
def test_region_counts_with_pruning(ctx, grid_case, prec):
    wl, cd, cr, _, _, _, _, _, ref = grid_case
    old = ctx.get_tuning()
    ctx.set_tuning(prune=1)
    try:
        _check(ctx.count_regions(tp.DD, cd, wl.edges_deg, precision=prec), ref["DD"])
        _check(ctx.count_regions(tp.DR, cd, wl.edges_deg, cat_b=cr, precision=prec), ref["DR"])
    finally:
        ctx.set_tuning(**old)


def test_region_errors(ctx, grid_case):
    wl, cd, cr, _, _, nreg, _, _, _ = grid_case
    d = wl.data[0]
    plain = ctx.upload_catalog(d.ra[:100], d.dec[:100])
    other = ctx.upload_catalog_regions(d.ra[:100], d.dec[:100], np.zeros(100, np.int32), nreg + 1)
    try:
        with pytest.raises(tp.TpcfError):      # unlabelled catalog
            ctx.count_regions(tp.DD, plain, wl.edges_deg)
        with pytest.raises(tp.TpcfError):      # different region counts
            ctx.count_regions(tp.DR, cd, wl.edges_deg, cat_b=other)
        with pytest.raises(tp.TpcfError):      # label out of range
            ctx.upload_catalog_regions(d.ra[:10], d.dec[:10], np.full(10, nreg, np.int32), nreg)
        with pytest.raises(tp.TpcfError):      # negative label
            ctx.upload_catalog_regions(d.ra[:10], d.dec[:10], np.full(10, -1, np.int32), nreg)
        with pytest.raises(tp.TpcfError):      # too many regions
            ctx.upload_catalog_regions(d.ra[:10], d.dec[:10], np.zeros(10, np.int32), tp.MAX_REGIONS + 1)
        assert len(ctx.catalog_regions(plain)) == 0
    finally:
        ctx.release_catalog(plain)
        ctx.release_catalog(other)


def test_full_octant_deleted_region_equals_reduced_catalog_counts(ctx):
    """1e6 data x 2e6 randoms over the octant, 8 x 8 regions: for two regions,
    total - touch[r] equals the plain count of the catalogs without region r
    (the plain path is itself checked against the oracle)."""
    wl = synthcat.octant_1e6x2e6()
    d, r = wl.data[0], wl.randoms[0]
    fp = synthcat.OCTANT
    nreg = 64
    rd = synthcat.grid_regions(d.ra, d.dec, fp, 8, 8)
    rr = synthcat.grid_regions(r.ra, r.dec, fp, 8, 8)
    cd = ctx.upload_catalog_regions(d.ra, d.dec, rd, nreg)
    cr = ctx.upload_catalog_regions(r.ra, r.dec, rr, nreg)
    try:
        dd_t, dd_touch = ctx.count_regions(tp.DD, cd, wl.edges_deg)
        dr_t, dr_touch = ctx.count_regions(tp.DR, cd, wl.edges_deg, cat_b=cr)
        assert np.array_equal(dd_t, ctx.count(tp.DD, cd, wl.edges_deg))
        # every pair touches one or two regions
        assert np.all(dd_touch.sum(axis=0) >= dd_t) and np.all(dd_touch.sum(axis=0) <= 2 * dd_t)
        for k in (0, 37):
            kd, kr = rd != k, rr != k
            sd = ctx.upload_catalog(d.ra[kd], d.dec[kd])
            sr = ctx.upload_catalog(r.ra[kr], r.dec[kr])
            try:
                assert np.array_equal(dd_t - dd_touch[k], ctx.count(tp.DD, sd, wl.edges_deg))
                assert np.array_equal(dr_t - dr_touch[k], ctx.count(tp.DR, sd, wl.edges_deg, cat_b=sr))
            finally:
                ctx.release_catalog(sd)
                ctx.release_catalog(sr)
        # the FP64 path agrees with the FP32 path at full size
        fdd = ctx.count_regions(tp.DD, cd, wl.edges_deg, precision=tp.FP64)
        assert np.array_equal(fdd[0], dd_t) and np.array_equal(fdd[1], dd_touch)
    finally:
        ctx.release_catalog(cd)
        ctx.release_catalog(cr)


@pytest.mark.parametrize("prec", PRECS)
def test_3d_regions_and_jackknife(ctx, prec):
    """3-D catalogs (a clustered box and uniform randoms) cut into 3 x 3 x 1
    slabs: totals and touch rows bit-exact against the oracle for every
    precision, and the jackknife of xi(r) equal to the oracle's recount."""
    g = synthcat.rng_for(98, 0)
    a = synthcat.box_clustered(2500, 60, 2.0, 120.0, g)
    b = synthcat.box_uniform(3000, 120.0, g)
    nreg = 9

    def labels(box):
        ix = np.minimum((box.x // 40).astype(np.int32), 2)
        iy = np.minimum((box.y // 40).astype(np.int32), 2)
        return (iy * 3 + ix).astype(np.int32)

    la, lb = labels(a), labels(b)
    e = synthcat.log_edges(0.5, 50.0, 15)
    ca = ctx.upload_catalog_3d_regions(*a.xyz(), la, nreg)
    cb = ctx.upload_catalog_3d_regions(*b.xyz(), lb, nreg)
    try:
        ref_dd = _cached("3d_dd", lambda: oracle.count_regions(oracle.DD, a.xyz(), la, e, nreg, metric=1))
        ref_dr = _cached("3d_dr", lambda: oracle.count_regions(oracle.DR, a.xyz(), la, e, nreg,
                                                               b_xyz=b.xyz(), b_region=lb, metric=1))
        ref_rr = _cached("3d_rr", lambda: oracle.count_regions(oracle.RR, b.xyz(), lb, e, nreg, metric=1))
        dd = ctx.count_regions(tp.DD, ca, e, precision=prec)
        dr = ctx.count_regions(tp.DR, ca, e, cat_b=cb, precision=prec)
        rr = ctx.count_regions(tp.RR, cb, e, precision=prec)
        _check(dd, ref_dd)
        _check(dr, ref_dr)
        _check(rr, ref_rr)
        s, m, c = tp.jackknife(dd[0], dd[1], dr[0], dr[1], rr[0], rr[1], a.n, ctx.catalog_regions(ca),
                               b.n, ctx.catalog_regions(cb))
        so, mo, co = _cached("3d_jk", lambda: oracle.jackknife(a.xyz(), la, b.xyz(), lb, e, nreg, metric=1))
        assert np.array_equal(np.isnan(s), np.isnan(so))
        np.testing.assert_allclose(s, so, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(c, co, rtol=1e-10, atol=1e-18)
    finally:
        ctx.release_catalog(ca)
        ctx.release_catalog(cb)
