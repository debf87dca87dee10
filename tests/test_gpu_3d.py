"""GPU parity of the 3-D distance counts (needs an MI355X).

3-D catalogs bin pairs by Euclidean distance (the spatial correlation
function xi(r)).  Counts are integers: bit-exact equality with the oracle's
``count3d`` for both 3-D precisions, on an integer lattice whose distances
fall exactly on edges (ties re-decided with the exact rule), clustered boxes
in full, ragged sizes around the tile sizes, row ranges, coordinates far
from the origin (a wide FP32 band), batches and jobs; at the full box size
(1e6 x 2e6) the three precisions agree and sampled row blocks equal the oracle.
"""

import numpy as np
import pytest

import oracle
import paper_1204_6630_amd as tp
import rounding_probes as rp
import synthcat

pytestmark = pytest.mark.gpu

PRECS3 = [tp.FP32_CHORD, tp.FP64]
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


def _lattice(n, offset=0.0):
    g = np.arange(n, dtype=np.float64) + offset
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


@pytest.mark.parametrize("prec", PRECS3)
@pytest.mark.parametrize("offset", [0.0, 4096.0])
def test_lattice_ties_on_edges(ctx, prec, offset):
    """12^3 integer lattice: edges 1, 2, 3, 5, 6 equal lattice distances, so
    many pairs sit exactly on an edge (upper bin); the offset moves the
    points far from the origin, which widens the FP32 band."""
    pts = _lattice(12, offset)
    edges = np.array([0.5, 1.0, 1.5, 2.0, 3.0, 4.5, 5.0, 6.0, 9.5])
    cid = ctx.upload_catalog_3d(*pts)
    try:
        got = ctx.count(tp.DD, cid, edges, precision=prec)
        ref = _cached(("lattice", offset), lambda: oracle.count3d(oracle.DD, pts, edges))
        assert np.array_equal(got, ref)
    finally:
        ctx.release_catalog(cid)


@pytest.mark.parametrize("prec", PRECS3)
def test_rounding_order_probes_3d(ctx, prec):
    """The exact FP64 rule of every 3-D path is (dx^2 + dy^2) + dz^2 of the
    rounded differences, unfused and left to right: probe pairs where fused or
    reordered evaluations give another distance bin, expected histograms from
    exact rational arithmetic (DR over all cross pairs, DD over the union)."""
    def build():
        a, b, edges = rp.box_probes()
        cross = [(i, j) for i in range(a.shape[0]) for j in range(b.shape[0])]
        u = np.concatenate([a, b])
        upper = [(i, j) for i in range(u.shape[0]) for j in range(i + 1, u.shape[0])]
        return (a, b, edges, u, rp.expected_box_hist(a, b, edges, cross),
                rp.expected_box_hist(u, u, edges, upper))
    a, b, edges, u, exp_dr, exp_dd = _cached("probes3d", build)
    ca = ctx.upload_catalog_3d(*a.T.copy())
    cb = ctx.upload_catalog_3d(*b.T.copy())
    cu = ctx.upload_catalog_3d(*u.T.copy())
    try:
        assert np.array_equal(ctx.count(tp.DR, ca, edges, cat_b=cb, precision=prec), exp_dr)
        assert np.array_equal(ctx.count(tp.DD, cu, edges, precision=prec), exp_dd)
    finally:
        for c in (ca, cb, cu):
            ctx.release_catalog(c)


@pytest.fixture(scope="module")
def box(ctx):
    wl = synthcat.box_1e6x2e6(scale=0.01)          # 1e4 data, 2e4 randoms, box 1000
    cd = ctx.upload_catalog_3d(*wl.data.xyz())
    cr = ctx.upload_catalog_3d(*wl.randoms.xyz())
    ref = _cached("box", lambda: {
        "DD": oracle.count3d(oracle.DD, wl.data.xyz(), wl.edges),
        "DR": oracle.count3d(oracle.DR, wl.data.xyz(), wl.edges, b_xyz=wl.randoms.xyz()),
        "RR": oracle.count3d(oracle.RR, wl.randoms.xyz(), wl.edges),
    })
    return wl, cd, cr, ref


@pytest.mark.parametrize("prec", PRECS3)
def test_box_full_bit_exact(ctx, box, prec):
    wl, cd, cr, ref = box
    assert np.array_equal(ctx.count(tp.DD, cd, wl.edges, precision=prec), ref["DD"])
    assert np.array_equal(ctx.count(tp.DR, cd, wl.edges, cat_b=cr, precision=prec), ref["DR"])
    assert np.array_equal(ctx.count(tp.RR, cr, wl.edges, precision=prec), ref["RR"])
    xi = tp.landy_szalay(ref["DD"], ref["DR"], ref["RR"], wl.data.n, wl.randoms.n)
    assert np.array_equal(np.isnan(xi), ref["RR"][1:-1] == 0)     # NaN exactly where RR is empty


@pytest.mark.parametrize("prec", PRECS3)
def test_box_row_ranges(ctx, box, prec):
    wl, cd, cr, ref = box
    n = wl.data.n
    parts = [(0, 1), (1, 1000), (1000, 1001), (1001, n)]
    dd = sum(ctx.count(tp.DD, cd, wl.edges, precision=prec, row_begin=a, row_end=b) for a, b in parts)
    dr = sum(ctx.count(tp.DR, cd, wl.edges, cat_b=cr, precision=prec, row_begin=a, row_end=b)
             for a, b in parts)
    assert np.array_equal(dd, ref["DD"]) and np.array_equal(dr, ref["DR"])
    # a single stored row block against the oracle on the same rows
    order = ctx.catalog_order(cd)
    xs = tuple(c[order] for c in wl.data.xyz())
    got = ctx.count(tp.DD, cd, wl.edges, precision=prec, row_begin=2000, row_end=2777)
    assert np.array_equal(got, oracle.count3d(oracle.DD, xs, wl.edges, row_begin=2000, row_end=2777))


@pytest.mark.parametrize("prec", PRECS3)
@pytest.mark.parametrize("na,nb", [(1, 1), (2, 63), (65, 257), (1023, 1025), (1025, 4097), (4097, 3)])
def test_ragged_sizes(ctx, prec, na, nb):
    g = synthcat.rng_for(31, na * 7 + nb)
    a = synthcat.box_clustered(na, max(1, na // 40), 1.5, 80.0, g, origin=-40.0)
    b = synthcat.box_uniform(nb, 80.0, g, origin=-40.0)
    edges = synthcat.log_edges(0.05, 60.0, 21)
    ca = ctx.upload_catalog_3d(*a.xyz())
    cb = ctx.upload_catalog_3d(*b.xyz())
    try:
        assert np.array_equal(ctx.count(tp.DD, ca, edges, precision=prec),
                              oracle.count3d(oracle.DD, a.xyz(), edges))
        assert np.array_equal(ctx.count(tp.DR, ca, edges, cat_b=cb, precision=prec),
                              oracle.count3d(oracle.DR, a.xyz(), edges, b_xyz=b.xyz()))
    finally:
        ctx.release_catalog(ca)
        ctx.release_catalog(cb)


def test_edge_zero_and_coincident_points(ctx):
    """Coincident points are at distance 0: at or past an edge of 0, below
    any positive edge."""
    x = np.array([1.0, 1.0, 1.0, 2.0, 5.0])
    y = np.array([2.0, 2.0, 2.0, 2.0, 2.0])
    z = np.zeros(5)
    cid = ctx.upload_catalog_3d(x, y, z)
    try:
        for edges in ([0.0, 1.0, 3.0, 10.0], [0.5, 1.0, 3.0, 10.0]):
            e = np.array(edges)
            ref = oracle.count3d(oracle.DD, (x, y, z), e)
            for prec in PRECS3:
                assert np.array_equal(ctx.count(tp.DD, cid, e, precision=prec), ref)
    finally:
        ctx.release_catalog(cid)


def test_batch_and_jobs_with_3d_catalogs(ctx, box):
    wl, cd, cr, ref = box
    jobs = [(tp.DD, cd, -1), (tp.DR, cd, cr), (tp.RR, cr, -1)]
    for graph in (False, True):
        out = ctx.count_batch(jobs, wl.edges, precision=tp.FP32_CHORD, graph=graph)
        assert np.array_equal(out[0], ref["DD"]) and np.array_equal(out[1], ref["DR"])
        assert np.array_equal(out[2], ref["RR"])
    j = ctx.submit(tp.DR, cd, wl.edges, cat_b=cr, precision=tp.FP64)
    assert np.array_equal(ctx.wait(j, wl.edges.size + 1), ref["DR"])


def test_3d_errors(ctx, box):
    wl, cd, cr, _ = box
    sky = ctx.upload_catalog(np.array([1.0, 2.0]), np.array([3.0, 4.0]))
    try:
        with pytest.raises(tp.TpcfError):      # a sky catalog against a 3-D one
            ctx.count(tp.DR, cd, wl.edges, cat_b=sky)
        with pytest.raises(tp.TpcfError):      # mixed batch
            ctx.count_batch([(tp.DD, cd, -1), (tp.DD, sky, -1)], wl.edges)
        with pytest.raises(tp.TpcfError):      # edges must increase
            ctx.count(tp.DD, cd, np.array([2.0, 1.0]))
        with pytest.raises(tp.TpcfError):      # coordinates beyond 2^50
            ctx.upload_catalog_3d(np.array([2.0 ** 51]), np.zeros(1), np.zeros(1))
        with pytest.raises(tp.TpcfError):
            ctx.upload_catalog_3d(np.array([np.nan]), np.zeros(1), np.zeros(1))
        # angular edges above 180 are fine as distances
        e = np.array([1.0, 200.0, 400.0])
        assert int(ctx.count(tp.DD, cd, e).sum()) == wl.data.n * (wl.data.n - 1) // 2
    finally:
        ctx.release_catalog(sky)


def _sample_blocks(n, nblocks, size, seed):
    g = np.random.default_rng(seed)
    starts = np.sort(g.choice(n - size, size=nblocks, replace=False))
    return [(int(s), int(s) + size) for s in starts]


def test_full_box_fp32_equals_fp64_and_sampled_rows_equal_oracle(ctx):
    """1e6 data x 2e6 randoms in a box of side 1000: DD, DR, RR agree between
    the precisions; sampled stored row blocks agree with the oracle."""
    wl = synthcat.box_1e6x2e6()
    cd = ctx.upload_catalog_3d(*wl.data.xyz())
    cr = ctx.upload_catalog_3d(*wl.randoms.xyz())
    try:
        for kind, a, b in ((tp.DD, cd, -1), (tp.DR, cd, cr), (tp.RR, cr, -1)):
            f32 = ctx.count(kind, a, wl.edges, cat_b=b, precision=tp.FP32_CHORD)
            f64 = ctx.count(kind, a, wl.edges, cat_b=b, precision=tp.FP64)
            assert np.array_equal(f32, f64)
        order = ctx.catalog_order(cd)
        xs = tuple(c[order] for c in wl.data.xyz())
        for r0, r1 in _sample_blocks(wl.data.n, 2, 192, 5):
            got = ctx.count(tp.DD, cd, wl.edges, row_begin=r0, row_end=r1)
            assert np.array_equal(got, oracle.count3d(oracle.DD, xs, wl.edges, row_begin=r0, row_end=r1))
            got = ctx.count(tp.DR, cd, wl.edges, cat_b=cr, row_begin=r0, row_end=r1)
            ref = oracle.count3d(oracle.DR, xs, wl.edges, b_xyz=wl.randoms.xyz(), row_begin=r0, row_end=r1)
            assert np.array_equal(got, ref)
    finally:
        ctx.release_catalog(cd)
        ctx.release_catalog(cr)


@pytest.mark.parametrize("prec", PRECS3)
def test_3d_pruning_keeps_counts_exact(ctx, box, prec):
    """Exact tile pruning with bounding balls: the box in full equals the
    oracle; dense blobs with wide bins (whole blocks inside one bin, and
    beyond the last edge) equal the oracle with pruned blocks counted."""
    wl, cd, cr, ref = box
    old = ctx.get_tuning()
    ctx.set_tuning(prune=1)
    try:
        ctx.stats(reset=True)
        assert np.array_equal(ctx.count(tp.DD, cd, wl.edges, precision=prec), ref["DD"])
        assert np.array_equal(ctx.count(tp.DR, cd, wl.edges, cat_b=cr, precision=prec), ref["DR"])
        assert np.array_equal(ctx.count(tp.RR, cr, wl.edges, precision=prec), ref["RR"])
        g = synthcat.rng_for(31, 77)
        blobs = synthcat.box_clustered(12000, 12, 0.8, 400.0, g)
        e = np.array([0.0, 3.0, 40.0, 150.0, 300.0])
        cb = ctx.upload_catalog_3d(*blobs.xyz())
        try:
            ctx.stats(reset=True)
            got = ctx.count(tp.DD, cb, e, precision=prec)
            st = ctx.stats(reset=True)
            assert np.array_equal(got, _cached("blobs", lambda: oracle.count3d(oracle.DD, blobs.xyz(), e)))
            assert st.pruned_pairs > 0
        finally:
            ctx.release_catalog(cb)
    finally:
        ctx.set_tuning(**old)


def test_3d_pruning_at_full_size_equals_brute_force(ctx):
    wl = synthcat.box_1e6x2e6()
    cd = ctx.upload_catalog_3d(*wl.data.xyz())
    cr = ctx.upload_catalog_3d(*wl.randoms.xyz())
    try:
        brute = [ctx.count(tp.DD, cd, wl.edges), ctx.count(tp.DR, cd, wl.edges, cat_b=cr)]
        ctx.set_tuning(prune=1)
        ctx.stats(reset=True)
        pruned = [ctx.count(tp.DD, cd, wl.edges), ctx.count(tp.DR, cd, wl.edges, cat_b=cr)]
        st = ctx.stats(reset=True)
        assert all(np.array_equal(a, b) for a, b in zip(brute, pruned))
        assert st.pruned_pairs > st.pairs // 2
    finally:
        ctx.set_tuning()
        ctx.release_catalog(cd)
        ctx.release_catalog(cr)
