"""GPU parity: libtpcf.so against the CPU oracle (needs an MI355X).

Counts are integers, so the bar is bit-exact equality of every slot, for
both precision modes.  Sizes: the small configuration in full, ragged sizes
around the tile sizes (64 lanes x 4 rows x 4 wavefronts = 1024 rows per
unit), the larger configurations in full on the GPU with sampled row blocks
checked against the oracle, plus exact-dot probes on every edge threshold.
"""

import math

import numpy as np
import pytest

import oracle
import paper_1204_6630_amd as tp
import rounding_probes as rp
import synthcat

pytestmark = pytest.mark.gpu

PRECS = [tp.FP32_CHORD, tp.FP64]
_cache = {}


@pytest.fixture(scope="module")
def ctx():
    c = tp.Context(0)
    yield c
    c.close()


def _xyz(cat):
    return oracle.radec_to_xyz(cat.ra, cat.dec)


def _workload(cfg):
    if cfg not in _cache:
        _cache[cfg] = synthcat.WORKLOADS[cfg]()
    return _cache[cfg]


def _stored(ctx, cid, xyz):
    """The catalog's coordinates in the library's stored row order."""
    order = ctx.catalog_order(cid)
    return tuple(c[order] for c in xyz)


def _oracle(key, fn):
    if key not in _cache:
        _cache[key] = fn()
    return _cache[key]


@pytest.fixture(scope="module")
def patch(ctx):
    wl = _workload("patch30_1e4")
    d, r = wl.data[0], wl.randoms[0]
    cd = ctx.upload_catalog(d.ra, d.dec)
    cr = ctx.upload_catalog(r.ra, r.dec)
    xd, xr = _xyz(d), _xyz(r)
    ref = {
        "DD": oracle.count(oracle.DD, xd, wl.edges_deg),
        "DR": oracle.count(oracle.DR, xd, wl.edges_deg, b_xyz=xr),
        "RR": oracle.count(oracle.RR, xr, wl.edges_deg),
    }
    return wl, cd, cr, ref


@pytest.mark.parametrize("prec", PRECS)
def test_patch_full_bit_exact(ctx, patch, prec):
    wl, cd, cr, ref = patch
    dd = ctx.count(tp.DD, cd, wl.edges_deg, precision=prec)
    dr = ctx.count(tp.DR, cd, wl.edges_deg, cat_b=cr, precision=prec)
    rr = ctx.count(tp.RR, cr, wl.edges_deg, precision=prec)
    assert np.array_equal(dd, ref["DD"])
    assert np.array_equal(dr, ref["DR"])
    assert np.array_equal(rr, ref["RR"])
    nd, nr = wl.data[0].n, wl.randoms[0].n
    for form in (0, 1):
        w = tp.landy_szalay(dd, dr, rr, nd, nr, form)
        wref = oracle.landy_szalay(ref["DD"][1:-1], ref["DR"][1:-1], ref["RR"][1:-1], nd, nr, form)
        fin = np.isfinite(wref)
        assert np.array_equal(np.isnan(w), np.isnan(wref))
        assert np.all(np.abs(w[fin] - wref[fin]) <= 1e-12 * np.maximum(1.0, np.abs(wref[fin])))


@pytest.mark.parametrize("prec", PRECS)
def test_ragged_sizes_and_tails(ctx, prec):
    g = synthcat.rng_for(95, 0)
    edges = np.concatenate([[0.0], synthcat.log_edges(0.002, 5.0, 17)])
    ra, dec = synthcat.clustered(6000, 30, 0.4, synthcat.PATCH_30, g)
    xyz = oracle.radec_to_xyz(ra, dec)
    cid = ctx.upload_catalog(ra, dec)
    for n in (0, 1, 2, 3, 63, 64, 65, 255, 256, 257, 1023, 1024, 1025, 2049, 4097, 6000):
        sub = ctx.upload_catalog(ra[:n], dec[:n])
        got = ctx.count(tp.DD, sub, edges, precision=prec)
        ref = oracle.count(oracle.DD, tuple(c[:n] for c in xyz), edges)
        assert np.array_equal(got, ref), n
        got = ctx.count(tp.DR, sub, edges, cat_b=cid, precision=prec)
        ref = oracle.count(oracle.DR, tuple(c[:n] for c in xyz), edges, b_xyz=xyz)
        assert np.array_equal(got, ref), n
        ctx.release_catalog(sub)
    ctx.release_catalog(cid)


@pytest.mark.parametrize("prec", PRECS)
def test_row_ranges(ctx, patch, prec):
    wl, cd, cr, _ = patch
    xd = _stored(ctx, cd, _xyz(wl.data[0]))
    xr = _xyz(wl.randoms[0])
    n = wl.data[0].n
    for rb, re in ((0, 1), (17, 1500), (1023, 1025), (n - 1, n), (5, 5), (0, n)):
        got = ctx.count(tp.DD, cd, wl.edges_deg, precision=prec, row_begin=rb, row_end=re)
        ref = oracle.count(oracle.DD, xd, wl.edges_deg, row_begin=rb, row_end=re)
        assert np.array_equal(got, ref), (rb, re)
        got = ctx.count(tp.DR, cd, wl.edges_deg, cat_b=cr, precision=prec, row_begin=rb, row_end=re)
        ref = oracle.count(oracle.DR, xd, wl.edges_deg, b_xyz=xr, row_begin=rb, row_end=re)
        assert np.array_equal(got, ref), (rb, re)


def _next(d, n):
    for _ in range(abs(n)):
        d = np.nextafter(d, np.inf if n > 0 else -np.inf)
    return d


@pytest.mark.parametrize("prec", PRECS)
def test_exact_dot_probes_on_every_threshold(ctx, prec):
    """P1: i = (1,0,0) and j = (d, sqrt(1 - d^2), 0) have FP64 dot exactly d;
    d runs over D_k and its neighbours for every edge, so ties at the edge and
    the D_k translation are exercised directly."""
    for edges in (synthcat.log_edges(0.01, 10.0, 20), synthcat.log_edges(0.0005, 30.0, 40),
                  np.array([0.0, 0.5, 60.0, 90.0, 120.0, 179.0])):
        D, _, _ = tp.compile_edges(edges)
        ds = []
        for Dk in D:
            if np.isfinite(Dk):
                ds += [_next(Dk, s) for s in (-3, -2, -1, 0, 1, 2, 3)]
        ds = np.array([x for x in ds if -1.0 <= x <= 1.0])
        a = (np.ones(1), np.zeros(1), np.zeros(1))
        b = (ds, np.sqrt(1.0 - ds * ds), np.zeros_like(ds))
        ca = ctx.upload_catalog_xyz(*a)
        cb = ctx.upload_catalog_xyz(*b)
        got = ctx.count(tp.DR, ca, edges, cat_b=cb, precision=prec)
        ref = oracle.count(oracle.DR, a, edges, b_xyz=b)
        assert np.array_equal(got, ref)
        # the same probes one per row (j > i via DD on the concatenation)
        u = tuple(np.concatenate([p, q]) for p, q in zip(a, b))
        cu = ctx.upload_catalog_xyz(*u)
        us = _stored(ctx, cu, u)
        row = int(np.nonzero(ctx.catalog_order(cu) == 0)[0][0])   # where (1,0,0) is stored
        got = ctx.count(tp.DD, cu, edges, precision=prec, row_begin=row, row_end=row + 1)
        ref = oracle.count(oracle.DD, us, edges, row_begin=row, row_end=row + 1)
        assert np.array_equal(got, ref)
        got = ctx.count(tp.DD, cu, edges, precision=prec)
        assert np.array_equal(got, oracle.count(oracle.DD, u, edges))
        for c in (ca, cb, cu):
            ctx.release_catalog(c)


def _probe_sets():
    if "probes" not in _cache:
        a, b, edges = rp.sky_probes()
        cross = [(i, j) for i in range(a.shape[0]) for j in range(b.shape[0])]
        u = np.concatenate([a, b])
        upper = [(i, j) for i in range(u.shape[0]) for j in range(i + 1, u.shape[0])]
        _cache["probes"] = (a, b, edges, u, rp.expected_sky_hist(a, b, edges, cross),
                            rp.expected_sky_hist(u, u, edges, upper))
    return _cache["probes"]


@pytest.mark.parametrize("prec", PRECS)
def test_rounding_order_probes(ctx, prec):
    """The exact FP64 rule of every path is the unfused, left-to-right dot
    product: probe pairs where fused or reordered evaluations land in another
    bin (edges placed between them), with expected histograms from exact
    rational arithmetic rounded after each operation, for DR (all cross pairs)
    and DD (the union, auto-pairs with the masked diagonal)."""
    a, b, edges, u, exp_dr, exp_dd = _probe_sets()
    ca = ctx.upload_catalog_xyz(*a.T.copy())
    cb = ctx.upload_catalog_xyz(*b.T.copy())
    cu = ctx.upload_catalog_xyz(*u.T.copy())
    try:
        assert np.array_equal(ctx.count(tp.DR, ca, edges, cat_b=cb, precision=prec), exp_dr)
        assert np.array_equal(ctx.count(tp.DD, cu, edges, precision=prec), exp_dd)
    finally:
        for c in (ca, cb, cu):
            ctx.release_catalog(c)


@pytest.mark.parametrize("prec", PRECS)
def test_duplicates_and_antipodes(ctx, prec):
    g = synthcat.rng_for(95, 1)
    p = np.stack(oracle.radec_to_xyz(*synthcat.uniform_sphere(700, g)), axis=1)
    pts = np.concatenate([p, p[:300], -p[:200]])
    xyz = tuple(pts.T.copy())
    for edges in (np.array([0.01, 1.0, 179.0]), np.array([0.0, 1e-4, 90.0, 180.0])):
        cid = ctx.upload_catalog_xyz(*xyz)
        got = ctx.count(tp.DD, cid, edges, precision=prec)
        ref = oracle.count(oracle.DD, xyz, edges)
        assert np.array_equal(got, ref)
        got = ctx.count(tp.DR, cid, edges, cat_b=cid, precision=prec)
        ref = oracle.count(oracle.DR, xyz, edges, b_xyz=xyz)
        assert np.array_equal(got, ref)
        ctx.release_catalog(cid)


@pytest.mark.parametrize("cfg", ["octant_1e5", "octant_1e6x2e6"])
def test_full_size_fp32_equals_fp64_and_pruning(ctx, cfg):
    """Whole catalogs at full size: the FP32 path equals the FP64 path and the
    pruned count, slot for slot, with closed totals (the oracle checks of these
    workloads are in test_gpu_oracle_density.py)."""
    wl = _workload(cfg)
    d, r = wl.data[0], wl.randoms[0]
    cd = ctx.upload_catalog(d.ra, d.dec)
    cr = ctx.upload_catalog(r.ra, r.dec)
    e = wl.edges_deg
    full = {}
    for prec in PRECS:
        dd = ctx.count(tp.DD, cd, e, precision=prec)
        dr = ctx.count(tp.DR, cd, e, cat_b=cr, precision=prec)
        rr = ctx.count(tp.RR, cr, e, precision=prec)
        assert int(dd.sum()) == d.n * (d.n - 1) // 2
        assert int(dr.sum()) == d.n * r.n
        assert int(rr.sum()) == r.n * (r.n - 1) // 2
        full[prec] = (dd, dr, rr)
    for p in PRECS[1:]:
        for a, b in zip(full[PRECS[0]], full[p]):
            assert np.array_equal(a, b), p
    try:    # exact tile pruning on the full catalogs
        ctx.set_tuning(prune=1)
        pruned = (ctx.count(tp.DD, cd, e), ctx.count(tp.DR, cd, e, cat_b=cr), ctx.count(tp.RR, cr, e))
    finally:
        ctx.set_tuning()
    for a, b in zip(full[PRECS[0]], pruned):
        assert np.array_equal(a, b)
    ctx.release_catalog(cd)
    ctx.release_catalog(cr)


def test_union_invariant_on_gpu(ctx, patch):
    """DD(A u B) = DD(A) + DD(B) + DR(A, B) and DR(A, B) = DR(B, A)."""
    wl, cd, cr, _ = patch
    d, r = wl.data[0], wl.randoms[0]
    cu = ctx.upload_catalog(np.concatenate([d.ra, r.ra]), np.concatenate([d.dec, r.dec]))
    e = wl.edges_deg
    for prec in PRECS:
        ddu = ctx.count(tp.DD, cu, e, precision=prec)
        parts = (ctx.count(tp.DD, cd, e, precision=prec) + ctx.count(tp.RR, cr, e, precision=prec)
                 + ctx.count(tp.DR, cd, e, cat_b=cr, precision=prec))
        assert np.array_equal(ddu, parts)
        assert np.array_equal(ctx.count(tp.DR, cd, e, cat_b=cr, precision=prec),
                              ctx.count(tp.DR, cr, e, cat_b=cd, precision=prec))
    ctx.release_catalog(cu)


def test_attach_torch_tensor_and_async(ctx, patch):
    import torch
    wl, cd, cr, ref = patch
    x = np.stack(_xyz(wl.data[0]))
    t = torch.from_numpy(x).to("cuda:0").contiguous()
    ca = ctx.attach_catalog(t)
    for prec in PRECS:
        got = ctx.count(tp.DD, ca, wl.edges_deg, precision=prec)
        assert np.array_equal(got, ref["DD"])
    out = torch.zeros(wl.edges_deg.size + 1, dtype=torch.int64, device="cuda:0")
    torch.cuda.synchronize()    # the fill runs on torch's stream, the count on the library's
    ctx.count_async(tp.DR, ca, wl.edges_deg, out.data_ptr(), cat_b=cr)
    ctx.synchronize()
    assert np.array_equal(out.cpu().numpy().astype(np.uint64), ref["DR"])
    ctx.release_catalog(ca)
    # the caller's own FP32 copies (round to nearest) are taken as they are
    t32 = t.to(torch.float32).contiguous()
    cb = ctx.attach_catalog(t, t32)
    for prec in PRECS:
        assert np.array_equal(ctx.count(tp.DD, cb, wl.edges_deg, precision=prec), ref["DD"])
    ctx.release_catalog(cb)
    # copies that are not the rounded FP64 values are refused
    bad = t32.clone()
    bad[0, 5] = torch.nextafter(bad[0, 5], torch.tensor(2.0, dtype=torch.float32, device="cuda:0"))
    with pytest.raises(tp.TpcfError):
        ctx.attach_catalog(t, bad)
    del t, t32, bad


def test_timing_and_stats(ctx, patch):
    wl, cd, cr, _ = patch
    ctx.stats(reset=True)
    ctx.kernel_time(reset=True)
    ctx.set_timing(True)
    ctx.count(tp.DR, cd, wl.edges_deg, cat_b=cr, precision=tp.FP32_CHORD)
    ms, n = ctx.kernel_time(reset=True)
    ctx.set_timing(False)
    st = ctx.stats(reset=True)
    pairs, flagged, exact, rare = st.pairs, st.flagged, st.exact, st.rare_steps
    beyond, one_slot, two_slot = st.beyond_steps, st.one_slot_steps, st.two_slot_steps
    assert n == 1 and ms > 0
    assert pairs == wl.data[0].n * wl.randoms[0].n
    assert exact <= flagged <= pairs
    assert rare <= flagged
    assert flagged < 0.2 * pairs
    # a 30 x 30 deg patch against edges up to 10 deg: many wavefront steps
    # (4 rows x 2 columns per lane) lie wholly beyond the last edge
    assert 0 < beyond * 512 < pairs
    assert (beyond + one_slot + two_slot + rare) * 512 <= pairs


def test_dot_product_path_settles_large_angle_steps(ctx, patch):
    """FP32 angular launches decide most steps of the 30 x 30 deg patch (edges
    up to 10 deg) from the dot product alone; the steps that formed the chord
    are counted apart; every count equals the oracle's.  A dense 0.3 x 0.3 deg
    patch binned to 0.1 deg keeps its steps on the chord (small angles, where
    the dot product cannot resolve the bins), with the same counts as the
    oracle."""
    wl, cd, cr, ref = patch
    steps = lambda st: st.pairs / 1024.0     # 4 rows x 4 columns per lane
    ctx.stats(reset=True)
    assert np.array_equal(ctx.count(tp.DR, cd, wl.edges_deg, cat_b=cr, precision=tp.FP32_CHORD), ref["DR"])
    st = ctx.stats(reset=True)
    assert st.beyond_steps > 0 and st.two_slot_steps > 0
    assert 0 < st.chord_steps < 0.5 * steps(st)
    # FP64 launches never take it
    assert np.array_equal(ctx.count(tp.DR, cd, wl.edges_deg, cat_b=cr, precision=tp.FP64), ref["DR"])
    assert ctx.stats(reset=True).chord_steps == 0
    g = synthcat.rng_for(97, 1)
    box = (10.0, 10.3, 20.0, 20.3)
    d, r = synthcat.uniform_patch(20_000, box, g), synthcat.uniform_patch(20_000, box, g)
    e = synthcat.log_edges(0.001, 0.1, 12)
    dr_ref = oracle.count(oracle.DR, oracle.radec_to_xyz(*d), e, oracle.radec_to_xyz(*r))
    a, b = ctx.upload_catalog(*d), ctx.upload_catalog(*r)
    try:
        assert np.array_equal(ctx.count(tp.DR, a, e, cat_b=b, precision=tp.FP32_CHORD), dr_ref)
        st = ctx.stats(reset=True)
        assert st.chord_steps > 0.9 * steps(st)
    finally:
        ctx.release_catalog(a)
        ctx.release_catalog(b)


@pytest.mark.parametrize("max_cols", [256, 4096])
def test_dot_path_staging_on_ragged_column_ranges(ctx, max_cols):
    """The dot-product steps read their columns from LDS, staged in blocks of
    64 per wavefront with the last block clamped to the column range's end.
    Uneven catalogs of dense 3 x 3 deg clumps 20 to 40 deg apart (data: 5003
    + 5004 points in two clumps, randoms: 9973 in a third), so that the pairs
    across clumps are settled from p; 30 edges from 0.5 to 120 deg; short
    column chunks (256 columns) or the default; row ranges that start the
    auto-pair column ranges at odd offsets.  DD and DR equal the oracle on
    the stored rows, and most steps were settled from p."""
    g = synthcat.rng_for(98, 1)
    pa = synthcat.uniform_patch(5003, (10.0, 13.0, 0.0, 3.0), g)
    pb = synthcat.uniform_patch(5004, (30.0, 33.0, 5.0, 8.0), g)
    d = tuple(np.concatenate([u, v]) for u, v in zip(pa, pb))
    r = synthcat.uniform_patch(9973, (50.0, 53.0, 20.0, 23.0), g)
    e = synthcat.log_edges(0.5, 120.0, 30)
    a, b = ctx.upload_catalog(*d), ctx.upload_catalog(*r)
    try:
        ctx.set_tuning(max_cols=max_cols)
        xa = tuple(c[ctx.catalog_order(a)] for c in oracle.radec_to_xyz(*d))
        xb = tuple(c[ctx.catalog_order(b)] for c in oracle.radec_to_xyz(*r))
        ctx.stats(reset=True)
        for rb, re in [(0, 10007), (333, 7777), (1001, 10006)]:
            got = ctx.count(tp.DD, a, e, precision=tp.FP32_CHORD, row_begin=rb, row_end=re)
            assert np.array_equal(got, oracle.count(oracle.DD, xa, e, row_begin=rb, row_end=re)), ("DD", rb)
            got = ctx.count(tp.DR, a, e, cat_b=b, precision=tp.FP32_CHORD, row_begin=rb, row_end=re)
            assert np.array_equal(got, oracle.count(oracle.DR, xa, e, b_xyz=xb, row_begin=rb, row_end=re)), \
                ("DR", rb)
        st = ctx.stats(reset=True)
        steps = st.pairs / 1024.0
        assert st.one_slot_steps + st.two_slot_steps > 0.4 * steps
        assert st.chord_steps < 0.5 * steps
    finally:
        ctx.set_tuning()
        ctx.release_catalog(a)
        ctx.release_catalog(b)


@pytest.mark.parametrize("prec", PRECS)
def test_pruning_keeps_counts_exact(ctx, patch, prec):
    """Exact tile pruning on the 30 x 30 deg patch: the same counts as the oracle, with
    some blocks binned whole, including row ranges (unaligned row tiles)."""
    wl, cd, cr, ref = patch
    e = wl.edges_deg
    try:
        ctx.set_tuning(prune=1)
        ctx.stats(reset=True)
        assert np.array_equal(ctx.count(tp.DD, cd, e, precision=prec), ref["DD"])
        assert np.array_equal(ctx.count(tp.DR, cd, e, cat_b=cr, precision=prec), ref["DR"])
        assert np.array_equal(ctx.count(tp.RR, cr, e, precision=prec), ref["RR"])
        st = ctx.stats(reset=True)
        assert 0 < st.pruned_pairs < st.pairs
        ctx.set_tuning()
        part = ctx.count(tp.DR, cd, e, cat_b=cr, precision=prec, row_begin=333, row_end=7777)
        ctx.set_tuning(prune=1)
        assert np.array_equal(ctx.count(tp.DR, cd, e, cat_b=cr, precision=prec, row_begin=333,
                                        row_end=7777), part)
    finally:
        ctx.set_tuning()


@pytest.mark.parametrize("prec", PRECS)
def test_pruning_exact_for_norms_at_the_accepted_limit(ctx, prec):
    """Vectors whose squared norms deviate from 1 by up to 0.95 x 2^-20 (the
    xyz entry's limit), in tight clusters a few 1e-6 rad from bin edges: the
    rule's dot product |a| |b| cos(phi) puts these pairs in other bins than
    their directions would, so a pruning test blind to the norm deviation
    would bin whole blocks wrongly.  DR and DD of the union, pruning off and
    on, against the oracle; the oracle's histograms differ from those of the
    normalised vectors (the test is sensitive), and pruning does bin blocks."""
    a, b, e = _cache.setdefault("near_limit", synthcat.near_limit_clusters())
    u = np.concatenate([a, b], axis=1)
    ref_dr = _oracle("near_limit_dr", lambda: oracle.count(oracle.DR, a, e, b_xyz=b))
    ref_dd = _oracle("near_limit_dd", lambda: oracle.count(oracle.DD, u, e))
    unit = lambda v: v / np.sqrt((v * v).sum(axis=0))
    assert not np.array_equal(ref_dr, oracle.count(oracle.DR, unit(a), e, b_xyz=unit(b)))
    ca = ctx.upload_catalog_xyz(*a)
    cb = ctx.upload_catalog_xyz(*b)
    cu = ctx.upload_catalog_xyz(*u)
    try:
        for prune in (0, 1):
            ctx.set_tuning(prune=prune)
            ctx.stats(reset=True)
            assert np.array_equal(ctx.count(tp.DR, ca, e, cat_b=cb, precision=prec), ref_dr), prune
            assert np.array_equal(ctx.count(tp.DD, cu, e, precision=prec), ref_dd), prune
            st = ctx.stats(reset=True)
            assert (st.pruned_pairs > 0) == (prune == 1)
    finally:
        ctx.set_tuning()
        for c in (ca, cb, cu):
            ctx.release_catalog(c)


@pytest.mark.parametrize("prec", PRECS)
def test_dense_patch_wide_bins_takes_every_branch(ctx, prec):
    """A dense 3 x 3 deg patch with four wide bins: many wavefront steps lie
    wholly beyond the last edge, many have all their pairs in one slot (one
    atomic per lane) or two adjacent slots (one threshold comparison per
    pair), the rest go through the per-pair lookups; the counts equal the
    oracle's."""
    g = synthcat.rng_for(97, 0)
    patch = (10.0, 13.0, 20.0, 23.0)
    d = synthcat.uniform_patch(20_000, patch, g)
    r = synthcat.uniform_patch(20_000, patch, g)
    e = synthcat.log_edges(0.01, 1.0, 4)
    cd = ctx.upload_catalog(*d)
    cr = ctx.upload_catalog(*r)
    xd = oracle.radec_to_xyz(*d)
    xr = oracle.radec_to_xyz(*r)
    ctx.stats(reset=True)
    dd_ref, dr_ref = oracle.count(oracle.DD, xd, e), oracle.count(oracle.DR, xd, e, xr)
    assert np.array_equal(ctx.count(tp.DD, cd, e, precision=prec), dd_ref)
    assert np.array_equal(ctx.count(tp.DR, cd, e, cat_b=cr, precision=prec), dr_ref)
    st = ctx.stats(reset=True)
    assert st.beyond_steps > 0
    assert st.one_slot_steps > 0
    assert st.two_slot_steps > 0
    # pruning bins whole blocks inside the wide bins and beyond the last edge
    try:
        ctx.set_tuning(prune=1)
        assert np.array_equal(ctx.count(tp.DD, cd, e, precision=prec), dd_ref)
        assert np.array_equal(ctx.count(tp.DR, cd, e, cat_b=cr, precision=prec), dr_ref)
        assert ctx.stats(reset=True).pruned_pairs > 0
    finally:
        ctx.set_tuning()
    ctx.release_catalog(cd)
    ctx.release_catalog(cr)


def test_repeatable(ctx, patch):
    wl, cd, cr, _ = patch
    a = [ctx.count(tp.DR, cd, wl.edges_deg, cat_b=cr, precision=tp.FP32_CHORD) for _ in range(3)]
    assert all(np.array_equal(a[0], x) for x in a[1:])


def test_gpu_error_paths(ctx, patch):
    wl, cd, cr, _ = patch
    e = wl.edges_deg
    with pytest.raises(tp.TpcfError) as ei:
        ctx.count(tp.DD, 9999, e)
    assert ei.value.code == -4
    with pytest.raises(tp.TpcfError) as ei:
        ctx.count(tp.DD, cd, e, cat_b=cr)
    assert ei.value.code == -1
    with pytest.raises(tp.TpcfError) as ei:
        ctx.count(tp.DR, cd, e, cat_b=9999)
    assert ei.value.code == -4
    with pytest.raises(tp.TpcfError):
        ctx.count(tp.DD, cd, e, row_begin=5, row_end=4)
    with pytest.raises(tp.TpcfError):
        ctx.count(tp.DD, cd, e, row_begin=0, row_end=10**9)
    with pytest.raises(tp.TpcfError):
        ctx.count(tp.DD, cd, e, precision=7)
    with pytest.raises(tp.TpcfError):
        ctx.count(tp.DD, cd, e[::-1].copy())
    with pytest.raises(tp.TpcfError):
        ctx.upload_catalog_xyz([2.0], [0.0], [0.0])
    with pytest.raises(tp.TpcfError):
        ctx.upload_catalog([np.nan], [0.0])
    with pytest.raises(tp.TpcfError) as ei:
        ctx.release_catalog(9999)
    assert ei.value.code == -4
    for bad in ({"rows_per_lane": 3}, {"hist_copies": 12}, {"max_cols": 300}, {"blocks_per_cu": -1},
                {"lut_bytes": 100}, {"lut_bytes": 40000}, {"lut_direct": 2}, {"prune": 3}):
        with pytest.raises(tp.TpcfError):
            ctx.set_tuning(**bad)
    assert ctx.get_tuning() == {k: 0 for k in ctx.get_tuning()}


def test_counts_do_not_depend_on_launch_shape(ctx, patch):
    """Race detector: every tuning choice (rows per lane, histogram copies,
    unit width, grid size, table layout and size) gives bit-identical counts."""
    wl, cd, cr, ref = patch
    e = wl.edges_deg
    try:
        for rpl in (2, 4):
            for hc in (32, 16, 8, 4):
                for mc, bpc, lb, lc, pr in ((256, 1, 0, 0, 1), (16384, 0, 4096, 1, 0),
                                            (4096, 3, 4096, 0, 1), (4096, 0, 33792, 1, 0)):
                    ctx.set_tuning(rows_per_lane=rpl, hist_copies=hc, max_cols=mc, blocks_per_cu=bpc,
                                   lut_bytes=lb, lut_direct=lc, prune=pr)
                    for prec in PRECS:
                        assert np.array_equal(ctx.count(tp.DD, cd, e, precision=prec), ref["DD"])
                        assert np.array_equal(ctx.count(tp.DR, cd, e, cat_b=cr, precision=prec),
                                              ref["DR"])
    finally:
        ctx.set_tuning()


def test_autotuner_picks_a_candidate(ctx, patch, tmp_path, monkeypatch):
    from paper_1204_6630_amd.autotune import CANDIDATES, autotune
    monkeypatch.setenv("TPCF_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    wl, cd, cr, ref = patch
    try:
        res = autotune(ctx, [(tp.DR, cd, cr, 0, 2048)], wl.edges_deg, tp.FP32_CHORD)
        assert not res["cached"]
        assert all(res["tuning"][k] in v for k, v in CANDIDATES.items())
        again = autotune(ctx, [(tp.DR, cd, cr, 0, 2048)], wl.edges_deg, tp.FP32_CHORD)
        assert again["cached"] and again["tuning"] == res["tuning"]
        assert np.array_equal(ctx.count(tp.DR, cd, wl.edges_deg, cat_b=cr), ref["DR"])
    finally:
        ctx.set_tuning()
