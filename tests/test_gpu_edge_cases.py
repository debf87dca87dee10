"""GPU parity at the limits of the bin count and on seeded random cases
(needs an MI355X).

* nbins from 1 to the maximum 256: past 125 bins the cell tables switch from
  one-byte to two-byte entries and the per-wavefront histogram copies drop
  from 16 to 8 and then 4, so each of those kernel variants meets the oracle
  here, for every precision and for 3-D catalogs too;
* edges that include 0 and 180 degrees exactly, on the full sphere;
* 16 seeded random cases: catalog sizes, bin counts, edge placements, point
  distributions (full sphere, clustered patch, duplicated points), kinds,
  precisions, launch shapes and FP32 table layouts (clamped or wrapped) drawn
  at random, each bit-exact against the oracle.
"""

import numpy as np
import pytest

import oracle
import paper_1204_6630_amd as tp
import synthcat

pytestmark = pytest.mark.gpu

PRECS = [tp.FP32_CHORD, tp.FP64]


@pytest.fixture(scope="module")
def ctx():
    c = tp.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def sphere(ctx):
    g = synthcat.rng_for(97, 0)
    ra_a, dec_a = synthcat.uniform_sphere(2500, g)
    ra_c, dec_c = synthcat.clustered(1500, 40, 2.0, (0.0, 360.0, -90.0, 90.0), g)
    ra_a = np.concatenate([ra_a, ra_c])
    dec_a = np.concatenate([dec_a, dec_c])
    ra_b, dec_b = synthcat.uniform_sphere(1700, g)
    ca = ctx.upload_catalog(ra_a, dec_a)
    cb = ctx.upload_catalog(ra_b, dec_b)
    return ca, cb, oracle.radec_to_xyz(ra_a, dec_a), oracle.radec_to_xyz(ra_b, dec_b)


_ref = {}


@pytest.mark.parametrize("nbins", [1, 20, 125])
def test_wrapped_table_on_the_full_sphere(ctx, sphere, nbins):
    """The wrapped FP32 table (q summed from a floor, key masked, no clamp)
    on the full sphere, where q reaches its largest values, with edges from
    0 to 180 degrees and log edges from 1e-4 degrees."""
    ca, cb, xa, xb = sphere
    ctx.set_tuning(lut_direct=1)
    try:
        for edges in (np.linspace(0.0, 180.0, nbins + 1), synthcat.log_edges(1e-4, 180.0, nbins)):
            got = ctx.count(tp.DR, ca, edges, cat_b=cb, precision=tp.FP32_CHORD)
            assert np.array_equal(got, oracle.count(oracle.DR, xa, edges, b_xyz=xb))
    finally:
        ctx.set_tuning()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("nbins", [1, 125, 126, 200, 256])
def test_bin_counts_up_to_the_maximum(ctx, sphere, prec, nbins):
    ca, cb, xa, xb = sphere
    edges = np.linspace(0.0, 180.0, nbins + 1)          # 0 and 180 exactly
    if nbins == 200:
        edges = np.concatenate([[0.0], synthcat.log_edges(1e-3, 180.0, nbins)])[:nbins + 1]
    if (nbins, "DD") not in _ref:
        _ref[(nbins, "DD")] = oracle.count(oracle.DD, xa, edges)
        _ref[(nbins, "DR")] = oracle.count(oracle.DR, xa, edges, b_xyz=xb)
    assert np.array_equal(ctx.count(tp.DD, ca, edges, precision=prec), _ref[(nbins, "DD")])
    assert np.array_equal(ctx.count(tp.DR, ca, edges, cat_b=cb, precision=prec), _ref[(nbins, "DR")])


@pytest.mark.parametrize("prec", PRECS)
def test_3d_with_256_bins(ctx, prec):
    g = synthcat.rng_for(97, 1)
    a = synthcat.box_clustered(3000, 60, 3.0, 200.0, g)
    edges = np.linspace(0.0, 120.0, 257)
    cid = ctx.upload_catalog_3d(*a.xyz())
    try:
        ref = _ref.setdefault("3d256", oracle.count3d(oracle.DD, a.xyz(), edges))
        assert np.array_equal(ctx.count(tp.DD, cid, edges, precision=prec), ref)
    finally:
        ctx.release_catalog(cid)


def _random_case(seed):
    g = np.random.default_rng(1000 + seed)
    na = int(g.choice([1, 2, 17, 64, 65, 1000, 1537, 3000]))
    nb = int(g.choice([1, 3, 64, 257, 999, 2500]))
    nbins = int(g.choice([1, 2, 7, 40, 125, 126, 199, 256]))
    style = g.choice(["sphere", "patch", "dups"])
    if style == "sphere":
        ra, dec = synthcat.uniform_sphere(na + nb, g)
    elif style == "patch":
        ra, dec = synthcat.clustered(na + nb, max(1, (na + nb) // 30), 0.5, synthcat.PATCH_30, g)
    else:
        # a few distinct positions, each repeated: many coincident pairs
        r0, d0 = synthcat.uniform_patch(max(1, (na + nb) // 8), synthcat.PATCH_30, g)
        pick = g.integers(0, r0.size, size=na + nb)
        ra, dec = r0[pick], d0[pick]
    lo = float(g.choice([0.0, 1e-4, 0.01]))
    hi = float(g.choice([1.0, 30.0, 180.0]))
    if g.uniform() < 0.5 and lo > 0.0:
        edges = synthcat.log_edges(lo, hi, nbins)
    else:
        edges = np.linspace(lo, hi, nbins + 1)
    kind = int(g.choice([tp.DD, tp.DR]))
    prec = int(g.choice(PRECS))
    tuning = {"rows_per_lane": int(g.choice([0, 2, 4])), "hist_copies": int(g.choice([0, 4, 8, 32])),
              "max_cols": int(g.choice([0, 256, 1024])), "lut_direct": int(g.choice([0, 1]))}
    return (ra[:na], dec[:na]), (ra[na:], dec[na:]), edges, kind, prec, tuning, style


@pytest.mark.parametrize("seed", range(16))
def test_seeded_random_cases(ctx, seed):
    (ra_a, dec_a), (ra_b, dec_b), edges, kind, prec, tuning, style = _random_case(seed)
    print(f"case {seed}: na={ra_a.size} nb={ra_b.size} nbins={edges.size - 1} kind={kind} "
          f"prec={prec} {style} {tuning}", flush=True)
    ca = ctx.upload_catalog(ra_a, dec_a)
    cb = ctx.upload_catalog(ra_b, dec_b)
    ctx.set_tuning(**tuning)
    try:
        xa = oracle.radec_to_xyz(ra_a, dec_a)
        if kind == tp.DD:
            got = ctx.count(tp.DD, ca, edges, precision=prec)
            ref = oracle.count(oracle.DD, xa, edges)
        else:
            got = ctx.count(tp.DR, ca, edges, cat_b=cb, precision=prec)
            ref = oracle.count(oracle.DR, xa, edges, b_xyz=oracle.radec_to_xyz(ra_b, dec_b))
        assert np.array_equal(got, ref)
    finally:
        ctx.set_tuning()
        ctx.release_catalog(ca)
        ctx.release_catalog(cb)


def test_huge_request_uses_wide_units_with_the_same_counts(ctx):
    """4e7 random points on the device (zero-copy attach) against 1e6 data
    rows, 2 rows per lane (512-row tiles): 4e13 pairs, beyond what
    4096-column units can list within the unit budget (16.7M units), so the
    plan widens its column chunks.  The counts must equal the sum over two
    halves of the rows, whose plans keep the usual width, and the totals must
    close."""
    import torch
    g = torch.Generator(device="cuda:0")
    g.manual_seed(1204)
    nr, nd = 40_000_000, 1_000_000

    def unit_vectors(n):
        v = torch.randn((3, n), dtype=torch.float64, device="cuda:0", generator=g)
        v /= torch.linalg.vector_norm(v, dim=0, keepdim=True)
        return v.contiguous()

    tr = unit_vectors(nr)
    td = unit_vectors(nd)
    cr = ctx.attach_catalog(tr)
    cd = ctx.attach_catalog(td)
    ctx.set_tuning(rows_per_lane=2)
    try:
        edges = synthcat.log_edges(0.01, 1.0, 20)
        full = ctx.count(tp.DR, cd, edges, cat_b=cr)
        halves = (ctx.count(tp.DR, cd, edges, cat_b=cr, row_begin=0, row_end=nd // 2)
                  + ctx.count(tp.DR, cd, edges, cat_b=cr, row_begin=nd // 2, row_end=nd))
        assert int(full.sum()) == nd * nr
        assert np.array_equal(full, halves)
    finally:
        ctx.set_tuning()
        ctx.release_catalog(cd)
        ctx.release_catalog(cr)
        del tr, td
        torch.cuda.empty_cache()
