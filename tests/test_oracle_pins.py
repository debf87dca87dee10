"""Pins for the CPU oracle (no GPU).

Each test fixes the oracle against something other than its own code:
exact trigonometric values, an independent angle formula (chord ->
2 asin(c/2) through scipy), constructed geometries with known separations,
the full-sphere closed form, exact algebraic invariants, and hand-worked
Landy-Szalay values.  A dropped term, a wrong sign or index, a transposed
operand, a degree/radian slip or a "<" for "<=" in the binning fails at least
one of them.
"""

import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
import rounding_probes as rp
import synthcat
from oracle import tiny

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DEG = math.pi / 180.0


def _xyz(ra, dec):
    return oracle.radec_to_xyz(ra, dec)


def _stack(xyz):
    return np.stack(xyz, axis=1)


def _chord_angles(a, b):
    """Independent angle formula: theta = 2 asin(|a-b| / 2) from scipy's
    Euclidean distance."""
    c = cdist(a, b)
    return 2.0 * np.arcsin(np.minimum(c / 2.0, 1.0))


def _random_rotation(g):
    q, r = np.linalg.qr(g.normal(size=(3, 3)))
    return q * np.sign(np.diag(r))


# --------------------------------------------------------------------------
# Unit vectors (Section 3: angles come from dot products of unit vectors)
# --------------------------------------------------------------------------

def test_unit_vectors_exact_values():
    rows = np.loadtxt(os.path.join(GOLDEN, "unit_vectors.txt"))
    x, y, z = _xyz(rows[:, 0], rows[:, 1])
    got = np.stack([x, y, z], axis=1)
    assert np.max(np.abs(got - rows[:, 2:5])) < 2e-16 * 4


def test_unit_vectors_have_unit_norm():
    g = synthcat.rng_for(90, 0)
    ra, dec = synthcat.uniform_sphere(20000, g)
    x, y, z = _xyz(ra, dec)
    n2 = x * x + y * y + z * z
    assert np.max(np.abs(n2 - 1.0)) < 8e-16


# --------------------------------------------------------------------------
# Angles: arc-cosine of the clamped dot product vs an independent formula
# --------------------------------------------------------------------------

def test_pair_angle_matches_chord_formula():
    g = synthcat.rng_for(90, 1)
    n = 4000
    a = _stack(_xyz(*synthcat.uniform_sphere(n, g)))
    # partners at log-uniform separations from 1e-6 rad to pi
    theta = np.exp(g.uniform(math.log(1e-6), math.log(math.pi), size=n))
    u = g.normal(size=(n, 3))
    u -= np.sum(u * a, axis=1)[:, None] * a
    u /= np.linalg.norm(u, axis=1)[:, None]
    b = np.cos(theta)[:, None] * a + np.sin(theta)[:, None] * u
    b /= np.linalg.norm(b, axis=1)[:, None]
    t_oracle = oracle.pair_angles(a.T, b.T)
    t_ref = np.array([_chord_angles(a[i:i + 1], b[i:i + 1])[0, 0] for i in range(n)])
    # acos loses accuracy as 1/sin(theta): the dot carries ~3 ulp of error
    tol = 6e-16 / np.maximum(np.sin(t_ref), 1e-300) + 4e-16 * t_ref + 1e-15
    assert np.all(np.abs(t_oracle - t_ref) <= tol)


def test_pair_angle_clamps_duplicates_and_antipodes():
    g = synthcat.rng_for(90, 2)
    a = _stack(_xyz(*synthcat.uniform_sphere(500, g)))
    t_same = oracle.pair_angles(a.T, a.T)
    assert np.all(t_same < 3e-8)          # acos(clamped d ~ 1)
    t_anti = oracle.pair_angles(a.T, (-a).T)
    assert np.all(np.abs(t_anti - math.pi) < 3e-8)
    assert np.all(np.isfinite(t_same)) and np.all(np.isfinite(t_anti))


# --------------------------------------------------------------------------
# Binning
# --------------------------------------------------------------------------

def _near_edge(theta, edges_rad, rel=1e-9):
    d = np.abs(theta[..., None] - edges_rad[None, :])
    return np.any(d <= rel * edges_rad[None, :] + 1e-12, axis=-1)


@pytest.mark.parametrize("cfg,scale", [("patch30_1e4", 0.015), ("octant_1e5", 0.0015)])
def test_histogram_matches_independent_binning(cfg, scale):
    """Per-pair slots and whole histograms against scipy chord distances
    binned with numpy.searchsorted (side='right': theta == e_k goes up)."""
    wl = synthcat.WORKLOADS[cfg](scale=scale)
    d = wl.data[0]
    edges = wl.edges_deg
    er = edges * DEG
    a = _stack(_xyz(d.ra, d.dec))
    n = a.shape[0]
    th = _chord_angles(a, a)
    iu, ju = np.triu_indices(n, k=1)
    t = th[iu, ju]
    ref = np.searchsorted(er, t, side="right")
    near = _near_edge(t, er)
    assert near.sum() <= 2  # only a handful of pairs can sit this close
    slots = oracle.pair_slots(a[iu].T, a[ju].T, edges)
    assert np.array_equal(slots[~near], ref[~near])
    hist = oracle.count(oracle.DD, a.T, edges)
    assert np.array_equal(hist, np.bincount(slots, minlength=edges.size + 1).astype(np.uint64))
    ref_hist = np.bincount(ref, minlength=edges.size + 1)
    assert np.sum(np.abs(hist.astype(np.int64) - ref_hist)) <= 2 * near.sum()


def test_tie_on_edge_goes_to_upper_bin():
    """A pair whose angle equals an edge exactly lands in the upper bin."""
    g = synthcat.rng_for(90, 3)
    a = _stack(_xyz(*synthcat.uniform_sphere(400, g)))
    b = _stack(_xyz(*synthcat.uniform_sphere(400, g)))
    t = oracle.pair_angles(a.T, b.T)
    found = 0
    for i in range(a.shape[0]):
        e0 = t[i] / DEG
        cands = [e0]
        for _ in range(4):
            cands.append(np.nextafter(cands[-1], np.inf))
        c2 = [e0]
        for _ in range(4):
            c2.append(np.nextafter(c2[-1], -np.inf))
        exact = [e for e in cands + c2 if e * DEG == t[i]]
        if not exact:
            continue
        found += 1
        e = exact[0]
        above = next(c for c in cands if c * DEG > t[i])
        below = next(c for c in c2 if c * DEG < t[i])
        pa, pb = a[i:i + 1].T, b[i:i + 1].T
        assert oracle.pair_slots(pa, pb, [e / 2, e, 2 * e])[0] == 2
        assert oracle.pair_slots(pa, pb, [below / 2, below, 2 * e])[0] == 2
        assert oracle.pair_slots(pa, pb, [e / 2, above, 2 * e])[0] == 1
        assert oracle.pair_slots(pa, pb, [e, 2 * e])[0] == 1
        assert oracle.pair_slots(pa, pb, [above, 2 * e])[0] == 0
    assert found >= 100


def test_isolated_probe_pairs_land_in_known_bins():
    """Probe pairs separated by each bin's geometric centre, with probes far
    apart from one another: bin k holds exactly the probes aimed at it and
    every other pair is overflow."""
    edges = synthcat.log_edges(0.01, 10.0, 20)
    nb = edges.size - 1
    g = synthcat.rng_for(90, 4)
    # bases on a coarse grid: mutual separations >= ~25 deg
    bases = []
    for dec in (-60.0, -30.0, 0.0, 30.0, 60.0):
        step = 30.0 / max(math.cos(math.radians(dec)), 0.5)
        ra = 0.0
        while ra < 360.0 - step / 2:
            bases.append((ra, dec))
            ra += step
    bases = np.array(bases)
    kbin = g.integers(0, nb, size=len(bases))
    centre = np.sqrt(edges[kbin] * edges[kbin + 1]) * DEG
    bx = _stack(_xyz(bases[:, 0], bases[:, 1]))
    u = g.normal(size=bx.shape)
    u -= np.sum(u * bx, axis=1)[:, None] * bx
    u /= np.linalg.norm(u, axis=1)[:, None]
    px = np.cos(centre)[:, None] * bx + np.sin(centre)[:, None] * u
    pts = np.concatenate([bx, px])
    n = pts.shape[0]
    # geometry check with the independent formula: cross-probe pairs are far
    th = _chord_angles(pts, pts)
    m = len(bases)
    for i in range(m):
        th[i, m + i] = th[m + i, i] = np.inf
    np.fill_diagonal(th, np.inf)
    assert th.min() > 15.0 * DEG
    hist = oracle.count(oracle.DD, pts.T, edges)
    expect = np.zeros(nb + 2, dtype=np.uint64)
    for k in kbin:
        expect[k + 1] += 1
    expect[nb + 1] = n * (n - 1) // 2 - m
    assert np.array_equal(hist, expect)
    # the same probes through the RA/Dec entry (degrees, not radians)
    ra = np.degrees(np.arctan2(pts[:, 1], pts[:, 0])) % 360.0
    dec = np.degrees(np.arcsin(np.clip(pts[:, 2], -1, 1)))
    hist2 = oracle.count(oracle.DD, _xyz(ra, dec), edges)
    assert np.array_equal(hist2, expect)


def test_duplicates_antipodes_and_tiny_catalogs():
    g = synthcat.rng_for(90, 5)
    p = _stack(_xyz(*synthcat.uniform_sphere(50, g)))
    edges = np.array([0.01, 1.0, 179.0])
    dup = np.concatenate([p, p])
    h = oracle.count(oracle.DR, p.T, edges, b_xyz=p.T)
    # DR of a catalog with itself: the 50 coincident pairs are underflow
    assert h[0] >= 50
    anti = oracle.count(oracle.DR, p.T, edges, b_xyz=(-p).T)
    assert anti[3] >= 50
    assert oracle.count(oracle.DD, dup.T, edges)[0] >= 50
    # e_0 = 0: coincident pairs are theta = 0 >= e_0, slot 1
    h0 = oracle.count(oracle.DR, p[:1].T, [0.0, 1.0], b_xyz=p[:1].T)
    assert list(h0) == [0, 1, 0]
    for n, tot in ((0, 0), (1, 0), (2, 1), (3, 3)):
        h = oracle.count(oracle.DD, p[:n].T, edges)
        assert int(h.sum()) == tot


def test_full_sphere_closed_form():
    """Uniform points on the whole sphere: P(theta in [a, b)) =
    (cos a - cos b) / 2 and pair indicators are pairwise uncorrelated, so each
    bin count is within 5 sigma of M p with sigma^2 = M p (1 - p)."""
    g = synthcat.rng_for(90, 6)
    n = 3000
    a = _xyz(*synthcat.uniform_sphere(n, g))
    edges = np.array([0.0, 0.5, 2.0, 5.0, 10.0, 20.0, 45.0, 90.0, 135.0, 170.0, 180.0])
    h = oracle.count(oracle.DD, a, edges).astype(np.float64)
    m = n * (n - 1) / 2
    assert h[0] == 0
    er = edges * DEG
    p = (np.cos(er[:-1]) - np.cos(er[1:])) / 2.0
    mean = m * p
    sd = np.sqrt(m * p * (1 - p))
    z = (h[1:-1] - mean) / sd
    assert np.all(np.abs(z) < 5.0), z
    assert h[-1] == 0   # no exact antipodes among random points


# --------------------------------------------------------------------------
# Totals and exact invariants
# --------------------------------------------------------------------------

def _small_sets(seed, na=700, nb=500):
    g = synthcat.rng_for(91, seed)
    a = _xyz(*synthcat.clustered(na, 20, 0.5, synthcat.PATCH_30, g))
    b = _xyz(*synthcat.uniform_patch(nb, synthcat.PATCH_30, g))
    return a, b


def test_totals():
    a, b = _small_sets(0)
    edges = synthcat.log_edges(0.01, 10.0, 20)
    na, nb = a[0].size, b[0].size
    assert int(oracle.count(oracle.DD, a, edges).sum()) == na * (na - 1) // 2
    assert int(oracle.count(oracle.DR, a, edges, b_xyz=b).sum()) == na * nb
    r = oracle.count(oracle.DD, a, edges, row_begin=100, row_end=250)
    assert int(r.sum()) == sum(na - 1 - i for i in range(100, 250))
    r = oracle.count(oracle.DR, a, edges, b_xyz=b, row_begin=10, row_end=20)
    assert int(r.sum()) == 10 * nb


def test_union_decomposition_and_symmetry():
    a, b = _small_sets(1)
    edges = synthcat.log_edges(0.01, 10.0, 20)
    u = tuple(np.concatenate([p, q]) for p, q in zip(a, b))
    ddu = oracle.count(oracle.DD, u, edges)
    dda = oracle.count(oracle.DD, a, edges)
    ddb = oracle.count(oracle.DD, b, edges)
    drab = oracle.count(oracle.DR, a, edges, b_xyz=b)
    drba = oracle.count(oracle.DR, b, edges, b_xyz=a)
    assert np.array_equal(ddu, dda + ddb + drab)
    assert np.array_equal(drab, drba)


def test_reflection_and_permutation_invariance():
    a, b = _small_sets(2)
    edges = synthcat.log_edges(0.01, 10.0, 20)
    base = oracle.count(oracle.DD, a, edges)
    refl = oracle.count(oracle.DD, (a[0], a[1], -a[2]), edges)
    perm = np.random.default_rng(5).permutation(a[0].size)
    per = oracle.count(oracle.DD, tuple(c[perm] for c in a), edges)
    assert np.array_equal(base, refl)
    assert np.array_equal(base, per)
    dr = oracle.count(oracle.DR, a, edges, b_xyz=b)
    dr2 = oracle.count(oracle.DR, (-a[0], a[1], a[2]), edges, b_xyz=(-b[0], b[1], b[2]))
    assert np.array_equal(dr, dr2)


def test_row_ranges_add_up():
    a, b = _small_sets(3)
    edges = synthcat.log_edges(0.01, 10.0, 20)
    full = oracle.count(oracle.DD, a, edges)
    cuts = [0, 1, 77, 300, 699, 700]
    parts = sum(oracle.count(oracle.DD, a, edges, row_begin=c0, row_end=c1)
                for c0, c1 in zip(cuts[:-1], cuts[1:]))
    assert np.array_equal(full, parts)
    fdr = oracle.count(oracle.DR, a, edges, b_xyz=b)
    pdr = sum(oracle.count(oracle.DR, a, edges, b_xyz=b, row_begin=c0, row_end=c1)
              for c0, c1 in zip(cuts[:-1], cuts[1:]))
    assert np.array_equal(fdr, pdr)


def test_thread_count_does_not_change_counts():
    a, b = _small_sets(4)
    edges = synthcat.log_edges(0.01, 10.0, 20)
    h1 = oracle.count(oracle.DR, a, edges, b_xyz=b, nthreads=1)
    h7 = oracle.count(oracle.DR, a, edges, b_xyz=b, nthreads=7)
    assert np.array_equal(h1, h7)


def test_pure_python_transcription_agrees_bit_for_bit():
    g = synthcat.rng_for(91, 9)
    ra, dec = synthcat.clustered(300, 10, 0.3, synthcat.PATCH_30, g)
    ra2, dec2 = synthcat.uniform_patch(120, synthcat.PATCH_30, g)
    edges = synthcat.log_edges(0.01, 10.0, 20)
    pa = [tiny.unit_vector(r, d) for r, d in zip(ra, dec)]
    pb = [tiny.unit_vector(r, d) for r, d in zip(ra2, dec2)]
    xa = _xyz(ra, dec)
    xb = _xyz(ra2, dec2)
    assert np.array_equal(np.array(pa), np.stack(xa, axis=1))
    assert list(oracle.count(oracle.DD, xa, edges)) == tiny.count_pairs(pa, edges)
    assert list(oracle.count(oracle.DR, xa, edges, b_xyz=xb)) == tiny.count_pairs(pa, edges, pb)


# --------------------------------------------------------------------------
# Landy-Szalay (Eq. 1)
# --------------------------------------------------------------------------

def test_landy_szalay_hand_worked_values():
    with open(os.path.join(GOLDEN, "landy_szalay_closed_form.json")) as f:
        fx = json.load(f)
    for case in fx["cases"]:
        for form, key in ((0, "w_form0"), (1, "w_form1")):
            w = oracle.landy_szalay(case["dd"], case["dr"], case["rr"],
                                    case["n_d"], case["n_r"], form=form)
            for got, want in zip(w, case[key]):
                if want is None:
                    assert math.isnan(got)
                else:
                    assert abs(got - want) <= 1e-14 * max(1.0, abs(want))


def test_landy_szalay_random_vs_random_is_zero():
    """Independent uniform D and R on the same patch give w ~ 0 within a few
    Poisson sigma (~1/sqrt(DD)), for both readings of Eq. 1; the literal
    formula applied to unordered counts would give w ~ -2 instead."""
    g1 = synthcat.rng_for(92, 0)
    g2 = synthcat.rng_for(92, 1)
    nd, nr = 3000, 6000
    d = _xyz(*synthcat.uniform_patch(nd, synthcat.PATCH_30, g1))
    r = _xyz(*synthcat.uniform_patch(nr, synthcat.PATCH_30, g2))
    edges = synthcat.log_edges(0.5, 10.0, 8)
    dd = oracle.count(oracle.DD, d, edges)[1:-1]
    dr = oracle.count(oracle.DR, d, edges, b_xyz=r)[1:-1]
    rr = oracle.count(oracle.RR, r, edges)[1:-1]
    sigma = np.sqrt(2.0 / dd.astype(np.float64))
    for form in (0, 1):
        w = oracle.landy_szalay(dd, dr, rr, nd, nr, form=form)
        assert np.all(np.abs(w) < 5 * sigma), (form, w, sigma)
    ratio = nr / nd
    naive = 1 + ratio ** 2 * dd / rr - 2 * ratio * dr / rr
    assert np.all(np.abs(naive + 2.0) < 0.2)


# --- jackknife regions (count_regions, jackknife) -----------------------------

def _regions_case(seed, n_d=400, n_r=500, nreg=5):
    g = synthcat.rng_for(93, seed)
    patch = (0.0, 20.0, 0.0, 20.0)
    ra_d, dec_d = synthcat.uniform_patch(n_d, patch, g)
    ra_r, dec_r = synthcat.uniform_patch(n_r, patch, g)
    # regions: RA stripes of 4 deg (a typical jackknife split)
    reg_d = np.minimum((ra_d // 4).astype(np.int32), nreg - 1)
    reg_r = np.minimum((ra_r // 4).astype(np.int32), nreg - 1)
    return _xyz(ra_d, dec_d), reg_d, _xyz(ra_r, dec_r), reg_r, nreg


def test_region_totals_equal_plain_counts_and_one_region_touches_all():
    d, rd, r, rr_, nreg = _regions_case(0)
    e = synthcat.log_edges(0.1, 10.0, 12)
    for kind, b, rb in ((oracle.DD, None, None), (oracle.DR, r, rr_)):
        total, touch = oracle.count_regions(kind, d, rd, e, nreg, b_xyz=b, b_region=rb)
        assert np.array_equal(total, oracle.count(kind, d, e, b_xyz=b))
        one_a = np.zeros_like(rd)
        one_b = None if rb is None else np.zeros_like(rb)
        t1, touch1 = oracle.count_regions(kind, d, one_a, e, 1, b_xyz=b, b_region=one_b)
        assert np.array_equal(touch1[0], t1)


def test_removing_a_region_removes_exactly_its_touch_row():
    """Deletion identity against recounts of the reduced catalogs: a planted
    double count of same-region pairs, a missing second region, or swapped
    DR labels would each break it."""
    d, rd, r, rr_, nreg = _regions_case(1)
    e = synthcat.log_edges(0.1, 10.0, 12)
    dd_t, dd_touch = oracle.count_regions(oracle.DD, d, rd, e, nreg)
    dr_t, dr_touch = oracle.count_regions(oracle.DR, d, rd, e, nreg, b_xyz=r, b_region=rr_)
    for k in range(nreg):
        kd, kr = rd != k, rr_ != k
        dsub = [c[kd] for c in d]
        rsub = [c[kr] for c in r]
        assert np.array_equal(dd_t - dd_touch[k], oracle.count(oracle.DD, dsub, e))
        assert np.array_equal(dr_t - dr_touch[k], oracle.count(oracle.DR, dsub, e, b_xyz=rsub))


def test_region_counts_match_pure_python():
    d, rd, r, rr_, nreg = _regions_case(2, n_d=60, n_r=70, nreg=3)
    e = synthcat.log_edges(0.5, 12.0, 6)
    er = [x * (math.pi / 180.0) for x in e]
    pa = list(zip(*d))
    pb = list(zip(*r))
    for kind in (oracle.DD, oracle.DR):
        total = np.zeros(e.size + 1, np.uint64)
        touch = np.zeros((nreg, e.size + 1), np.uint64)
        if kind == oracle.DD:
            pairs = [(pa[i], pa[j], rd[i], rd[j]) for i in range(len(pa)) for j in range(i + 1, len(pa))]
        else:
            pairs = [(pa[i], pb[j], rd[i], rr_[j]) for i in range(len(pa)) for j in range(len(pb))]
        for p, q, ri, rj in pairs:
            s = tiny.slot(tiny.angle(p, q), er)
            total[s] += 1
            touch[ri, s] += 1
            if rj != ri:
                touch[rj, s] += 1
        got_t, got_touch = oracle.count_regions(kind, d, rd, e, nreg,
                                                b_xyz=None if kind == oracle.DD else r,
                                                b_region=None if kind == oracle.DD else rr_)
        assert np.array_equal(got_t, total) and np.array_equal(got_touch, touch)


def test_jackknife_samples_and_covariance():
    """Samples by recount equal Landy-Szalay of (total - touch) with the
    region's points removed from N_D and N_R; the covariance equals
    (K-1)^2/K times numpy's unbiased sample covariance."""
    d, rd, r, rr_, nreg = _regions_case(3)
    e = synthcat.log_edges(0.5, 10.0, 6)
    samples, mean, cov = oracle.jackknife(d, rd, r, rr_, e, nreg)
    dd_t, dd_touch = oracle.count_regions(oracle.DD, d, rd, e, nreg)
    dr_t, dr_touch = oracle.count_regions(oracle.DR, d, rd, e, nreg, b_xyz=r, b_region=rr_)
    rr_t, rr_touch = oracle.count_regions(oracle.RR, r, rr_, e, nreg)
    for k in range(nreg):
        nd = int((rd != k).sum())
        nr = int((rr_ != k).sum())
        w = oracle.landy_szalay((dd_t - dd_touch[k])[1:-1], (dr_t - dr_touch[k])[1:-1],
                                (rr_t - rr_touch[k])[1:-1], nd, nr)
        assert np.array_equal(np.isnan(w), np.isnan(samples[k]))
        fin = np.isfinite(w)
        assert np.allclose(w[fin], samples[k][fin], rtol=0, atol=1e-13)
    fin = np.all(np.isfinite(samples), axis=0)
    ref = (nreg - 1) ** 2 / nreg * np.cov(samples[:, fin].T, ddof=1)
    assert np.allclose(cov[np.ix_(fin, fin)], ref, rtol=1e-12, atol=1e-15)
    assert np.allclose(mean, samples.mean(axis=0), equal_nan=True)


# --- 3-D distances (count3d, pair_distances) ---------------------------------

def _lattice(n, offset=0.0):
    g = np.arange(n, dtype=np.float64) + offset
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def _lattice_histogram(n, edges):
    """Closed form for the unordered pairs of an n^3 integer lattice: the
    displacement (a, b, c) occurs (n-|a|)(n-|b|)(n-|c|) times as an ordered
    pair, and its squared length a^2 + b^2 + c^2 is an exact integer.  An
    edge e (a double whose square is exact) lies at or below the distance
    exactly when e^2 <= a^2 + b^2 + c^2; on this lattice no squared distance
    is close enough to an e^2 for the rounding of the square root to matter."""
    e2 = [float(e) * float(e) for e in edges]
    hist = np.zeros(len(edges) + 1, dtype=np.int64)
    for a in range(-(n - 1), n):
        for b in range(-(n - 1), n):
            for c in range(-(n - 1), n):
                if a == 0 and b == 0 and c == 0:
                    continue
                mult = (n - abs(a)) * (n - abs(b)) * (n - abs(c))
                r2 = a * a + b * b + c * c
                hist[sum(1 for t in e2 if t <= r2)] += mult
    assert np.all(hist % 2 == 0)
    return (hist // 2).astype(np.uint64)


def test_3d_lattice_closed_form_with_ties_on_edges():
    """Edges 1, 2, 3, 4 equal lattice distances exactly (ties go to the upper
    bin); 1.5, 2.5 and 5.25 fall between squared distances.  A dropped
    coordinate term, a compare of r^2 against e (no square root), i <= j, or
    a tie sent down each changes this histogram."""
    n = 6
    edges = np.array([0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 4.0, 5.25])
    got = oracle.count3d(oracle.DD, _lattice(n), edges)
    assert np.array_equal(got, _lattice_histogram(n, edges))
    assert int(got.sum()) == n ** 3 * (n ** 3 - 1) // 2


def test_3d_exact_distances_of_pythagorean_pairs():
    a = [np.zeros(4), np.zeros(4), np.zeros(4)]
    b = [np.array([3.0, 1.0, 2.0, 0.0]), np.array([4.0, 2.0, 3.0, 0.0]), np.array([0.0, 2.0, 6.0, 0.0])]
    assert list(oracle.pair_distances(a, b)) == [5.0, 3.0, 7.0, 0.0]


def test_3d_histogram_matches_scipy_distances():
    """scipy's Euclidean distances (its own arithmetic) binned with
    numpy.searchsorted(side='right'); pairs whose distance lies within 1e-12
    relative of an edge (none expected) are left out of the comparison."""
    g = synthcat.rng_for(96, 0)
    a = g.uniform(0.0, 100.0, size=(700, 3))
    b = g.uniform(20.0, 140.0, size=(600, 3))
    edges = synthcat.log_edges(0.5, 80.0, 15)
    for kind, other in ((oracle.DR, b), (oracle.DD, None)):
        dist = cdist(a, a if other is None else other)
        if other is None:
            dist = dist[np.triu_indices(a.shape[0], k=1)]
        else:
            dist = dist.ravel()
        near = np.min(np.abs(dist[:, None] - edges[None, :]) / edges[None, :], axis=1) < 1e-12
        assert not near.any()
        ref = np.bincount(np.searchsorted(edges, dist, side="right"), minlength=edges.size + 1)
        got = oracle.count3d(kind, a.T, edges, b_xyz=None if other is None else other.T)
        assert np.array_equal(got, ref.astype(np.uint64))


def test_3d_power_of_two_scaling_and_exact_translation():
    """Scaling coordinates and edges by 4 is exact in every operation, the
    square root included, so counts are identical; so is a translation of
    integer coordinates by 1024 (exact differences)."""
    g = synthcat.rng_for(96, 1)
    pts = np.round(g.uniform(0.0, 60.0, size=(500, 3)))
    edges = np.array([0.0, 1.0, 2.0, 3.5, 7.0, 12.0, 20.0, 33.0])
    base = oracle.count3d(oracle.DD, pts.T, edges)
    assert np.array_equal(base, oracle.count3d(oracle.DD, (4.0 * pts).T, 4.0 * edges))
    assert np.array_equal(base, oracle.count3d(oracle.DD, (pts + 1024.0).T, edges))
    # edge 0: every pair, coincident points included, is at or above it
    assert int(base[0]) == 0


def test_3d_union_symmetry_and_totals():
    g = synthcat.rng_for(96, 2)
    a = g.normal(50.0, 10.0, size=(400, 3))
    b = g.uniform(0.0, 100.0, size=(300, 3))
    edges = synthcat.log_edges(0.2, 60.0, 12)
    dd_a = oracle.count3d(oracle.DD, a.T, edges)
    dd_b = oracle.count3d(oracle.DD, b.T, edges)
    dr = oracle.count3d(oracle.DR, a.T, edges, b_xyz=b.T)
    assert np.array_equal(dr, oracle.count3d(oracle.DR, b.T, edges, b_xyz=a.T))
    ab = np.concatenate([a, b])
    assert np.array_equal(oracle.count3d(oracle.DD, ab.T, edges), dd_a + dd_b + dr)
    assert int(dr.sum()) == 400 * 300 and int(dd_a.sum()) == 400 * 399 // 2
    # row ranges add up
    parts = sum(oracle.count3d(oracle.DD, a.T, edges, row_begin=r0, row_end=r1)
                for r0, r1 in ((0, 130), (130, 131), (131, 400)))
    assert np.array_equal(parts, dd_a)


def test_3d_region_counts_deletion_identity_and_pure_python():
    """3-D jackknife regions (slabs in x): total equals count3d; removing a
    region removes exactly its touch row (recounts of the reduced catalogs);
    a pure-Python loop with math.sqrt gives the same total and touch rows."""
    g = synthcat.rng_for(96, 3)
    a = g.uniform(0.0, 40.0, size=(300, 3))
    b = g.uniform(0.0, 40.0, size=(260, 3))
    nreg = 4
    ra_ = np.minimum((a[:, 0] // 10).astype(np.int32), nreg - 1)
    rb_ = np.minimum((b[:, 0] // 10).astype(np.int32), nreg - 1)
    e = synthcat.log_edges(0.5, 30.0, 9)
    dd_t, dd_touch = oracle.count_regions(oracle.DD, a.T, ra_, e, nreg, metric=1)
    dr_t, dr_touch = oracle.count_regions(oracle.DR, a.T, ra_, e, nreg, b_xyz=b.T, b_region=rb_, metric=1)
    assert np.array_equal(dd_t, oracle.count3d(oracle.DD, a.T, e))
    assert np.array_equal(dr_t, oracle.count3d(oracle.DR, a.T, e, b_xyz=b.T))
    for k in range(nreg):
        ka, kb = ra_ != k, rb_ != k
        assert np.array_equal(dd_t - dd_touch[k], oracle.count3d(oracle.DD, a[ka].T, e))
        assert np.array_equal(dr_t - dr_touch[k], oracle.count3d(oracle.DR, a[ka].T, e, b_xyz=b[kb].T))
    tot = np.zeros(e.size + 1, np.uint64)
    touch = np.zeros((nreg, e.size + 1), np.uint64)
    for i in range(a.shape[0]):
        for j in range(i + 1, a.shape[0]):
            dx, dy, dz = (float(a[i, c]) - float(a[j, c]) for c in range(3))
            s = sum(1 for t in e if t <= math.sqrt((dx * dx + dy * dy) + dz * dz))
            tot[s] += 1
            touch[ra_[i], s] += 1
            if ra_[j] != ra_[i]:
                touch[ra_[j], s] += 1
    assert np.array_equal(tot, dd_t) and np.array_equal(touch, dd_touch)


# --------------------------------------------------------------------------
# FP64 operation order of the rule.  The angle is the arc-cosine of the dot
# product (Section 3, first bullet), read as (x_i x_j + y_i y_j) + z_i z_j
# with each operation rounded and no FMA (the paper's CPU in Table 1 has
# none); the 3-D squared distance likewise.  The probes are pairs where a
# fused, reordered or correctly rounded evaluation gives another angle, with
# edges placed between the two, and the expected values come from exact
# rational arithmetic rounded after each operation (tests/rounding_probes.py).
# --------------------------------------------------------------------------

ORDERS = ("fma_xy_then_add_z", "fma_yx_then_add_z", "add_xy_then_fma_z", "fma_chain_x_y_z",
          "fma_chain_y_x_z", "x_plus_yz", "xz_plus_y", "correctly_rounded")


def _sky_expected(a, b):
    return np.array([rp.angle_of(rp.dot_orders(a[i], b[i])["rule"]) for i in range(a.shape[0])])


def _box_expected(a, b):
    return np.array([math.sqrt(rp.d2_orders(a[i], b[i])["rule"]) for i in range(a.shape[0])])


def test_dot_product_order_is_pinned_by_probes():
    a, b, edges = rp.sky_probes()
    er = edges * DEG
    assert a.shape[0] == 40 and np.all(np.abs(a) >= 0.05) and np.all(np.abs(b) >= 0.05)
    # the oracle's angles are the rule's, bit for bit
    assert np.array_equal(oracle.pair_angles(a.T, b.T), _sky_expected(a, b))
    slots = oracle.pair_slots(a.T, b.T, edges)
    rule = np.array([rp.slot(t, er) for t in _sky_expected(a, b)])
    assert np.array_equal(slots, rule)
    # every other order moves at least one probe to another bin
    for name in ORDERS:
        alt = np.array([rp.slot(rp.angle_of(rp.dot_orders(a[i], b[i])[name]), er)
                        for i in range(a.shape[0])])
        assert np.any(alt != rule), name
    # whole DR histogram of every cross pair
    pairs = [(i, j) for i in range(a.shape[0]) for j in range(b.shape[0])]
    exp = rp.expected_sky_hist(a, b, edges, pairs)
    assert np.array_equal(oracle.count(oracle.DR, a.T, edges, b_xyz=b.T), exp)
    assert not np.array_equal(rp.expected_sky_hist(a, b, edges, pairs, "fma_chain_x_y_z"), exp)


def test_squared_distance_order_is_pinned_by_probes():
    a, b, edges = rp.box_probes()
    assert np.array_equal(oracle.pair_distances(a.T, b.T), _box_expected(a, b))
    rule = np.array([rp.slot(r, edges) for r in _box_expected(a, b)])
    for name in ORDERS:
        alt = np.array([rp.slot(math.sqrt(rp.d2_orders(a[i], b[i])[name]), edges)
                        for i in range(a.shape[0])])
        assert np.any(alt != rule), name
    pairs = [(i, j) for i in range(a.shape[0]) for j in range(b.shape[0])]
    exp = rp.expected_box_hist(a, b, edges, pairs)
    assert np.array_equal(oracle.count3d(oracle.DR, a.T, edges, b_xyz=b.T), exp)


def _has_fma_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            return " fma " in f.read().replace("\n", " ")
    except OSError:
        return False


def _planted_oracle(tmp_path, how):
    """A copy of the C oracle with the rounding order broken: `fma_call`
    rewrites the dot product and the squared distance with fma(); `contracted`
    builds the unchanged source with contraction on and FMA instructions."""
    import ctypes
    import subprocess
    with open(os.path.join(os.path.dirname(oracle.__file__), "tpcf_oracle.c")) as f:
        src = f.read()
    flags = ["-ffp-contract=off"]
    if how == "fma_call":
        for old, new in (("double d = (xi * xj + yi * yj) + zi * zj;",
                          "double d = fma(zi, zj, fma(yi, yj, xi * xj));"),
                         ("double d2 = (dx * dx + dy * dy) + dz * dz;",
                          "double d2 = fma(dz, dz, fma(dy, dy, dx * dx));")):
            assert old in src
            src = src.replace(old, new)
    else:
        flags = ["-ffp-contract=fast", "-mfma"]
    c = tmp_path / "planted.c"
    c.write_text(src)
    so = tmp_path / "planted.so"
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", *flags, "-fno-fast-math", "-fno-builtin", "-fPIC",
                           "-shared", "-pthread", str(c), "-o", str(so), "-lm"])
    lib = ctypes.CDLL(str(so))
    P, i64 = ctypes.c_void_p, ctypes.c_int64
    for fn in (lib.oracle_pair_angles, lib.oracle_pair_distances):
        fn.argtypes = [i64, P, P, P, P, P, P, P]
        fn.restype = ctypes.c_int
    return lib


def _call_pairs(fn, a, b):
    cols = [np.ascontiguousarray(a[:, c]) for c in range(3)] + \
           [np.ascontiguousarray(b[:, c]) for c in range(3)]
    out = np.empty(a.shape[0])
    fn(a.shape[0], *[v.ctypes.data for v in cols], out.ctypes.data)
    return out


@pytest.mark.parametrize("how", ["fma_call", "contracted"])
def test_rounding_order_pins_catch_a_fused_oracle(tmp_path, how):
    """Planted mistake: an oracle whose dot product and squared distance use
    fused multiply-adds (by an fma() call, or by building the same source with
    contraction on) fails the probes above."""
    if how == "contracted" and not _has_fma_cpu():
        pytest.skip("host CPU has no FMA instructions")
    lib = _planted_oracle(tmp_path, how)
    a, b, edges = rp.sky_probes()
    assert not np.array_equal(_call_pairs(lib.oracle_pair_angles, a, b), _sky_expected(a, b))
    a, b, edges = rp.box_probes()
    assert not np.array_equal(_call_pairs(lib.oracle_pair_distances, a, b), _box_expected(a, b))
