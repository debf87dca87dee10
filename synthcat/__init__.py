"""Seeded synthetic galaxy and random catalogs.

This module produces inputs only: right ascension and declination in degrees
(FP64) and bin-edge arrays in degrees.  It holds none of the pair-counting
arithmetic (no unit vectors as seen by the counter, no dot products, no
arc-cosines, no binning).  Both the CPU oracle tests and the GPU path draw
their inputs from here and nowhere else.

The paper measures on the MICE mock galaxy catalogs (Section 4), which are not
available here.  The recipes below stand in for them: uniform random catalogs
over a patch of the sky, and clustered "data" catalogs made of Gaussian blobs
around uniformly drawn centres, optionally mixed with an unclustered
background.  Every generator takes a ``numpy.random.Generator`` (PCG64) so a
(family, stream) seed reproduces the same catalog bit for bit.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 12046630

# Sky footprints as (ra_lo, ra_hi, dec_lo, dec_hi) in degrees.  Points are
# uniform in RA and in sin(Dec) inside the footprint, i.e. uniform in area.
PATCH_30 = (0.0, 30.0, 0.0, 30.0)
OCTANT = (0.0, 90.0, 0.0, 90.0)


def rng_for(family: int, stream: int) -> np.random.Generator:
    """PCG64 generator for one (workload family, stream) pair.  Families are
    small integers, one per workload below (1 patch, 2 and 3 octant, 4
    batched, 5 serving, 30 box); tests draw from families of their own."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + 1000 * family + stream))


def log_edges(lo_deg: float, hi_deg: float, nbins: int) -> np.ndarray:
    """nbins+1 logarithmically spaced edges in degrees, with both ends exact."""
    if nbins < 1 or not (0.0 < lo_deg < hi_deg):
        raise ValueError("need nbins >= 1 and 0 < lo < hi")
    a, b = math.log10(lo_deg), math.log10(hi_deg)
    e = np.array([10.0 ** (a + k * (b - a) / nbins) for k in range(nbins + 1)],
                 dtype=np.float64)
    e[0] = lo_deg
    e[-1] = hi_deg
    return e


def uniform_patch(n: int, footprint, rng: np.random.Generator):
    """n points uniform in area over an RA x Dec footprint (degrees)."""
    ra0, ra1, de0, de1 = footprint
    ra = rng.uniform(ra0, ra1, size=n)
    s0, s1 = math.sin(math.radians(de0)), math.sin(math.radians(de1))
    dec = np.degrees(np.arcsin(rng.uniform(s0, s1, size=n)))
    return ra.astype(np.float64), dec.astype(np.float64)


def uniform_sphere(n: int, rng: np.random.Generator):
    """n points uniform over the whole sphere."""
    return uniform_patch(n, (0.0, 360.0, -90.0, 90.0), rng)


def _inside(ra, dec, footprint):
    ra0, ra1, de0, de1 = footprint
    return (ra >= ra0) & (ra < ra1) & (dec >= de0) & (dec < de1)


def _blob_offsets(cra, cdec, sigma_deg, rng):
    """Gaussian offsets in the tangent plane at each centre, projected back to
    the sphere; returns (ra, dec) in degrees."""
    a = np.radians(cra)
    d = np.radians(cdec)
    s = math.radians(sigma_deg)
    xi = rng.normal(0.0, s, size=a.shape)
    eta = rng.normal(0.0, s, size=a.shape)
    ca, sa, cd, sd = np.cos(a), np.sin(a), np.cos(d), np.sin(d)
    # centre, east and north basis vectors
    px = cd * ca - xi * sa - eta * sd * ca
    py = cd * sa + xi * ca - eta * sd * sa
    pz = sd + eta * cd
    r = np.sqrt(px * px + py * py + pz * pz)
    px, py, pz = px / r, py / r, pz / r
    ra = np.degrees(np.arctan2(py, px)) % 360.0
    dec = np.degrees(np.arcsin(np.clip(pz, -1.0, 1.0)))
    return ra, dec


def clustered(n: int, n_centres: int, sigma_deg: float, footprint,
              rng: np.random.Generator, centres=None):
    """n points in Gaussian blobs (angular sigma) around uniform centres.

    Each point picks its centre uniformly; points that land outside the
    footprint are redrawn (with a fresh centre) until all are inside.
    """
    if centres is None:
        cra, cdec = uniform_patch(n_centres, footprint, rng)
    else:
        cra, cdec = centres
    ra = np.empty(n, dtype=np.float64)
    dec = np.empty(n, dtype=np.float64)
    todo = np.arange(n)
    while todo.size:
        pick = rng.integers(0, cra.size, size=todo.size)
        r, d = _blob_offsets(cra[pick], cdec[pick], sigma_deg, rng)
        ok = _inside(r, d, footprint)
        ra[todo[ok]] = r[ok]
        dec[todo[ok]] = d[ok]
        todo = todo[~ok]
    return ra, dec


def grid_regions(ra, dec, footprint, n_ra: int, n_dec: int) -> np.ndarray:
    """Jackknife region labels (int32): the footprint cut into an n_ra x n_dec
    grid of equal RA and Dec steps, label = dec_cell * n_ra + ra_cell.  Points
    on or past the far edges fall into the last cell of each axis."""
    ra0, ra1, de0, de1 = footprint
    ia = np.clip(((np.asarray(ra) - ra0) / (ra1 - ra0) * n_ra).astype(np.int64), 0, n_ra - 1)
    idc = np.clip(((np.asarray(dec) - de0) / (de1 - de0) * n_dec).astype(np.int64), 0, n_dec - 1)
    return (idc * n_ra + ia).astype(np.int32)


@dataclass
class Catalog:
    ra: np.ndarray
    dec: np.ndarray

    @property
    def n(self) -> int:
        return int(self.ra.size)


@dataclass
class Workload:
    name: str
    data: list          # list[Catalog]
    randoms: list       # list[Catalog]
    edges_deg: np.ndarray
    extra: dict = field(default_factory=dict)


def patch30_1e4(scale: float = 1.0) -> Workload:
    """Small plain case: 1e4 clustered points (200 centres, sigma 0.5 deg) and
    1e4 uniform randoms on a 30x30 deg patch; 20 log bins over [0.01, 10] deg."""
    n = max(2, int(round(10_000 * scale)))
    g = rng_for(1, 0)
    d = clustered(n, 200, 0.5, PATCH_30, g)
    r = uniform_patch(n, PATCH_30, rng_for(1, 1))
    return Workload("patch30_1e4", [Catalog(*d)], [Catalog(*r)],
                    log_edges(0.01, 10.0, 20))


def octant_1e5(scale: float = 1.0) -> Workload:
    """1e5 clustered points (2000 centres, sigma 0.3 deg) and 1e5 uniform
    randoms over the octant; 30 log bins over [0.001, 20] deg."""
    n = max(2, int(round(100_000 * scale)))
    d = clustered(n, 2000, 0.3, OCTANT, rng_for(2, 0))
    r = uniform_patch(n, OCTANT, rng_for(2, 1))
    return Workload("octant_1e5", [Catalog(*d)], [Catalog(*r)],
                    log_edges(0.001, 20.0, 30))


def octant_1e6x2e6(scale: float = 1.0) -> Workload:
    """1e6 data points (70% in blobs around 20000 centres with sigma 0.2 deg,
    30% uniform background) and 2e6 uniform randoms over the octant; 40 log
    bins over [0.0005, 30] deg."""
    nd = max(2, int(round(1_000_000 * scale)))
    nr = max(2, int(round(2_000_000 * scale)))
    g = rng_for(3, 0)
    ncl = int(round(0.7 * nd))
    a = clustered(ncl, 20000, 0.2, OCTANT, g)
    b = uniform_patch(nd - ncl, OCTANT, g)
    ra = np.concatenate([a[0], b[0]])
    dec = np.concatenate([a[1], b[1]])
    perm = g.permutation(nd)
    r = uniform_patch(nr, OCTANT, rng_for(3, 1))
    return Workload("octant_1e6x2e6", [Catalog(ra[perm], dec[perm])],
                    [Catalog(*r)], log_edges(0.0005, 30.0, 40))


def batched_64(n_catalogs: int = 64, scale: float = 1.0) -> Workload:
    """64 data catalogs of log-uniform size in [5e3, 5e5], clustered (50 points
    per centre, sigma 0.3 deg) inside a random 20x20 deg sub-patch of the
    octant each, against one 1e6-point uniform octant random catalog; 30 log
    bins over [0.001, 20] deg."""
    g = rng_for(4, 0)
    data = []
    for _ in range(n_catalogs):
        n = int(round(math.exp(g.uniform(math.log(5e3), math.log(5e5))) * scale))
        n = max(2, n)
        a0 = g.uniform(0.0, 70.0)
        d0 = g.uniform(0.0, 70.0)
        fp = (a0, a0 + 20.0, d0, d0 + 20.0)
        data.append(Catalog(*clustered(n, max(1, n // 50), 0.3, fp, g)))
    nr = max(2, int(round(1_000_000 * scale)))
    r = uniform_patch(nr, OCTANT, rng_for(4, 1))
    return Workload("batched_64", data, [Catalog(*r)],
                    log_edges(0.001, 20.0, 30))


def serving_jobs(n_jobs: int = 2000, size_lo: int = 1000, size_hi: int = 1_000_000,
                 seed_stream: int = 0):
    """Job stream for the serving case: kinds DD/DR/RR with mix 40/40/20,
    catalog sizes log-uniform in [size_lo, size_hi], clustered (50 points per
    centre, sigma 0.3 deg) or uniform over the octant with probability 1/2
    each; DR and RR jobs name one of three resident random catalogs.
    Returns a list of dicts; catalogs are generated lazily by
    :func:`serving_catalog`."""
    g = rng_for(5, seed_stream)
    jobs = []
    for j in range(n_jobs):
        u = g.uniform()
        kind = "DD" if u < 0.4 else ("DR" if u < 0.8 else "RR")
        n = int(round(math.exp(g.uniform(math.log(size_lo), math.log(size_hi)))))
        jobs.append({"id": j, "kind": kind, "n": max(2, n),
                     "clustered": bool(g.uniform() < 0.5),
                     "random": int(g.integers(0, 3)),
                     "seed": int(g.integers(0, 2**62))})
    return jobs


def serving_catalog(job) -> Catalog:
    g = np.random.Generator(np.random.PCG64(job["seed"]))
    if job["clustered"]:
        return Catalog(*clustered(job["n"], max(1, job["n"] // 50), 0.3, OCTANT, g))
    return Catalog(*uniform_patch(job["n"], OCTANT, g))


def serving_randoms(n: int = 2_000_000):
    return [Catalog(*uniform_patch(n, OCTANT, rng_for(5, 100 + r))) for r in range(3)]


# --- 3-D boxes (the spatial variant xi(r)) ----------------------------------

@dataclass
class Box:
    """Cartesian points (comoving coordinates, e.g. Mpc/h), float64."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray

    @property
    def n(self) -> int:
        return int(self.x.size)

    def xyz(self):
        return self.x, self.y, self.z


def box_uniform(n: int, side: float, rng: np.random.Generator, origin: float = 0.0) -> Box:
    """n points uniform in the cube [origin, origin + side)^3."""
    p = rng.uniform(origin, origin + side, size=(3, n))
    return Box(p[0].copy(), p[1].copy(), p[2].copy())


def box_clustered(n: int, n_centres: int, sigma: float, side: float, rng: np.random.Generator,
                  origin: float = 0.0) -> Box:
    """n points in isotropic Gaussian blobs (per-axis sigma) around uniform
    centres in the cube; points outside the cube are redrawn."""
    c = rng.uniform(origin, origin + side, size=(n_centres, 3))
    out = np.empty((n, 3), dtype=np.float64)
    todo = np.arange(n)
    while todo.size:
        pick = rng.integers(0, n_centres, size=todo.size)
        p = c[pick] + rng.normal(0.0, sigma, size=(todo.size, 3))
        ok = np.all((p >= origin) & (p < origin + side), axis=1)
        out[todo[ok]] = p[ok]
        todo = todo[~ok]
    return Box(out[:, 0].copy(), out[:, 1].copy(), out[:, 2].copy())


@dataclass
class Workload3d:
    name: str
    data: Box
    randoms: Box
    edges: np.ndarray


def box_1e6x2e6(scale: float = 1.0, side: float = 1000.0) -> Workload3d:
    """3-D analogue of the 1e6 x 2e6 octant workload: 1e6 data points (70% in blobs around 20000
    centres with per-axis sigma 2, 30% uniform) and 2e6 uniform randoms in a
    box of side 1000 (Mpc/h); 30 log bins over [0.5, 150]."""
    nd = max(2, int(round(1_000_000 * scale)))
    nr = max(2, int(round(2_000_000 * scale)))
    g = rng_for(30, 0)
    ncl = int(round(0.7 * nd))
    a = box_clustered(ncl, max(1, int(round(20000 * scale))), 2.0, side, g)
    b = box_uniform(nd - ncl, side, g)
    perm = g.permutation(nd)
    d = Box(*(np.concatenate([u, v])[perm] for u, v in zip(a.xyz(), b.xyz())))
    r = box_uniform(nr, side, rng_for(30, 1))
    return Workload3d(f"box{int(side)}_{nd:.0e}x{nr:.0e}".replace("+0", ""), d, r, log_edges(0.5, 150.0, 30))


def near_limit_clusters(n_per: int = 1024, stream: int = 0):
    """Caller-given FP64 vectors (for the xyz entry point) whose squared norms
    deviate from 1 by 0.90 .. 0.95 x 2^-20, the largest deviation that entry
    accepts, in pairs of tight clusters (radius ~1e-6 rad) whose centres lie
    a few 1e-6 rad on either side of a bin edge.  A pair's dot product is then
    |a| |b| cos(phi), which moves its angle by up to ~1e-6 cot(phi): tens of
    1e-6 rad, far more than the clusters' distance from the edge, so binning
    the true directions instead of the given vectors puts these pairs in the
    wrong bin.  Squared norms are above 1 where the centres lie past the edge
    and below 1 where they lie short of it (both cross the edge); clusters
    short of an edge hold n_per / 2 points, the others n_per, so the two
    crossings do not cancel in a histogram.  Cluster pairs sit 30 deg apart,
    beyond the last edge of each other.
    Returns (a_xyz (3, 4.5 n_per), b_xyz (3, 4.5 n_per), edges_deg)."""
    g = rng_for(97, stream)
    limit = 2.0 ** -20
    edges = np.array([0.1, 0.5, 2.0, 5.0])
    specs = [(0.5, 5e-6, 1.0), (0.5, -5e-6, -1.0), (2.0, 4e-6, 1.0), (2.0, -4e-6, -1.0),
             (0.1, 3e-6, 1.0), (0.1, -3e-6, -1.0)]

    def tangent_basis(c):
        t = np.cross(c, [0.0, 0.0, 1.0] if abs(c[2]) < 0.9 else [1.0, 0.0, 0.0])
        t /= np.linalg.norm(t)
        return t, np.cross(c, t)

    def cluster(c, sign):
        n = n_per if sign > 0 else n_per // 2
        e1, e2 = tangent_basis(c)
        x = g.normal(0.0, 2e-7, size=(n, 1))
        y = g.normal(0.0, 2e-7, size=(n, 1))
        p = c[None, :] + x * e1[None, :] + y * e2[None, :]
        p /= np.linalg.norm(p, axis=1)[:, None]
        return p * np.sqrt(1.0 + sign * limit * g.uniform(0.90, 0.95, size=(n, 1)))

    A, B = [], []
    for k, (edge_deg, offset, sign) in enumerate(specs):
        ra, dec = math.radians(30.0 * k), math.radians(20.0)
        c = np.array([math.cos(dec) * math.cos(ra), math.cos(dec) * math.sin(ra), math.sin(dec)])
        e1, e2 = tangent_basis(c)
        phi = g.uniform(0.0, 2.0 * math.pi)
        t = math.cos(phi) * e1 + math.sin(phi) * e2
        theta = math.radians(edge_deg) + offset
        c2 = math.cos(theta) * c + math.sin(theta) * t
        A.append(cluster(c, sign))
        B.append(cluster(c2 / np.linalg.norm(c2), sign))
    a = np.concatenate(A).T.copy()
    b = np.concatenate(B).T.copy()
    return a, b, edges


WORKLOADS = {"patch30_1e4": patch30_1e4, "octant_1e5": octant_1e5,
             "octant_1e6x2e6": octant_1e6x2e6, "batched_64": batched_64}
