"""CPU oracle for angular two-point pair counting -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
and never imports it.

Contents
  * ``radec_to_xyz``, ``count``, ``pair_slots``, ``pair_angles``: thin ctypes
    wrappers over ``tpcf_oracle.c`` (plain FP64 double loops, libm acos).
  * ``landy_szalay``: the Landy-Szalay estimator (paper Eq. 1) written out in
    FP64 numpy.
  * ``count3d``, ``pair_distances``: the same counting by 3-D distance of
    Cartesian points (FP64 differences, libm sqrt).
  * ``count_regions``: counts plus, per jackknife region, the pairs with a
    member in it; ``jackknife``: delete-one jackknife of w by recounting the
    catalogs with each region removed.
  * ``tiny``: a pure-Python loop version of the counting for small inputs.

Every function is pinned by ``tests/test_oracle_pins.py`` against closed forms,
invariants and constructed geometries, not against itself.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tpcf_oracle.c")
_LIB = os.path.join(_HERE, "libtpcf_oracle.so")
_lib = None

DD, DR, RR = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the C oracle with contraction and fast-math off, and with the
    math builtins off so sin and cos stay separate libm calls (gcc would
    otherwise merge them into sincos, which can differ in the last bit)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fno-builtin",
            "-fPIC", "-shared", "-pthread", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_radec_to_xyz.argtypes = [i64, P, P, P, P, P]
        lib.oracle_radec_to_xyz.restype = None
        lib.oracle_count.argtypes = [ctypes.c_int, i64, P, P, P, i64, P, P, P,
                                     ctypes.c_int32, P, i64, i64, ctypes.c_int, P]
        lib.oracle_count.restype = ctypes.c_int
        lib.oracle_pair_slots.argtypes = [i64, P, P, P, P, P, P, ctypes.c_int32, P, P]
        lib.oracle_pair_slots.restype = ctypes.c_int
        lib.oracle_pair_angles.argtypes = [i64, P, P, P, P, P, P, P]
        lib.oracle_pair_angles.restype = ctypes.c_int
        lib.oracle_count3d.argtypes = [ctypes.c_int, i64, P, P, P, i64, P, P, P,
                                       ctypes.c_int32, P, i64, i64, ctypes.c_int, P]
        lib.oracle_count3d.restype = ctypes.c_int
        lib.oracle_pair_distances.argtypes = [i64, P, P, P, P, P, P, P]
        lib.oracle_pair_distances.restype = ctypes.c_int
        lib.oracle_count_regions.argtypes = [ctypes.c_int, i64, P, P, P, P, i64, P, P, P, P,
                                             ctypes.c_int32, P, ctypes.c_int32, P, P]
        lib.oracle_count_regions.restype = ctypes.c_int
        lib.oracle_count_regions3d.argtypes = lib.oracle_count_regions.argtypes
        lib.oracle_count_regions3d.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    """Host threads for the row loop: the cores this process may run on,
    at most OMP_NUM_THREADS when that is set (a shared machine's share of
    cores), and at most 64."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    try:
        cap = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        cap = 0
    if cap > 0:
        n = min(n, cap)
    return max(1, min(n, 64))


def radec_to_xyz(ra_deg, dec_deg):
    """Unit vectors (x, y, z) from RA/Dec in degrees (FP64, host libm)."""
    ra, dec = _f64(ra_deg), _f64(dec_deg)
    n = ra.size
    x, y, z = (np.empty(n, np.float64) for _ in range(3))
    _load().oracle_radec_to_xyz(n, _ptr(ra), _ptr(dec), _ptr(x), _ptr(y), _ptr(z))
    return x, y, z


def count(kind: int, a_xyz, edges_deg, b_xyz=None, row_begin: int = -1,
          row_end: int = -1, nthreads: int | None = None) -> np.ndarray:
    """Histogram of pair angles, nbins+2 uint64 slots
    [theta < e_0, bins 0..nbins-1, theta >= e_nbins].

    kind DD or RR: unordered pairs i < j of ``a_xyz`` (rows i restricted to
    [row_begin, row_end) when given).  kind DR: all pairs (i, j) with i a row
    of ``a_xyz`` and j in ``b_xyz``."""
    edges = _f64(edges_deg)
    nbins = edges.size - 1
    ax, ay, az = (_f64(c) for c in a_xyz)
    if kind == DR:
        if b_xyz is None:
            raise ValueError("DR needs a second catalog")
        bx, by, bz = (_f64(c) for c in b_xyz)
        cross = 1
    else:
        if b_xyz is not None:
            raise ValueError("DD/RR take one catalog")
        bx, by, bz = ax, ay, az
        cross = 0
    out = np.zeros(nbins + 2, dtype=np.uint64)
    rc = _load().oracle_count(cross, ax.size, _ptr(ax), _ptr(ay), _ptr(az), bx.size,
                              _ptr(bx), _ptr(by), _ptr(bz), nbins, _ptr(edges),
                              row_begin, row_end, nthreads or default_threads(), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_count rejected its arguments")
    return out


def count3d(kind: int, a_xyz, edges, b_xyz=None, row_begin: int = -1,
            row_end: int = -1, nthreads: int | None = None) -> np.ndarray:
    """Histogram of 3-D pair distances, nbins+2 uint64 slots
    [r < e_0, bins 0..nbins-1, r >= e_nbins]; points are Cartesian
    coordinates and edges distances in the same unit.  Pairs as ``count``."""
    e = _f64(edges)
    nbins = e.size - 1
    ax, ay, az = (_f64(c) for c in a_xyz)
    if kind == DR:
        if b_xyz is None:
            raise ValueError("DR needs a second catalog")
        bx, by, bz = (_f64(c) for c in b_xyz)
        cross = 1
    else:
        if b_xyz is not None:
            raise ValueError("DD/RR take one catalog")
        bx, by, bz = ax, ay, az
        cross = 0
    out = np.zeros(nbins + 2, dtype=np.uint64)
    rc = _load().oracle_count3d(cross, ax.size, _ptr(ax), _ptr(ay), _ptr(az), bx.size,
                                _ptr(bx), _ptr(by), _ptr(bz), nbins, _ptr(e),
                                row_begin, row_end, nthreads or default_threads(), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_count3d rejected its arguments")
    return out


def pair_distances(a_xyz, b_xyz) -> np.ndarray:
    """3-D distance of each listed pair (a_i, b_i)."""
    ax, ay, az = (_f64(c) for c in a_xyz)
    bx, by, bz = (_f64(c) for c in b_xyz)
    out = np.empty(ax.size, dtype=np.float64)
    _load().oracle_pair_distances(ax.size, _ptr(ax), _ptr(ay), _ptr(az), _ptr(bx),
                                  _ptr(by), _ptr(bz), _ptr(out))
    return out


def pair_slots(a_xyz, b_xyz, edges_deg) -> np.ndarray:
    """Output slot of each listed pair (a_i, b_i)."""
    edges = _f64(edges_deg)
    ax, ay, az = (_f64(c) for c in a_xyz)
    bx, by, bz = (_f64(c) for c in b_xyz)
    out = np.empty(ax.size, dtype=np.int32)
    rc = _load().oracle_pair_slots(ax.size, _ptr(ax), _ptr(ay), _ptr(az), _ptr(bx),
                                   _ptr(by), _ptr(bz), edges.size - 1, _ptr(edges), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_pair_slots rejected its arguments")
    return out


def pair_angles(a_xyz, b_xyz) -> np.ndarray:
    """Angle in radians of each listed pair (a_i, b_i)."""
    ax, ay, az = (_f64(c) for c in a_xyz)
    bx, by, bz = (_f64(c) for c in b_xyz)
    out = np.empty(ax.size, dtype=np.float64)
    _load().oracle_pair_angles(ax.size, _ptr(ax), _ptr(ay), _ptr(az), _ptr(bx),
                               _ptr(by), _ptr(bz), _ptr(out))
    return out


def landy_szalay(dd, dr, rr, n_d: int, n_r: int, form: int = 0) -> np.ndarray:
    """Landy-Szalay estimator per bin (paper Eq. 1), FP64.

    The three arrays are taken bin by bin (pass the in-range bins, or whole
    slot arrays), with DD and RR counting unordered pairs.

    form 0 (default): each count is normalised by its number of pairs,
        n_DD = N_D (N_D - 1) / 2, n_DR = N_D N_R, n_RR = N_R (N_R - 1) / 2,
        w = (DD/n_DD - 2 DR/n_DR + RR/n_RR) / (RR/n_RR).
    form 1: Eq. 1 as printed, with its garbled "2" read as a square and DD and
        RR doubled to ordered-pair counts:
        w = 1 + (N_R/N_D)^2 (2 DD)/(2 RR) - 2 (N_R/N_D) DR/(2 RR).
    A bin with RR = 0 gives NaN.
    """
    dd = np.asarray(dd, dtype=np.float64)
    dr = np.asarray(dr, dtype=np.float64)
    rr = np.asarray(rr, dtype=np.float64)
    if dd.shape != dr.shape or dd.shape != rr.shape:
        raise ValueError("DD, DR and RR must have the same length")
    nd = float(n_d)
    nr = float(n_r)
    w = np.empty(dd.shape, dtype=np.float64)
    for k in range(dd.size):
        if rr[k] == 0.0:
            w[k] = np.nan
            continue
        if form == 0:
            n_dd = nd * (nd - 1.0) / 2.0
            n_dr = nd * nr
            n_rr = nr * (nr - 1.0) / 2.0
            fdd = dd[k] / n_dd
            fdr = dr[k] / n_dr
            frr = rr[k] / n_rr
            w[k] = (fdd - 2.0 * fdr + frr) / frr
        elif form == 1:
            ratio = nr / nd
            w[k] = 1.0 + ratio * ratio * (2.0 * dd[k]) / (2.0 * rr[k]) \
                - 2.0 * ratio * dr[k] / (2.0 * rr[k])
        else:
            raise ValueError("form must be 0 or 1")
    return w


def count_regions(kind: int, a_xyz, a_region, edges_deg, nreg: int, b_xyz=None, b_region=None,
                  metric: int = 0):
    """(total, touch): total as ``count`` (``count3d`` with metric 1, edges
    then distances); touch[r] counts the pairs with at least one member in
    region r (once for a pair inside one region)."""
    edges = _f64(edges_deg)
    nbins = edges.size - 1
    ax, ay, az = (_f64(c) for c in a_xyz)
    ra = np.ascontiguousarray(a_region, dtype=np.int32)
    if kind == DR:
        bx, by, bz = (_f64(c) for c in b_xyz)
        rb = np.ascontiguousarray(b_region, dtype=np.int32)
        cross = 1
    else:
        bx, by, bz, rb = ax, ay, az, ra
        cross = 0
    total = np.zeros(nbins + 2, dtype=np.uint64)
    touch = np.zeros((nreg, nbins + 2), dtype=np.uint64)
    fn = _load().oracle_count_regions3d if metric else _load().oracle_count_regions
    rc = fn(cross, ax.size, _ptr(ax), _ptr(ay), _ptr(az), _ptr(ra), bx.size, _ptr(bx), _ptr(by), _ptr(bz),
            _ptr(rb), nbins, _ptr(edges), nreg, _ptr(total), _ptr(touch))
    if rc != 0:
        raise ValueError("oracle_count_regions rejected its arguments")
    return total, touch


def jackknife(d_xyz, d_region, r_xyz, r_region, edges_deg, nreg: int, form: int = 0, metric: int = 0):
    """Delete-one jackknife of the Landy-Szalay w: for every region r, w from
    the catalogs with region r removed (recounted), then
    cov = (K - 1) / K sum_r (w_r - mean)(w_r - mean)^T with K = nreg.
    Returns (samples [K, nbins], mean [nbins], cov [nbins, nbins])."""
    dx = [_f64(c) for c in d_xyz]
    rx = [_f64(c) for c in r_xyz]
    dreg = np.asarray(d_region)
    rreg = np.asarray(r_region)
    samples = []
    for r in range(nreg):
        kd = dreg != r
        kr = rreg != r
        d = [c[kd] for c in dx]
        rr_ = [c[kr] for c in rx]
        cnt = count3d if metric else count
        dd = cnt(DD, d, edges_deg)
        dr = cnt(DR, d, edges_deg, b_xyz=rr_)
        rr = cnt(RR, rr_, edges_deg)
        samples.append(landy_szalay(dd[1:-1], dr[1:-1], rr[1:-1], int(kd.sum()), int(kr.sum()), form))
    samples = np.array(samples)
    mean = samples.mean(axis=0)
    dev = samples - mean
    cov = (nreg - 1.0) / nreg * (dev.T @ dev)
    return samples, mean, cov
