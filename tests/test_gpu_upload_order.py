"""Stored row order of large catalogs (needs an MI355X).

The library prepares big catalogs on several host threads: each thread sorts
a chunk of Morton keys and the chunks are merged.  The key ends in the point
index, so the stored order must be the one a plain sort of (region, Morton
key, index) gives, whatever the chunking.  The expected order here is that
plain sort, computed with numpy from the key's definition: each unit-vector
component mapped to 21 bits as floor((c + 1) / 2 * (2^21 - 1)), the three
codes interleaved x, y, z from the lowest bit.
"""

import numpy as np
import pytest

import oracle
import paper_1204_6630_amd as tp

pytestmark = pytest.mark.gpu


def _code21(c):
    t = (c + 1.0) / 2.0 * 2097151.0
    t = np.where(t > 0.0, t, 0.0)
    return np.minimum(t, 2097151.0).astype(np.uint64)


def _spread3(v):
    out = np.zeros_like(v)
    for b in range(21):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
    return out


def _expected_order(x, y, z, region=None):
    key = _spread3(_code21(x)) | _spread3(_code21(y)) << np.uint64(1) | _spread3(_code21(z)) << np.uint64(2)
    idx = np.arange(x.size)
    reg = np.zeros(x.size, np.int64) if region is None else region.astype(np.int64)
    return np.lexsort((idx, key, reg))


def _coarse_sphere(n, seed):
    """Unit vectors on a coarse lattice of directions: many points share a
    Morton key, so ties are decided by the index."""
    g = np.random.default_rng(seed)
    v = np.round(g.normal(size=(3, n)) * 8.0) / 8.0
    v[0] += 1e-9                              # no zero vector
    v /= np.sqrt((v * v).sum(axis=0))
    return v[0].copy(), v[1].copy(), v[2].copy()


@pytest.fixture(scope="module")
def ctx():
    c = tp.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n", [1, 32767, 65536, 100003, 229377, 1_000_000])
def test_stored_order_is_the_plain_sort(ctx, n):
    x, y, z = _coarse_sphere(n, 11 + n)
    cid = ctx.upload_catalog_xyz(x, y, z)
    try:
        got = ctx.catalog_order(cid)
    finally:
        ctx.release_catalog(cid)
    np.testing.assert_array_equal(got, _expected_order(x, y, z))


@pytest.mark.parametrize("n", [65536, 229377])
def test_stored_order_with_regions(ctx, n):
    """RA/Dec upload with region labels: regions first, then the Morton key
    of the unit vectors (the oracle's, from the same host libm), then the
    index."""
    g = np.random.default_rng(5 + n)
    ra = np.round(g.uniform(0.0, 90.0, n), 1)          # coarse: repeated keys
    dec = np.round(np.degrees(np.arcsin(g.uniform(0.0, 1.0, n))), 1)
    reg = g.integers(0, 7, n).astype(np.int32)
    cid = ctx.upload_catalog_regions(ra, dec, reg, 7)
    try:
        got = ctx.catalog_order(cid)
        counts = ctx.catalog_regions(cid)
    finally:
        ctx.release_catalog(cid)
    np.testing.assert_array_equal(counts, np.bincount(reg, minlength=7))
    x, y, z = oracle.radec_to_xyz(ra, dec)
    np.testing.assert_array_equal(got, _expected_order(x, y, z, reg))
