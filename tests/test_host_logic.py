"""CPU tests of libtpcf.so's host logic (no GPU needed).

* every symbol declared in include/tpcf.h is exported;
* edge thresholds D_k bracket the counting rule (checked with Python's
  math.acos, an independent caller of the same libm routine);
* FP32 chord^2 bands: pairs placed at theta = e_k (1 +- 10^-s) in random
  orientations; every decision the band calls certain agrees with the oracle;
* a numpy emulation of the kernels' table-driven classification (FP32 q and
  FP64 e = 1 - d, one lookup, threshold comparison in flagged cells, exact
  d <= D_k when still undecided) reproduces the oracle slot of every pair;
* Landy-Szalay and argument errors of host-only entry points.
"""

import math
import os
import re

import numpy as np
import pytest

import oracle
import paper_1204_6630_amd as tp
import synthcat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEG = math.pi / 180.0


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "tpcf.h")).read()
    declared = set(re.findall(r"^\s*(?:int|const char \*)\s*(tpcf_\w+)\s*\(", header, re.M))
    assert declared, "no declarations found"
    L = tp.lib()
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared == set(tp.EXPORTED_SYMBOLS)


def _next(d, n=1):
    for _ in range(abs(n)):
        d = np.nextafter(d, np.inf if n > 0 else -np.inf)
    return d


@pytest.mark.parametrize("edges", [
    synthcat.log_edges(0.01, 10.0, 20),
    synthcat.log_edges(0.0005, 30.0, 40),
    np.array([0.0, 1e-6, 0.1, 45.0, 89.0, 91.0, 135.0, 179.9, 180.0]),
])
def test_thresholds_bracket_the_rule(edges):
    D, _, _ = tp.compile_edges(edges)
    for k, e_deg in enumerate(edges):
        e = e_deg * DEG
        if e == 0.0:
            assert D[k] == np.inf
            continue
        if math.acos(-1.0) < e:
            assert D[k] == -np.inf
            continue
        assert -1.0 <= D[k] <= 1.0
        assert math.acos(D[k]) >= e
        if D[k] < 1.0:
            assert math.acos(_next(D[k])) < e
        for s in range(1, 40):
            lo = _next(D[k], -s)
            if lo >= -1.0:
                assert math.acos(lo) >= e
            hi = _next(D[k], s)
            if hi <= 1.0:
                assert math.acos(hi) < e
    finite = D[np.isfinite(D)]
    assert np.all(np.diff(finite) <= 0)


def test_edges_validation():
    with pytest.raises(tp.TpcfError):
        tp.compile_edges([1.0, 1.0, 2.0])
    with pytest.raises(tp.TpcfError):
        tp.compile_edges([1.0, 0.5])
    with pytest.raises(tp.TpcfError):
        tp.compile_edges([1.0, 181.0])
    with pytest.raises(tp.TpcfError):
        tp.compile_edges([-1.0, 1.0])
    with pytest.raises(tp.TpcfError):
        tp.compile_edges([1.0, np.nan])
    with pytest.raises(tp.TpcfError):
        tp.compile_edges([1.0])             # nbins = 0
    with pytest.raises(tp.TpcfError):
        tp.compile_edges(np.linspace(1, 2, 258))  # nbins = 257
    with pytest.raises(tp.TpcfError):
        tp.compile_edges([1.0, 2.0], delta_max=1e-3)


def _rand_perp(g, a):
    u = g.normal(size=a.shape)
    u -= np.sum(u * a, axis=1)[:, None] * a
    return u / np.linalg.norm(u, axis=1)[:, None]


def _pairs_at(g, theta):
    n = theta.size
    a = g.normal(size=(n, 3))
    a /= np.linalg.norm(a, axis=1)[:, None]
    u = _rand_perp(g, a)
    b = np.cos(theta)[:, None] * a + np.sin(theta)[:, None] * u
    b /= np.linalg.norm(b, axis=1)[:, None]
    return a, b


def _q32(a, b, q0=None):
    """Kernel arithmetic in FP32 (separate multiply and add; the band covers
    both this and the fused form).  With a floor q0 (the wrapped layout) the
    sum starts at q0."""
    fa = a.astype(np.float32)
    fb = b.astype(np.float32)
    d = fa - fb
    q = d[:, 0] * d[:, 0]
    if q0 is not None:
        q = q + np.float32(q0)
    q = q + d[:, 1] * d[:, 1]
    q = q + d[:, 2] * d[:, 2]
    return q.astype(np.float32)


def _q32_fused(a, b, q0):
    """The same with each step fused (one rounding): the product of two FP32
    values and the FP32 sum are exact in FP64 up to a final rounding that can
    only differ from the fused one by a double rounding, so this is checked
    with a band margin of two FP32 ulps elsewhere, not bit for bit."""
    d = (a.astype(np.float32) - b.astype(np.float32)).astype(np.float64)
    q = np.float32(d[:, 0] * d[:, 0] + np.float64(q0))
    q = np.float32(d[:, 1] * d[:, 1] + q.astype(np.float64))
    q = np.float32(d[:, 2] * d[:, 2] + q.astype(np.float64))
    return q


def _dot64(a, b):
    return (a[:, 0] * b[:, 0] + a[:, 1] * b[:, 1]) + a[:, 2] * b[:, 2]


@pytest.mark.parametrize("floored", [False, True])
@pytest.mark.parametrize("edges", [synthcat.log_edges(0.0005, 30.0, 40),
                                   synthcat.log_edges(0.001, 20.0, 30)])
def test_fp32_band_adversary(edges, floored):
    """P10: pairs at theta = e_k (1 +- 10^-s), s = 3..9, every edge; also for
    the wrapped layout's band, whose q is summed from the floor q0."""
    g = np.random.default_rng(7)
    D, qlo, qhi = tp.compile_edges(edges, delta_max=4.5e-16)
    q0 = None
    if floored:
        w = tp.compile_wrap32(edges, delta_max=4.5e-16)
        qlo, qhi, q0 = w["qlo"], w["qhi"], w["q0"]
    er = edges * DEG
    thetas, rel, edge_of = [], [], []
    for k, e in enumerate(er):
        for s in range(3, 10):
            for sign in (-1.0, 1.0):
                thetas.append(np.full(60, e * (1.0 + sign * 10.0 ** -s)))
                rel.append(np.full(60, 10.0 ** -s))
                edge_of.append(np.full(60, k))
    theta = np.concatenate(thetas)
    rel = np.concatenate(rel)
    edge_of = np.concatenate(edge_of)
    a, b = _pairs_at(g, theta)
    q = _q32(a, b, q0)
    d = _dot64(a, b)
    truth = oracle.pair_slots(a.T, b.T, edges)
    if floored:
        # the fused form (each step one rounding) against the same band
        qf = _q32_fused(a, b, q0)
        for k in range(edges.size):
            past = truth >= k + 1
            assert np.all(past[qf >= qhi[k]]) and not np.any(past[qf < qlo[k]]), k
    in_band = np.zeros(theta.size, bool)
    for k in range(edges.size):
        above = q >= qhi[k]
        below = q < qlo[k]
        # rule: past edge k  <=>  d <= D_k  <=>  slot >= k+1
        past = truth >= k + 1
        assert np.all(past[above]), k
        assert not np.any(past[below]), k
        assert np.array_equal(past, d <= D[k])
        in_band |= ~above & ~below & (edge_of == k)
    # tightness: the chord half-width is about a = 2^-23 plus ~5 ulp of q, so
    # in theta the band reaches a relative distance ~ 1.2e-7 / e_k + 6e-7
    half = 1.2e-7 / er[edge_of] + 6e-7
    assert not np.any(in_band & (rel > 3.0 * half))
    assert np.all(in_band[rel < 0.1 * half])


def _two_slot_decided(x, w):
    """The kernels' two-slot test, on the int32 bit patterns as they make
    it: a lane decides its pairs when every x lies above the pattern of
    -w (x >= 0 or x < -w), nothing for a NaN width.  Checked against the
    float form of the same condition."""
    x = np.asarray(x, np.float32)
    w = np.asarray(w, np.float32)
    nw = -w
    lim = np.where(np.isnan(nw), np.int32(np.iinfo(np.int32).max), nw.view(np.int32))
    dec = x.view(np.int32) > lim
    with np.errstate(invalid="ignore"):
        ref = ~np.isnan(w) & ((x >= 0) | (-x > w))
    assert np.array_equal(dec, ref)
    return dec


@pytest.mark.parametrize("edges", [synthcat.log_edges(0.0005, 30.0, 40),
                                   synthcat.log_edges(0.001, 20.0, 30),
                                   np.array([0.0, 1.0, 90.0, 180.0])])
def test_two_slot_decision_matches_the_band(edges):
    """The kernels' two-slot steps: for a pair whose slot is k or k+1, the
    FP32 difference x = fl(q - qhi_k) decides it when x >= 0 or
    -x > fl(qhi_k - qlo_k) (the kernels test both at once on the int32 bit
    patterns: x above -fl(qhi_k - qlo_k)), and then the sign of x gives the
    slot the FP64 rule gives.  Pairs at
    theta = e_k (1 +- 10^-s), s = 2..9, and spread between the neighbouring
    edges; band pairs are never decided, and most pairs are."""
    g = np.random.default_rng(11)
    D, qlo, qhi = tp.compile_edges(edges, delta_max=4.5e-16)
    er = edges * DEG
    thetas, ks = [], []
    for k, e in enumerate(er):
        for s in range(2, 10):
            for sign in (-1.0, 1.0):
                thetas.append(np.full(40, e * (1.0 + sign * 10.0 ** -s)))
                ks.append(np.full(40, k))
        lo = er[k - 1] if k else 0.5 * e
        hi = er[k + 1] if k + 1 < er.size else min(1.5 * e + 1e-3, math.pi)
        thetas.append(g.uniform(lo, hi, 400))
        ks.append(np.full(400, k))
    theta = np.clip(np.concatenate(thetas), 0.0, math.pi)
    k = np.concatenate(ks)
    a, b = _pairs_at(g, theta)
    q = _q32(a, b)
    truth = oracle.pair_slots(a.T, b.T, edges)
    ours = (truth == k) | (truth == k + 1)
    thr = qhi.astype(np.float32)[k]
    with np.errstate(invalid="ignore"):
        # an edge at 0 has qlo = qhi = -inf: the width is NaN and, as in the
        # kernel, no pair is decided by the comparison (the lookup settles it)
        width = qhi.astype(np.float32)[k] - qlo.astype(np.float32)[k]
        x = q - thr                                 # FP32, round to nearest
        decided = _two_slot_decided(x, width)
    slot = k + (x >= 0).astype(np.int64)
    assert np.array_equal(slot[ours & decided], truth[ours & decided])
    in_band = (q >= qlo[k]) & (q < qhi[k])
    assert not np.any(in_band & decided)
    assert decided[ours].mean() > 0.25


@pytest.mark.parametrize("precision", [tp.FP32_CHORD, tp.FP64])
def test_cell_slot_ranges_never_decrease(precision):
    """Each cell entry bounds the slots of its keys ([s, s] for a certain
    slot, [k, k+1] for one undecided edge); the kernels' one- and two-slot
    steps rely on both ends being non-decreasing along the table."""
    edges = synthcat.log_edges(0.0005, 30.0, 40)
    _, _, _, cells, _ = tp.compile_cells(edges, precision, delta_max=4.5e-16)
    c = cells.astype(np.int64)
    multi = c == 0xFFFF
    flag = (c & 0x8000) != 0
    lo = np.where(flag, c & 0x7FFF, c)
    hi = np.where(flag, (c & 0x7FFF) + 1, c)
    keep = ~multi
    assert np.all(np.diff(lo[keep]) >= 0) and np.all(np.diff(hi[keep]) >= 0)
    assert np.all(hi - lo <= 1)


def _p32(a, b, fused):
    """The FP32 dot product of the FP32 copies, with a separate multiply and
    add at each step, or (fused) each step rounded once: the products of
    two floats are exact in FP64, so the FP64 sum rounded to FP32 is one
    rounding up to a double rounding, which the screen's bound covers."""
    fa, fb = a.astype(np.float32), b.astype(np.float32)
    if not fused:
        p = fa[:, 0] * fb[:, 0]
        p = p + fa[:, 1] * fb[:, 1]
        return p + fa[:, 2] * fb[:, 2]
    da, db = fa.astype(np.float64), fb.astype(np.float64)
    p = np.float32(da[:, 0] * db[:, 0])
    p = np.float32(da[:, 1] * db[:, 1] + p.astype(np.float64))
    return np.float32(da[:, 2] * db[:, 2] + p.astype(np.float64))


@pytest.mark.parametrize("delta", [4.5e-16, 2.0 ** -21])
@pytest.mark.parametrize("edges", [synthcat.log_edges(0.0005, 30.0, 40),
                                   synthcat.log_edges(0.001, 20.0, 30),
                                   synthcat.log_edges(0.01, 120.0, 12),
                                   np.array([0.0, 1.0, 179.0])])
def test_dot_screen_never_screens_a_pair_before_the_last_edge(edges, delta):
    """The FP32 kernels' screen of steps beyond the last edge: p = fl32(f_i .
    f_j) <= p_beyond must imply that the FP64 rule puts the pair at or past
    the last edge.  Pairs at theta = e_last (1 +- 10^-s), s = 2..9, random
    orientations, norms perturbed by up to delta; separate and fused sums.
    Pairs a relative 1e-4 past the edge are screened (the screen is not
    vacuous)."""
    g = np.random.default_rng(21)
    p_beyond = tp.compile_screen(edges, delta_max=delta)
    e = edges[-1] * DEG
    thetas = [np.full(2000, e * (1.0 + sgn * 10.0 ** -s)) for s in range(2, 10) for sgn in (-1.0, 1.0)]
    theta = np.clip(np.concatenate(thetas), 0.0, math.pi)
    a, b = _pairs_at(g, theta)
    # squared norms within 1 +- delta (as the library's bound allows)
    a *= np.sqrt(1.0 + g.uniform(-delta, delta, size=theta.size))[:, None]
    b *= np.sqrt(1.0 + g.uniform(-delta, delta, size=theta.size))[:, None]
    truth = oracle.pair_slots(a.T, b.T, edges)
    last = edges.size          # the overflow slot
    for fused in (False, True):
        screened = _p32(a, b, fused) <= np.float32(p_beyond)
        assert np.all(truth[screened] == last), fused
    if 0.0 < edges[-1] < 179.0:
        far = theta > e * (1.0 + 1e-4)
        assert np.all((_p32(a, b, True) <= np.float32(p_beyond))[far])


def _slot_range(code):
    """[lo, hi] of cell codes (0xFFFF: several undecided edges -> None)."""
    c = code.astype(np.int64)
    flag = (c & 0x8000) != 0
    lo = np.where(flag, c & 0x7FFF, c)
    return lo, np.where(flag, lo + 1, lo), c == 0xFFFF


@pytest.mark.parametrize("delta", [4.5e-16, 2.0 ** -21])
@pytest.mark.parametrize("edges", [synthcat.log_edges(0.0005, 30.0, 40),
                                   synthcat.log_edges(0.001, 20.0, 30),
                                   synthcat.log_edges(0.01, 120.0, 12),
                                   np.array([0.0, 1.0, 179.0])])
def test_dot_path_decides_like_the_rule(edges, delta):
    """The angular FP32 kernels' dot-product path.  For p = fl32(f_i . f_j)
    (separate or fused roundings) and the key q' = fl32(2 - 2p) (negative read
    as +0): the cell of q' bounds the rule's slot; q' >= khi_k and q' < klo_k
    decide edge k as the rule does; p <= plo_k and p >= phi_k too; and the
    two-slot decision (x = fl(p - phi_k) with x >= 0 or -x > fl(phi_k -
    plo_k), the sign bit meaning past the edge) gives the rule's slot.  Pairs at
    theta = e_k (1 +- 10^-s), s = 2..9, and spread between the edges, with
    norms perturbed by up to delta; most pairs away from the edges are
    decided (the path is not vacuous)."""
    g = np.random.default_rng(31)
    t = tp.compile_dot(edges, delta_max=delta)
    er = edges * DEG
    thetas, ks, near = [], [], []
    for k, e in enumerate(er):
        for s_ in range(2, 10):
            for sgn in (-1.0, 1.0):
                thetas.append(np.full(30, e * (1.0 + sgn * 10.0 ** -s_)))
                ks.append(np.full(30, k))
                near.append(np.full(30, s_ >= 4))
        lo = er[k - 1] if k else 0.5 * e
        hi = er[k + 1] if k + 1 < er.size else min(1.5 * e + 1e-3, math.pi)
        thetas.append(g.uniform(lo, hi, 300))
        ks.append(np.full(300, k))
        near.append(np.zeros(300, bool))
    theta = np.clip(np.concatenate(thetas), 0.0, math.pi)
    k = np.concatenate(ks)
    near = np.concatenate(near)
    a, b = _pairs_at(g, theta)
    a *= np.sqrt(1.0 + g.uniform(-delta, delta, size=theta.size))[:, None]
    b *= np.sqrt(1.0 + g.uniform(-delta, delta, size=theta.size))[:, None]
    truth = oracle.pair_slots(a.T, b.T, edges)
    klo, khi = t["klo"][k], t["khi"][k]
    plo, phi = t["plo"][k], t["phi"][k]
    past = truth >= k + 1
    for fused in (False, True):
        p = _p32(a, b, fused)
        qd = np.float32(2.0 - 2.0 * p.astype(np.float64))     # one rounding of the exact 2 - 2p
        qd = np.where(qd.view(np.int32) < 0, np.float32(0.0), qd).astype(np.float32)
        key = (qd.view(np.uint32) >> np.uint32(t["shift"])).astype(np.int64)
        lo_s, hi_s, multi = _slot_range(t["cells"][np.clip(key, t["lo"], t["hi"]) - t["lo"]])
        assert np.all(((truth >= lo_s) & (truth <= hi_s)) | multi), fused
        assert np.all(past[qd >= khi]) and not np.any(past[qd < klo]), fused
        assert np.all(past[p <= plo]) and not np.any(past[p >= phi]), fused
        with np.errstate(invalid="ignore"):
            x = (p - phi).astype(np.float32)
            w = (phi - plo).astype(np.float32)
            decided = _two_slot_decided(x, w)
        two = (truth == k) | (truth == k + 1)
        got = np.where(x < 0, k + 1, k)
        assert np.array_equal(got[decided & two], truth[decided & two]), fused
        if 0.0 < edges[-1] < 179.0 and delta < 1e-10:
            far = ~near & (edges[k] >= 1.0)
            assert np.mean(decided[far]) > 0.9, fused
            assert np.mean(~multi[far]) > 0.9, fused


def test_dot_cell_slot_ranges_never_decrease():
    """The dot-product key's cells: both ends of the slot range are
    non-decreasing along the table (q' grows with the angle), as the
    one- and two-slot steps need."""
    t = tp.compile_dot(synthcat.log_edges(0.0005, 30.0, 40), delta_max=4.5e-16)
    lo, hi, multi = _slot_range(t["cells"])
    keep = ~multi
    assert np.all(np.diff(lo[keep]) >= 0) and np.all(np.diff(hi[keep]) >= 0)
    assert np.all(hi - lo <= 1)
    # the table reaches from the small angles (multi) to beyond the last edge
    assert multi[0] and lo[-1] == 41


def _emulate(a, b, edges, precision, delta, direct=None):
    """Numpy transcription of the kernels' per-pair classification."""
    D, qlo, qhi = tp.compile_edges(edges, delta_max=delta)
    shift, lo, hi, cells, E = tp.compile_cells(edges, precision, delta_max=delta, direct=direct)
    d = _dot64(a, b)
    if precision == tp.FP32_CHORD and direct:
        # wrapped layout: q summed from the floor, cell = key mod 2^w of the
        # table image, no clamp; the band is the floored one
        nb = edges.size - 1
        w = tp.compile_wrap32(edges, delta_max=delta, aux_bytes=_aux_bytes(nb))
        assert (w["shift"], w["lo"], w["hi"]) == (shift, lo, hi)
        qlo, qhi = w["qlo"], w["qhi"]
        q = _q32(a, b, w["q0"])
        key = (q.view(np.uint32) >> np.uint32(shift)).astype(np.int64)
        assert key.min() >= lo and key.max() <= hi
        img = w["image"][key & ((1 << w["wrap_bits"]) - 1)].astype(np.int64)
        # one-byte codes back to the 16-bit ones of compile_cells
        c = key - lo
        assert np.array_equal(np.where(img == 0xFF, 0xFFFF, np.where(img & 0x80, 0x8000 | (img & 0x7F), img)),
                              cells[c].astype(np.int64))
    elif precision == tp.FP32_CHORD:
        q = _q32(a, b)
        key = q.view(np.uint32) >> np.uint32(shift)
        c = np.clip(key.astype(np.int64), lo, hi) - lo
    else:
        e = 1.0 - d
        hiw = (e.view(np.uint64) >> np.uint64(32)).astype(np.uint32).view(np.int32)
        key = hiw.astype(np.int64) >> shift
        c = np.clip(key, lo, hi) - lo
    ent = cells[c].astype(np.int64)
    slot = ent.copy()
    flag = ent >= 0x8000
    exact = np.zeros(ent.shape, bool)
    for idx in np.nonzero(flag)[0]:
        en = ent[idx]
        if en != 0xFFFF:
            k = en & 0x7FFF
            if precision == tp.FP32_CHORD:
                if q[idx] < qlo[k]:
                    slot[idx] = k
                    continue
                if q[idx] >= qhi[k]:
                    slot[idx] = k + 1
                    continue
            else:
                if e[idx] > E[k]:
                    slot[idx] = k + 1
                    continue
                if e[idx] < E[k]:
                    slot[idx] = k
                    continue
            exact[idx] = True
            slot[idx] = k + (1 if d[idx] <= D[k] else 0)
        else:
            exact[idx] = True
            slot[idx] = int(np.sum(d[idx] <= D))
    return slot, flag, exact


def _aux_bytes(nbins, copies=16):
    """LDS bytes of the histograms and thresholds of a default launch (four
    wavefronts, `copies` histogram copies of nbins + 3 words, 48 bytes of
    thresholds per edge)."""
    nslots = nbins + 2
    allowed = 32 if nslots + 1 <= 48 else 16 if nslots + 1 <= 96 else 8 if nslots + 1 <= 192 else 4
    return 4 * (nslots + 1) * min(copies, allowed) * 4 + (nbins + 1) * 48


@pytest.mark.parametrize("nbins,budget", [(1, 32768), (20, 32768), (40, 32768), (125, 32768), (40, 31744),
                                          (60, 32768)])
def test_wrapped_table_layout(nbins, budget):
    """The wrapped table: keys of every reachable q (coincident points give
    q = q0, antipodal ones the largest q) lie in [lo, hi]; the image holds
    cell c at c mod 2^w and zeros elsewhere; the free piece for the
    histograms and thresholds misses every cell; the floor is a power of two
    at most a quarter of the smallest positive threshold."""
    edges = synthcat.log_edges(0.0005, 30.0, nbins)
    aux = _aux_bytes(nbins)
    w = tp.compile_wrap32(edges, delta_max=4.5e-16, max_bytes=budget, aux_bytes=aux)
    size = 1 << w["wrap_bits"]
    assert max(size, w["aux_off"] + aux) <= budget and w["image"].size == size
    q0 = float(w["q0"])
    assert np.frexp(q0)[0] == 0.5
    _, qlo0, qhi0 = tp.compile_edges(edges, delta_max=4.5e-16)
    pos = np.concatenate([qlo0[qlo0 > 0], qhi0[qhi0 > 0]])
    assert 2.0 ** -100 <= q0 <= pos.min() / 4
    lo, hi = w["lo"], w["hi"]
    if w["aux_off"] >= size:
        assert w["aux_off"] == size and hi - lo + 1 <= size     # the free bytes follow the table
    else:
        assert hi - lo + 1 + aux <= size
    arc = np.arange(lo, hi + 1) & (size - 1)
    assert np.unique(arc).size == arc.size
    free = np.ones(size, bool)
    free[arc] = False
    assert w["aux_off"] % 16 == 0 and np.all(free[w["aux_off"]:w["aux_off"] + aux])
    assert np.all(w["image"][free] == 0)
    _, clo, chi, cells, _ = tp.compile_cells(edges, tp.FP32_CHORD, delta_max=4.5e-16, direct=True,
                                             max_cells=budget)
    assert (clo, chi) == (lo, hi)
    img = w["image"][arc].astype(np.int64)
    assert np.array_equal(np.where(img == 0xFF, 0xFFFF, np.where(img & 0x80, 0x8000 | (img & 0x7F), img)),
                          cells.astype(np.int64))
    g = np.random.default_rng(nbins)
    a = g.normal(size=(4000, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = np.concatenate([a[:1000], -a[1000:2000], g.normal(size=(2000, 3))])
    b[2000:] /= np.linalg.norm(b[2000:], axis=1, keepdims=True)
    for q in (_q32(a, b, w["q0"]), _q32_fused(a, b, w["q0"])):
        key = q.view(np.uint32) >> np.uint32(w["shift"])
        assert key.min() >= lo and key.max() <= hi
    assert np.all(_q32(a[:1000], b[:1000], w["q0"]) == np.float32(q0))


@pytest.mark.parametrize("precision,direct", [(tp.FP32_CHORD, True), (tp.FP32_CHORD, False),
                                              (tp.FP64, False)])
@pytest.mark.parametrize("cfg,scale", [("patch30_1e4", 0.06), ("octant_1e5", 0.006),
                                       ("octant_1e6x2e6", 0.0006)])
def test_emulated_classification_matches_oracle(cfg, scale, precision, direct):
    wl = synthcat.WORKLOADS[cfg](scale=scale)
    d = wl.data[0]
    r = wl.randoms[0]
    xa = np.stack(oracle.radec_to_xyz(d.ra, d.dec), axis=1)
    xb = np.stack(oracle.radec_to_xyz(r.ra, r.dec), axis=1)
    ia, ib = np.triu_indices(xa.shape[0], k=1)
    a = np.concatenate([xa[ia], xa[:, None, :].repeat(xb.shape[0], 1).reshape(-1, 3)])
    b = np.concatenate([xa[ib], np.tile(xb, (xa.shape[0], 1))])
    delta = 4.5e-16
    slot, flag, exact = _emulate(a, b, wl.edges_deg, precision, delta, direct)
    truth = oracle.pair_slots(a.T, b.T, wl.edges_deg)
    assert np.array_equal(slot, truth)
    assert flag.mean() < 0.05


def test_emulation_on_exact_dot_probes():
    """P1 on the CPU: i = (1,0,0), j = (d, sqrt(1-d^2), 0) has FP64 dot d
    exactly; d in {D_k, next up, next down} for every edge."""
    edges = synthcat.log_edges(0.01, 10.0, 20)
    D, _, _ = tp.compile_edges(edges)
    ds = []
    for Dk in D:
        ds += [Dk, _next(Dk, 1), _next(Dk, -1)]
    ds = np.array([x for x in ds if -1.0 <= x <= 1.0])
    a = np.tile([1.0, 0.0, 0.0], (ds.size, 1))
    b = np.stack([ds, np.sqrt(1.0 - ds * ds), np.zeros_like(ds)], axis=1)
    assert np.array_equal(_dot64(a, b), ds)
    truth = oracle.pair_slots(a.T, b.T, edges)
    for prec, direct in ((tp.FP32_CHORD, True), (tp.FP32_CHORD, False), (tp.FP64, False)):
        # the probe vectors' norms deviate from 1 by a few ulps
        n2 = np.sum(b * b, axis=1)
        delta = float(np.max(np.abs(n2 - 1.0))) + 4 * 2.0 ** -53
        slot, _, _ = _emulate(a, b, edges, prec, delta, direct)
        assert np.array_equal(slot, truth)


def test_landy_szalay_library_matches_oracle():
    g = np.random.default_rng(3)
    nb = 25
    dd = g.integers(0, 10**9, size=nb + 2).astype(np.uint64)
    dr = g.integers(0, 10**9, size=nb + 2).astype(np.uint64)
    rr = g.integers(1, 10**9, size=nb + 2).astype(np.uint64)
    rr[5] = 0
    for form in (0, 1):
        w = tp.landy_szalay(dd, dr, rr, 123457, 234567, form)
        ref = oracle.landy_szalay(dd[1:-1], dr[1:-1], rr[1:-1], 123457, 234567, form)
        fin = np.isfinite(ref)
        assert np.array_equal(np.isnan(w), np.isnan(ref))
        assert np.all(np.abs(w[fin] - ref[fin]) <= 1e-12 * np.maximum(1.0, np.abs(ref[fin])))


def test_landy_szalay_argument_errors():
    z = np.zeros(5, np.uint64)
    with pytest.raises(tp.TpcfError) as ei:
        tp.landy_szalay(z, z, z, 1, 10)
    assert ei.value.code == -1
    with pytest.raises(tp.TpcfError):
        tp.landy_szalay(z, z, z, 10, 10, form=2)


def test_open_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(tp.TpcfError):
        tp.Context(0)


def test_host_jackknife_equals_oracle_recount():
    """tpcf_jackknife on oracle region counts against the oracle's delete-one
    jackknife by recount of the reduced catalogs (an independent route:
    removing points and counting again)."""
    g = synthcat.rng_for(94, 0)
    patch = (0.0, 16.0, 0.0, 16.0)
    ra_d, dec_d = synthcat.uniform_patch(350, patch, g)
    ra_r, dec_r = synthcat.uniform_patch(420, patch, g)
    nreg = 6
    reg_d = synthcat.grid_regions(ra_d, dec_d, patch, 3, 2)
    reg_r = synthcat.grid_regions(ra_r, dec_r, patch, 3, 2)
    d = oracle.radec_to_xyz(ra_d, dec_d)
    r = oracle.radec_to_xyz(ra_r, dec_r)
    e = synthcat.log_edges(0.5, 10.0, 7)
    dd = oracle.count_regions(oracle.DD, d, reg_d, e, nreg)
    dr = oracle.count_regions(oracle.DR, d, reg_d, e, nreg, b_xyz=r, b_region=reg_r)
    rr = oracle.count_regions(oracle.RR, r, reg_r, e, nreg)
    nd_reg = np.bincount(reg_d, minlength=nreg)
    nr_reg = np.bincount(reg_r, minlength=nreg)
    for form in (0, 1):
        s, m, c = tp.jackknife(dd[0], dd[1], dr[0], dr[1], rr[0], rr[1], 350, nd_reg, 420, nr_reg, form)
        so, mo, co = oracle.jackknife(d, reg_d, r, reg_r, e, nreg, form)
        assert np.array_equal(np.isnan(s), np.isnan(so))
        np.testing.assert_allclose(s, so, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(m, mo, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(c, co, rtol=1e-10, atol=1e-18)


def test_host_jackknife_argument_errors():
    z = np.zeros(5, np.uint64)
    t = np.zeros((3, 5), np.uint64)
    n = np.ones(3, np.int64)
    with pytest.raises(ValueError):
        tp.jackknife(z, t, z, t, z, t, 10, np.ones(2, np.int64), 10, n)
    with pytest.raises(tp.TpcfError):
        tp.jackknife(z, t, z, t, z, t, 10, n, 10, n, form=2)
    one = np.zeros((1, 5), np.uint64)
    with pytest.raises(tp.TpcfError):   # a single region has no jackknife
        tp.jackknife(z, one, z, one, z, one, 10, np.ones(1, np.int64), 10, np.ones(1, np.int64))
    big = np.ones((3, 5), np.uint64)
    with pytest.raises(tp.TpcfError):   # a region count above its total
        tp.jackknife(z, big, z, t, z, t, 10, n, 10, n)


# --- 3-D distances: thresholds S_k and the FP32 band ---------------------------

@pytest.mark.parametrize("edges", [
    synthcat.log_edges(0.5, 150.0, 40),
    np.array([0.0, 1e-9, 0.3, 1.0, 2.0, 7.5, 1e6, 3e40, 1e120]),
])
def test_3d_thresholds_bracket_sqrt(edges):
    S, _, _ = tp.compile_edges_3d(edges, rmax=1000.0)
    for k, e in enumerate(edges):
        if e == 0.0:
            assert S[k] == -np.inf
            continue
        assert math.sqrt(S[k]) >= e
        assert math.sqrt(_next(S[k], -1)) < e
        for s in range(1, 40):
            assert math.sqrt(_next(S[k], s)) >= e
            lo = _next(S[k], -s)
            if lo >= 0.0:
                assert math.sqrt(lo) < e
    assert np.all(np.diff(S[np.isfinite(S)]) > 0)


def test_3d_edges_validation():
    for bad in ([1.0, 1.0, 2.0], [2.0, 1.0], [-1.0, 1.0], [1.0, np.inf], [1.0, 2e150], [1.0]):
        with pytest.raises(tp.TpcfError):
            tp.compile_edges_3d(bad, rmax=1.0)
    with pytest.raises(tp.TpcfError):
        tp.compile_edges_3d([1.0, 2.0], rmax=-1.0)


def _pairs_at_distance(g, r, rmax):
    """Pairs (a, b) with |a - b| = r (to FP64 rounding), a random direction,
    and both points within the ball of radius rmax."""
    n = r.size
    u = g.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    base = g.uniform(-1.0, 1.0, size=(n, 3)) * (0.3 * rmax)
    return base, base + r[:, None] * u


@pytest.mark.parametrize("rmax", [1.0, 1000.0, 3.0e5])
def test_3d_fp32_band_adversary(rmax):
    """Pairs at r = e_k (1 +- 10^-s), s = 2..9, for every edge: each FP32
    decision the band calls certain agrees with the oracle's distance rule,
    and the band is no wider than its error analysis allows."""
    g = np.random.default_rng(11)
    edges = synthcat.log_edges(1e-3 * rmax, 0.3 * rmax, 24)
    S, qlo, qhi = tp.compile_edges_3d(edges, rmax=rmax)
    rs, rel, edge_of = [], [], []
    for k, e in enumerate(edges):
        for s in range(2, 10):
            for sign in (-1.0, 1.0):
                rs.append(np.full(50, e * (1.0 + sign * 10.0 ** -s)))
                rel.append(np.full(50, 10.0 ** -s))
                edge_of.append(np.full(50, k))
    r = np.concatenate(rs)
    rel = np.concatenate(rel)
    edge_of = np.concatenate(edge_of)
    a, b = _pairs_at_distance(g, r, rmax)
    assert np.all(np.linalg.norm(a, axis=1) <= rmax) and np.all(np.linalg.norm(b, axis=1) <= rmax)
    q = _q32(a, b)
    dist = oracle.pair_distances(a.T, b.T)
    d = a - b
    r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    in_band = np.zeros(r.size, bool)
    for k in range(edges.size):
        past = dist >= edges[k]
        assert np.array_equal(past, r2 >= S[k]), k
        above = q >= qhi[k]
        below = q < qlo[k]
        assert np.all(past[above]), k
        assert not np.any(past[below]), k
        in_band |= ~above & ~below & (edge_of == k)
    # half-width in r: a = 2^-23 rmax from the FP32 copies plus ~3 ulp of q
    half = 2.0 ** -23 * rmax / edges[edge_of] + 4e-7
    assert not np.any(in_band & (rel > 3.0 * half))
    assert np.all(in_band[rel < 0.1 * half])


@pytest.mark.parametrize("precision", [tp.FP32_CHORD, tp.FP64])
def test_edge_at_zero_never_flags(precision):
    """An edge at 0 degrees (D_0 = +inf, E_0 = -inf) is passed by every pair,
    so no cell may leave it undecided (0x8000 | 0) and every cell's slot is
    at least 1; the bottom cell, open towards -inf, included."""
    for edges in (np.array([0.0, 1.0, 120.0]), np.linspace(0.0, 180.0, 31)):
        _, _, _, cells, _ = tp.compile_cells(edges, precision)
        cells = cells.astype(np.int64)
        assert not np.any(cells == 0x8000)
        certain = cells < 0x8000
        assert np.all(cells[certain] >= 1)
        assert np.all((cells[~certain] & 0x7FFF) >= 1) or np.all(cells[~certain] == 0xFFFF)
