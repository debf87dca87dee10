"""Probe pairs that tell the counting rule's FP64 operation order apart from
fused or reordered evaluations (test helper, no GPU).

The counting rule takes the angle of a pair as the arc-cosine of the dot
product of the two unit vectors (paper, Section 3, first bullet).  The reading
fixed for it is the dot product d = (x_i x_j + y_i y_j) + z_i z_j with every
product and every sum rounded to FP64, left to right, and no fused
multiply-add (the paper's CPU, Table 1, has no FMA unit).  In 3-D the squared
distance is (dx^2 + dy^2) + dz^2 of the rounded coordinate differences, in the
same order.

The helpers evaluate the rule and the alternatives a compiler or a different
code could produce (an FMA for one or both sums, other summation orders, a
correctly rounded dot) in exact rational arithmetic, rounding to the nearest
double after each operation.  The expected values therefore do not depend on
how this interpreter or any library evaluates floating point, and no value
comes from the code under test.

``sky_probes`` and ``box_probes`` search seeded random pairs for ones where
some alternative gives a different angle (distance) than the rule, and place
bin edges right at those angles, so that the rule and every alternative that
differs put the pair in different bins.
"""

from __future__ import annotations

import math
from fractions import Fraction as F

import numpy as np

DEG = math.pi / 180.0   # the rule's degree factor (FP64 pi over 180)


def rnd(q: F) -> float:
    """Nearest double to an exact rational (ties to even): CPython's integer
    true division, which Fraction.__float__ uses, is correctly rounded."""
    return float(q)


def dot_orders(a, b) -> dict:
    """FP64 dot product of a and b under the rule and under alternatives,
    each operation rounded once (an FMA rounds its product and sum once)."""
    ex = [F(float(a[c])) * F(float(b[c])) for c in range(3)]   # exact products
    p = [rnd(e) for e in ex]                                     # rounded products
    px, py, pz = (F(v) for v in p)
    fx, fy, fz = ex
    return {
        "rule": rnd(F(rnd(px + py)) + pz),
        "fma_xy_then_add_z": rnd(F(rnd(fy + px)) + pz),
        "fma_yx_then_add_z": rnd(F(rnd(fx + py)) + pz),
        "add_xy_then_fma_z": rnd(fz + F(rnd(px + py))),
        "fma_chain_x_y_z": rnd(fz + F(rnd(fy + px))),
        "fma_chain_y_x_z": rnd(fz + F(rnd(fx + py))),
        "x_plus_yz": rnd(px + F(rnd(py + pz))),
        "xz_plus_y": rnd(F(rnd(px + pz)) + py),
        "correctly_rounded": rnd(fx + fy + fz),
    }


def d2_orders(a, b) -> dict:
    """FP64 squared distance of points a and b under the rule
    ((dx^2 + dy^2) + dz^2 of the rounded differences) and alternatives."""
    d = [rnd(F(float(a[c])) - F(float(b[c]))) for c in range(3)]
    ex = [F(v) * F(v) for v in d]
    sx, sy, sz = (F(rnd(e)) for e in ex)
    fx, fy, fz = ex
    return {
        "rule": rnd(F(rnd(sx + sy)) + sz),
        "fma_xy_then_add_z": rnd(F(rnd(fy + sx)) + sz),
        "fma_yx_then_add_z": rnd(F(rnd(fx + sy)) + sz),
        "add_xy_then_fma_z": rnd(fz + F(rnd(sx + sy))),
        "fma_chain_x_y_z": rnd(fz + F(rnd(fy + sx))),
        "fma_chain_y_x_z": rnd(fz + F(rnd(fx + sy))),
        "x_plus_yz": rnd(sx + F(rnd(sy + sz))),
        "xz_plus_y": rnd(F(rnd(sx + sz)) + sy),
        "correctly_rounded": rnd(fx + fy + fz),
    }


def angle_of(d: float) -> float:
    """The rule's angle of a dot product: acos of the clamped value."""
    return math.acos(min(max(d, -1.0), 1.0))


def _deg_for(lo: float, hi: float) -> float | None:
    """An edge in degrees whose radian value fl(deg * DEG) lies in (lo, hi],
    preferring hi itself; None if no such double is near hi / DEG."""
    best = None
    for direction in (-math.inf, math.inf):
        t = hi / DEG
        for _ in range(128):
            r = t * DEG
            if lo < r <= hi:
                if r == hi:
                    return t
                if best is None:
                    best = t
            t = math.nextafter(t, direction)
    return best


def _edges_around(rule: float, others, to_unit) -> list:
    """Edges (in the caller's unit) that separate `rule` from every value in
    `others`: one at the rule's own value (a tie goes up, so values below
    fall under it) and one just above it at the smallest larger value."""
    out = []
    below = [v for v in others if v < rule]
    above = [v for v in others if v > rule]
    if below:
        e = to_unit(max(below), rule)
        if e is not None:
            out.append(e)
    if above:
        e = to_unit(rule, min(above))
        if e is not None:
            out.append(e)
    return out


def _unit(g, n):
    v = g.normal(size=n)
    return v / np.linalg.norm(v)


def sky_probes(seed: int = 1204, n: int = 40, max_tries: int = 20000):
    """n pairs of FP64 unit vectors (all components of magnitude >= 0.05) at
    separations log-uniform in [1e-5, 0.3] rad, each kept only if some
    alternative order gives it a different angle than the rule, and edges in
    degrees (strictly increasing) placed at the rule's and the alternatives'
    angles.  Returns (a [n, 3], b [n, 3], edges_deg)."""
    g = np.random.default_rng(seed)
    A, B, edges = [], [], []
    tries = 0
    while len(A) < n and tries < max_tries:
        tries += 1
        a = _unit(g, 3)
        if np.min(np.abs(a)) < 0.05:
            continue
        th = math.exp(g.uniform(math.log(1e-5), math.log(0.3)))
        u = _unit(g, 3)
        u = u - np.dot(u, a) * a
        u /= np.linalg.norm(u)
        b = math.cos(th) * a + math.sin(th) * u
        b /= np.linalg.norm(b)
        if np.min(np.abs(b)) < 0.05:
            continue
        orders = dot_orders(a, b)
        t_rule = angle_of(orders["rule"])
        others = sorted({angle_of(v) for k, v in orders.items() if k != "rule"} - {t_rule})
        if not others:
            continue
        e = _edges_around(t_rule, others, _deg_for)
        if not e:
            continue
        A.append(a)
        B.append(b)
        edges += e
    edges = sorted(set(edges))
    return np.array(A), np.array(B), np.array(edges, dtype=np.float64)


def box_probes(seed: int = 1205, n: int = 40, side: float = 1000.0, max_tries: int = 20000):
    """n pairs of 3-D points in [-side, side]^3 at distances log-uniform in
    [1e-2, 100], kept only if some alternative order gives a different
    distance (sqrt of the squared distance) than the rule, and edges placed at
    those distances.  Returns (a [n, 3], b [n, 3], edges)."""
    g = np.random.default_rng(seed)
    A, B, edges = [], [], []
    tries = 0

    def exact(lo, hi):
        return hi

    while len(A) < n and tries < max_tries:
        tries += 1
        a = g.uniform(-side, side, size=3)
        r = math.exp(g.uniform(math.log(1e-2), math.log(100.0)))
        b = a + r * _unit(g, 3)
        orders = d2_orders(a, b)
        r_rule = math.sqrt(orders["rule"])
        others = sorted({math.sqrt(v) for k, v in orders.items() if k != "rule"} - {r_rule})
        if not others:
            continue
        A.append(a)
        B.append(b)
        edges += _edges_around(r_rule, others, exact)
    edges = sorted(set(edges))
    return np.array(A), np.array(B), np.array(edges, dtype=np.float64)


def slot(value: float, edges_unit) -> int:
    """Number of edges at or below value (ties go up)."""
    return int(np.searchsorted(np.asarray(edges_unit), value, side="right"))


def expected_sky_hist(a_list, b_list, edges_deg, pairs, order="rule"):
    """Histogram (nbins+2 slots) of the listed index pairs (i into a_list, j
    into b_list) under the named order of the dot product."""
    er = [e * DEG for e in edges_deg]
    h = np.zeros(len(edges_deg) + 1, dtype=np.uint64)
    for i, j in pairs:
        h[slot(angle_of(dot_orders(a_list[i], b_list[j])[order]), er)] += 1
    return h


def expected_box_hist(a_list, b_list, edges, pairs, order="rule"):
    """Histogram of the listed index pairs under the named order of the
    squared distance (edges are distances)."""
    h = np.zeros(len(edges) + 1, dtype=np.uint64)
    for i, j in pairs:
        h[slot(math.sqrt(d2_orders(a_list[i], b_list[j])[order]), edges)] += 1
    return h
