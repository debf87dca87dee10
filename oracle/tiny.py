"""Pure-Python pair counting for small inputs -- TEST INFRASTRUCTURE ONLY.

A second, independent transcription of the counting definition (paper
Section 1 for DD/DR/RR, Section 3 for the dot product and arc-cosine), with
Python's ``math`` module for the trigonometry.  It is meant for a few hundred
to a couple of thousand points.
"""

from __future__ import annotations

import math


def unit_vector(ra_deg: float, dec_deg: float):
    a = ra_deg * (math.pi / 180.0)
    b = dec_deg * (math.pi / 180.0)
    return (math.cos(b) * math.cos(a), math.cos(b) * math.sin(a), math.sin(b))


def angle(p, q) -> float:
    d = (p[0] * q[0] + p[1] * q[1]) + p[2] * q[2]
    d = min(max(d, -1.0), 1.0)
    return math.acos(d)


def slot(theta: float, edges_rad) -> int:
    return sum(1 for e in edges_rad if e <= theta)


def count_pairs(points_a, edges_deg, points_b=None):
    """Histogram (list of nbins+2 ints) of pair angles.  With one list of unit
    vectors: unordered pairs i < j; with two: every (a, b) pair."""
    edges = [e * (math.pi / 180.0) for e in edges_deg]
    hist = [0] * (len(edges) + 1)
    if points_b is None:
        for i in range(len(points_a)):
            for j in range(i + 1, len(points_a)):
                hist[slot(angle(points_a[i], points_a[j]), edges)] += 1
    else:
        for p in points_a:
            for q in points_b:
                hist[slot(angle(p, q), edges)] += 1
    return hist
