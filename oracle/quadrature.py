"""Quadrature rules used by the oracle (test infrastructure only).

Triangle rules are the symmetric Gauss rules of Dunavant (1985), the family
the paper names when it speaks of K Gauss points per panel and K_fine points
in the near-singular region (sec. 3, parameter tables).  A rule is returned
as barycentric coordinates (K, 3) and weights (K,) that sum to one; the
physical weight of a point on a panel of area A is w * A.

The angular rule of the semi-analytic singular integral is Gauss-Legendre
(numpy's ``leggauss``), with N_k points per sub-triangle.
"""

from __future__ import annotations

import math

import numpy as np


def _orbit3(a, w):
    """(a, b, b) and its cyclic permutations, b = (1 - a)/2."""
    b = (1.0 - a) / 2.0
    return [(a, b, b), (b, a, b), (b, b, a)], [w, w, w]


def _orbit6(a, b, w):
    c = 1.0 - a - b
    pts = [(a, b, c), (a, c, b), (b, a, c), (b, c, a), (c, a, b), (c, b, a)]
    return pts, [w] * 6


def triangle_rule(k: int):
    """Symmetric K-point rule on a triangle (K in 1, 3, 4, 7, 19).

    Degrees of exactness: K=1 -> 1, K=3 -> 2, K=4 -> 3 (negative centroid
    weight), K=7 -> 5, K=19 -> 9.
    """
    pts, wts = [], []
    third = 1.0 / 3.0
    if k == 1:
        pts, wts = [(third, third, third)], [1.0]
    elif k == 3:
        pts, wts = _orbit3(2.0 / 3.0, 1.0 / 3.0)
    elif k == 4:
        p, w = _orbit3(0.6, 25.0 / 48.0)
        pts, wts = [(third, third, third)] + p, [-27.0 / 48.0] + w
    elif k == 7:
        s15 = math.sqrt(15.0)
        p1, w1 = _orbit3((9.0 - 2.0 * s15) / 21.0, (155.0 + s15) / 1200.0)
        p2, w2 = _orbit3((9.0 + 2.0 * s15) / 21.0, (155.0 - s15) / 1200.0)
        pts = [(third, third, third)] + p1 + p2
        wts = [0.225] + w1 + w2
    elif k == 19:
        groups = [
            _orbit3(0.020634961602525, 0.031334700227139),
            _orbit3(0.125820817014127, 0.077827541004774),
            _orbit3(0.623592928761935, 0.079647738927210),
            _orbit3(0.910540973211095, 0.025577675658698),
            _orbit6(0.036838412054736, 0.221962989160766, 0.043283539377289),
        ]
        pts, wts = [(third, third, third)], [0.097135796282799]
        for p, w in groups:
            pts += p
            wts += w
    else:
        raise ValueError(f"no {k}-point triangle rule")
    return np.array(pts, dtype=np.float64), np.array(wts, dtype=np.float64)


def rule_degree(k: int) -> int:
    return {1: 1, 3: 2, 4: 3, 7: 5, 19: 9}[k]


def gauss_legendre(n: int):
    """n-point Gauss-Legendre nodes and weights on [-1, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w
