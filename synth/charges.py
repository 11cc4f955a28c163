"""Seeded point-charge sets (positions in angstrom, values in e)."""

from __future__ import annotations

import numpy as np


def _isotropic(rng, n):
    d = rng.normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def ball_charges(n, rmax, seed, center_charge=None, qlow=-1.0, qhigh=1.0):
    """``n`` charges uniform in the ball |x| <= rmax with q ~ U(qlow, qhigh).

    Radius r = rmax * u^(1/3), isotropic direction.  When ``center_charge`` is
    given, a charge of that value at the origin is prepended.
    """
    rng = np.random.default_rng(seed)
    u = rng.random(n)
    r = rmax * np.cbrt(u)
    x = _isotropic(rng, n) * r[:, None]
    q = rng.uniform(qlow, qhigh, size=n)
    if center_charge is not None:
        x = np.vstack([np.zeros((1, 3)), x])
        q = np.concatenate([[float(center_charge)], q])
    return x.astype(np.float64), q.astype(np.float64)


def star_interior_charges(shape, n, seed, clearance=2.0, qstd=0.3, exclude=()):
    """``n`` charges uniform inside a star-shaped surface, by rejection.

    A point x is kept when |x| < r(x/|x|) - clearance and it lies farther than
    radius + clearance from every excluded sphere (center, radius) in
    ``exclude``.  Values q ~ N(0, qstd^2).
    """
    rng = np.random.default_rng(seed)
    rbox = shape.r0 * 1.6
    out = []
    while len(out) < n:
        m = max(4 * (n - len(out)), 64)
        x = rng.uniform(-rbox, rbox, size=(m, 3))
        rr = np.linalg.norm(x, axis=1)
        ok = rr > 1e-9
        x, rr = x[ok], rr[ok]
        keep = rr < shape.radius(x / rr[:, None]) - clearance
        for c, rad in exclude:
            keep &= np.linalg.norm(x - np.asarray(c), axis=1) > rad + clearance
        out.extend(x[keep])
    x = np.array(out[:n], dtype=np.float64)
    q = rng.normal(0.0, qstd, size=n)
    return x, q
