"""Closed triangulated surfaces used as stand-ins for molecular surfaces.

Triangles are returned counter-clockwise when seen from outside, i.e. the
right-hand normal points away from the enclosed region.  Vertex arrays are
float64 (n_v, 3) in angstrom, triangle arrays int32 (n_p, 3).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.special import sph_harm_y


def icosahedron():
    """Unit icosahedron: 12 vertices, 20 outward-oriented faces."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array(
        [
            [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
            [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
            [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
        ],
        dtype=np.float64,
    )
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array(
        [
            [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
            [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
            [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
            [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
        ],
        dtype=np.int32,
    )
    return _orient_outward(v, f)


def octahedron():
    """Unit octahedron: 6 vertices, 8 outward-oriented faces."""
    v = np.array(
        [[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
        dtype=np.float64,
    )
    f = np.array(
        [
            [0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4],
            [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5],
        ],
        dtype=np.int32,
    )
    return _orient_outward(v, f)


def _orient_outward(v, f):
    """Flip any face whose right-hand normal points toward the origin."""
    f = f.copy()
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    nrm = np.cross(b - a, c - a)
    inward = np.einsum("ij,ij->i", nrm, a + b + c) < 0
    f[inward] = f[inward][:, [0, 2, 1]]
    return v, f


def geodesic_sphere(base: str, nu: int, radius: float = 1.0, center=(0.0, 0.0, 0.0)):
    """Class-I geodesic sphere of frequency ``nu``.

    Every base face is cut into nu*nu triangles on a barycentric lattice and
    the lattice points are pushed out to the sphere.  The icosahedron gives
    20*nu^2 faces and 10*nu^2+2 vertices; the octahedron 8*nu^2 and 4*nu^2+2.
    Lattice points on shared edges are identified through a canonical key, so
    the mesh is closed and every vertex is stored once.
    """
    if base == "ico":
        bv, bf = icosahedron()
    elif base == "oct":
        bv, bf = octahedron()
    else:
        raise ValueError(f"unknown base solid {base!r}")
    if nu < 1:
        raise ValueError("nu must be >= 1")
    index = {}
    coords = []

    def vid(face, i, j, k):
        # canonical key: base-vertex ids with their integer lattice weights
        parts = sorted((int(face[m]), w) for m, w in enumerate((i, j, k)) if w > 0)
        key = tuple(parts)
        got = index.get(key)
        if got is None:
            p = np.zeros(3)
            for gid, w in parts:
                p = p + w * bv[gid]
            p = p / nu
            got = len(coords)
            index[key] = got
            coords.append(p)
        return got

    tris = []
    for face in bf:
        ids = {}
        for i in range(nu + 1):
            for j in range(nu + 1 - i):
                k = nu - i - j
                ids[(i, j)] = vid(face, i, j, k)
        # lattice point (i, j) sits at (i*A + j*B + k*C)/nu
        for i in range(nu):
            for j in range(nu - i):
                a = ids[(i, j)]
                b = ids[(i + 1, j)]
                c = ids[(i, j + 1)]
                tris.append((a, b, c))
                if i + j < nu - 1:
                    d = ids[(i + 1, j + 1)]
                    tris.append((b, d, c))
    v = np.array(coords, dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array(tris, dtype=np.int32)
    v, f = _orient_outward(v, f)
    v = v * float(radius) + np.asarray(center, dtype=np.float64)
    return v, f


def _real_sph_harm(l, m, polar, azim):
    """Orthonormal real spherical harmonic Y_lm."""
    if m == 0:
        return sph_harm_y(l, 0, polar, azim).real
    y = sph_harm_y(l, abs(m), polar, azim)
    s = math.sqrt(2.0) * (-1.0) ** m
    return s * (y.real if m > 0 else y.imag)


@dataclass
class StarShape:
    """Star-shaped radius function r(u) = R0 * (1 + sum a_lm Y_lm(u)).

    Coefficients a_lm ~ N(0, (std0/l)^2) for 1 <= l <= lmax, drawn from
    ``numpy.random.default_rng(seed)`` in (l, m = -l..l) order.
    """

    r0: float
    seed: int
    lmax: int = 8
    std0: float = 0.04

    def __post_init__(self):
        rng = np.random.default_rng(self.seed)
        self.coef = []
        for l in range(1, self.lmax + 1):
            for m in range(-l, l + 1):
                self.coef.append((l, m, rng.normal(0.0, self.std0 / l)))

    def radius(self, dirs):
        """r along unit directions ``dirs`` (n, 3)."""
        dirs = np.asarray(dirs, dtype=np.float64)
        polar = np.arccos(np.clip(dirs[:, 2], -1.0, 1.0))
        azim = np.arctan2(dirs[:, 1], dirs[:, 0])
        s = np.zeros(len(dirs))
        for l, m, a in self.coef:
            s += a * _real_sph_harm(l, m, polar, azim)
        return self.r0 * (1.0 + s)


def star_surface(shape: StarShape, nu: int, base: str = "ico", offset: float = 0.0):
    """Geodesic sphere whose vertices are moved radially to r(u) + offset."""
    v, f = geodesic_sphere(base, nu, 1.0)
    r = shape.radius(v) + offset
    return v * r[:, None], f


def radial_offset(verts, delta):
    """Move every vertex radially outward by ``delta`` (same connectivity)."""
    verts = np.asarray(verts, dtype=np.float64)
    r = np.linalg.norm(verts, axis=1, keepdims=True)
    return verts * ((r + delta) / r)
