"""Panel geometry for flat triangular boundary elements (oracle).

Follows the discretisation of sec. 2.2 (single-surface problems, Eq.
nBEM_disc): flat triangles carrying a constant potential and normal
derivative, collocated at the panel centre.  The normal of a panel whose
vertices are counter-clockwise seen from the outer region points into that
region.  L = sqrt(2 A) is the characteristic panel length used by the
near-singular threshold (sec. 3, lysozyme parameter table).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .quadrature import triangle_rule


@dataclass
class Panels:
    v0: np.ndarray
    v1: np.ndarray
    v2: np.ndarray
    centre: np.ndarray  # collocation points (n, 3)
    normal: np.ndarray  # unit normals (n, 3)
    area: np.ndarray  # (n,)
    length: np.ndarray  # L = sqrt(2 A)

    @property
    def n(self):
        return len(self.area)


def panels(verts, tris) -> Panels:
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris)
    v0, v1, v2 = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    c = np.cross(v1 - v0, v2 - v0)
    cn = np.linalg.norm(c, axis=1)
    area = 0.5 * cn
    normal = c / cn[:, None]
    centre = (v0 + v1 + v2) / 3.0
    return Panels(v0, v1, v2, centre, normal, area, np.sqrt(2.0 * area))


def gauss_points(p: Panels, k: int):
    """Quadrature points y (n, K, 3) and physical weights W = w * A (n, K)."""
    bary, w = triangle_rule(k)
    y = (bary[None, :, 0, None] * p.v0[:, None, :]
         + bary[None, :, 1, None] * p.v1[:, None, :]
         + bary[None, :, 2, None] * p.v2[:, None, :])
    centroid = np.all(np.abs(bary - 1.0 / 3.0) < 1e-15, axis=1)
    # the centroid point is formed exactly like the collocation point
    y[:, centroid, :] = p.centre[:, None, :]
    W = w[None, :] * p.area[:, None]
    return y, W
