"""Seeded synthetic inputs: triangulated surfaces and point charges.

This package holds input data only (vertex and triangle arrays, charge
positions and values).  It computes nothing of the boundary-element method:
no panel geometry, quadrature, Green's function or energy.  Both the CPU
oracle and the GPU path read their inputs from here, so that each side is fed
bit-identical arrays while sharing no arithmetic.
"""

from .meshes import (
    icosahedron,
    octahedron,
    geodesic_sphere,
    star_surface,
    radial_offset,
    StarShape,
)
from .charges import ball_charges, star_interior_charges
from .configs import (
    Surface,
    Region,
    Problem,
    born_sphere,
    config1_kirkwood_sphere,
    config2_star,
    config3_multisurface,
    config4_batch,
    config5_small,
    concentric_spheres,
    born_pair,
    star_pair,
    ion_cavity_protein,
)

__all__ = [
    "icosahedron",
    "octahedron",
    "geodesic_sphere",
    "star_surface",
    "radial_offset",
    "StarShape",
    "ball_charges",
    "star_interior_charges",
    "Surface",
    "Region",
    "Problem",
    "born_sphere",
    "config1_kirkwood_sphere",
    "config2_star",
    "config3_multisurface",
    "config4_batch",
    "config5_small",
    "concentric_spheres",
    "born_pair",
    "star_pair",
    "ion_cavity_protein",
]
