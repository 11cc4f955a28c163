"""Workload recipes: surfaces, dielectric regions and charges.

A problem is a set of regions (permittivity eps, inverse Debye length kappa;
kappa = 0 means the Laplace equation holds there), closed surfaces that each
separate an inner region from an outer region, and point charges that live in
one region.  These recipes only assemble arrays; see ``meshes`` and
``charges`` for the generators.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .charges import ball_charges, star_interior_charges
from .meshes import StarShape, geodesic_sphere, radial_offset, star_surface


@dataclass
class Region:
    eps: float
    kappa: float
    name: str = ""


@dataclass
class Surface:
    verts: np.ndarray  # (n_v, 3) float64, angstrom
    tris: np.ndarray  # (n_p, 3) int32, counter-clockwise seen from ``outer``
    inner: int
    outer: int
    name: str = ""

    @property
    def n_panels(self):
        return int(len(self.tris))


@dataclass
class Problem:
    regions: list
    surfaces: list
    charges: dict = field(default_factory=dict)  # region id -> (xyz, q)
    name: str = ""

    @property
    def n_panels(self):
        return sum(s.n_panels for s in self.surfaces)

    @property
    def n_charges(self):
        return sum(len(q) for _, q in self.charges.values())

    def all_charges(self):
        """Charges in region order: (xyz, q, region id per charge)."""
        xs, qs, rs = [], [], []
        for r in sorted(self.charges):
            x, q = self.charges[r]
            xs.append(np.asarray(x, dtype=np.float64).reshape(-1, 3))
            qs.append(np.asarray(q, dtype=np.float64).reshape(-1))
            rs.append(np.full(len(q), r, dtype=np.int32))
        if not xs:
            return np.zeros((0, 3)), np.zeros(0), np.zeros(0, dtype=np.int32)
        return np.vstack(xs), np.concatenate(qs), np.concatenate(rs)


def born_sphere(nu=16, base="oct", radius=4.0, eps_in=4.0, eps_out=80.0,
                kappa=0.0, charges=None):
    """Dielectric sphere; by default one +1 e charge at its centre."""
    v, f = geodesic_sphere(base, nu, radius)
    if charges is None:
        charges = (np.zeros((1, 3)), np.ones(1))
    return Problem(
        regions=[Region(eps_in, 0.0, "molecule"), Region(eps_out, kappa, "solvent")],
        surfaces=[Surface(v, f, 0, 1, "sphere")],
        charges={0: charges},
        name=f"born-{base}{nu}",
    )


def config1_kirkwood_sphere(nu=16, base="oct", seed=1):
    """Sphere a = 4 A, +1 e at the centre plus 8 charges q ~ U(-1, 1) in r <= 3.

    eps 4 / 80, kappa = 0.125 / A.  oct nu = 16 gives 2,048 panels.
    """
    x, q = ball_charges(8, 3.0, seed, center_charge=1.0)
    p = born_sphere(nu, base, 4.0, 4.0, 80.0, 0.125, (x, q))
    p.name = f"kirkwood-sphere-{base}{nu}"
    return p


def config2_star(nu=45, seed=2, n_charges=2000, r0=20.0):
    """Star-shaped protein-like surface, ico nu = 45 (40,500 panels).

    r(u) = 20 A * (1 + sum_{l<=8} a_lm Y_lm(u)), a_lm ~ N(0, (0.04/l)^2);
    2,000 charges uniform in |x| < r(u) - 2 A with q ~ N(0, 0.3^2);
    eps 4 / 80, kappa = 0.125 / A.
    """
    shape = StarShape(r0, seed)
    v, f = star_surface(shape, nu, "ico")
    x, q = star_interior_charges(shape, n_charges, seed, clearance=2.0)
    return Problem(
        regions=[Region(4.0, 0.0, "protein"), Region(80.0, 0.125, "solvent")],
        surfaces=[Surface(v, f, 0, 1, "SES")],
        charges={0: (x, q)},
        name=f"star-ico{nu}",
    )


def config3_multisurface(nu=64, cav_nu=16, seed=3, n_charges=4000, r0=20.0,
                         shape_seed=2, stern=2.0, eps_out=80.0, kappa=0.125):
    """Protein + Stern layer + two solvent-filled cavities.

    Protein: the star surface of ``shape_seed`` at ico ``nu`` (81,920 panels
    at nu = 64).  Stern: the same connectivity moved radially out by 2 A.
    Cavities: spheres of radius 3 A at (+-7, 0, 0), oct ``cav_nu``.  Charges:
    ``n_charges`` in the protein region, >= 2 A from every surface,
    q ~ N(0, 0.3^2).  Regions: protein eps 4; Stern, solvent and cavities
    eps_out; kappa = 0 except in the solvent.
    """
    shape = StarShape(r0, shape_seed)
    vp, fp = star_surface(shape, nu, "ico")
    vs = radial_offset(vp, stern)
    cav = [((-7.0, 0.0, 0.0), 3.0), ((7.0, 0.0, 0.0), 3.0)]
    regions = [
        Region(4.0, 0.0, "protein"),
        Region(eps_out, 0.0, "stern"),
        Region(eps_out, kappa, "solvent"),
        Region(eps_out, 0.0, "cavity1"),
        Region(eps_out, 0.0, "cavity2"),
    ]
    surfaces = [Surface(vp, fp, 0, 1, "SES"), Surface(vs, fp.copy(), 1, 2, "stern")]
    for i, (c, rad) in enumerate(cav):
        vc, fc = geodesic_sphere("oct", cav_nu, rad, c)
        surfaces.append(Surface(vc, fc, 3 + i, 0, f"cavity{i + 1}"))
    x, q = star_interior_charges(shape, n_charges, seed, clearance=2.0, exclude=cav)
    return Problem(regions, surfaces, {0: (x, q)}, name=f"multisurface-ico{nu}")


def config5_small(seed=3, n_charges=4000):
    """Reduced three-region system: protein and Stern at ico nu = 16 (5,120
    panels each), cavities at oct nu = 8 (512 each): 22,528 unknowns."""
    p = config3_multisurface(nu=16, cav_nu=8, seed=seed, n_charges=n_charges)
    p.name = "multisurface-ico16"
    return p


def config4_batch(n_mol=64, seed0=4000, nu_cap=None):
    """Uneven batch of star-shaped molecules.

    Molecule i uses seed 4000 + i: radius R ~ U(8, 30) A; panels
    20 nu^2 ~ 1,280 * 32^((R - 8)/22) (1,280 .. 40,960); charges
    round(50 * 40^((R - 8)/22)) (50 .. 2,000); otherwise as the star workload.
    """
    out = []
    for i in range(n_mol):
        seed = seed0 + i
        rng = np.random.default_rng(seed)
        R = rng.uniform(8.0, 30.0)
        t = (R - 8.0) / 22.0
        target = 1280.0 * 32.0 ** t
        nu = max(8, int(round(math.sqrt(target / 20.0))))
        if nu_cap is not None:
            nu = min(nu, nu_cap)
        nq = int(round(50.0 * 40.0 ** t))
        shape = StarShape(R, seed)
        v, f = star_surface(shape, nu, "ico")
        clear = min(2.0, 0.25 * R)
        x, q = star_interior_charges(shape, nq, seed, clearance=clear)
        out.append(Problem(
            regions=[Region(4.0, 0.0, "protein"), Region(80.0, 0.125, "solvent")],
            surfaces=[Surface(v, f, 0, 1, "SES")],
            charges={0: (x, q)},
            name=f"batch-{i}",
        ))
    return out


def concentric_spheres(radii, eps, kappa, charges, charge_region, nu=16, base="oct"):
    """Nested spheres about the origin for layered closed-form checks.

    ``radii`` ascending (m spheres), ``eps``/``kappa`` per region from the
    innermost (index 0) to the outermost (index m).  Sphere i separates
    region i (inside) from region i + 1 (outside).  All charges sit in
    ``charge_region``.
    """
    regions = [Region(e, k, f"layer{i}") for i, (e, k) in enumerate(zip(eps, kappa))]
    surfaces = []
    for i, a in enumerate(radii):
        v, f = geodesic_sphere(base, nu, a)
        surfaces.append(Surface(v, f, i, i + 1, f"sphere{i}"))
    return Problem(regions, surfaces, {charge_region: charges}, name="concentric")


def _translated(v, offset):
    return np.asarray(v, dtype=np.float64) + np.asarray(offset, dtype=np.float64)[None, :]


def _pair(rec, lig, name):
    """Complex of two single-surface molecules sharing the outer region.

    ``rec`` and ``lig`` are one-surface problems (region 0 inside, region 1
    outside, charges in region 0) with the same solvent.  The complex has
    regions [receptor interior, ligand interior, solvent].
    """
    sa, sb = rec.surfaces[0], lig.surfaces[0]
    ra, rb, rs = rec.regions[0], lig.regions[0], rec.regions[1]
    cplx = Problem(
        regions=[Region(ra.eps, ra.kappa, "receptor"), Region(rb.eps, rb.kappa, "ligand"),
                 Region(rs.eps, rs.kappa, "solvent")],
        surfaces=[Surface(sa.verts, sa.tris, 0, 2, "receptor"),
                  Surface(sb.verts, sb.tris, 1, 2, "ligand")],
        charges={0: rec.charges[0], 1: lig.charges[0]},
        name=name,
    )
    return cplx, rec, lig


def born_pair(distance, radius=2.0, q=(1.0, -1.0), nu=8, base="oct", eps_in=4.0,
              eps_out=80.0, kappa=0.0):
    """Two Born ions (spheres of ``radius`` with a central charge each) whose
    centres are ``distance`` apart along x: (complex, receptor, ligand)."""
    rec = born_sphere(nu, base, radius, eps_in, eps_out, kappa,
                      (np.zeros((1, 3)), np.array([q[0]], dtype=np.float64)))
    v, f = geodesic_sphere(base, nu, radius, center=(distance, 0.0, 0.0))
    lig = Problem(
        regions=[Region(eps_in, 0.0, "molecule"), Region(eps_out, kappa, "solvent")],
        surfaces=[Surface(v, f, 0, 1, "sphere")],
        charges={0: (np.array([[distance, 0.0, 0.0]]), np.array([q[1]], dtype=np.float64))},
        name="born-ligand",
    )
    return _pair(rec, lig, f"born-pair-{distance:g}")


def star_pair(gap=4.0, r_rec=14.0, r_lig=9.0, nu_rec=24, nu_lig=16, n_rec=600, n_lig=200,
              seed=6, kappa=0.125):
    """Receptor and ligand star-shaped molecules (seeded as the star
    workload) placed along x with at least ``gap`` angstrom between their
    surfaces: (complex, receptor, ligand)."""
    out = []
    for r0, nu, nq, s in ((r_rec, nu_rec, n_rec, seed), (r_lig, nu_lig, n_lig, seed + 1)):
        shape = StarShape(r0, s)
        v, f = star_surface(shape, nu, "ico")
        x, q = star_interior_charges(shape, nq, s, clearance=2.0)
        out.append((v, f, x, q))
    ra = float(np.max(np.linalg.norm(out[0][0], axis=1)))
    rb = float(np.max(np.linalg.norm(out[1][0], axis=1)))
    off = np.array([ra + rb + gap, 0.0, 0.0])
    probs = []
    for k, (v, f, x, q) in enumerate(out):
        shift = off if k == 1 else np.zeros(3)
        probs.append(Problem(
            regions=[Region(4.0, 0.0, "protein"), Region(80.0, kappa, "solvent")],
            surfaces=[Surface(_translated(v, shift), f, 0, 1, "SES")],
            charges={0: (_translated(x, shift), q)},
            name=("receptor", "ligand")[k],
        ))
    return _pair(probs[0], probs[1], "star-pair")


def ion_cavity_protein(nu=16, cav_nu=8, seed=7, n_charges=400, r0=20.0, shape_seed=2,
                       stern=2.0, eps_out=80.0, kappa=0.125, ion_radius=3.0, cav_stern=1.5):
    """Protein with a Stern layer, one solvent-filled cavity and one cavity
    large enough to hold ions, with its own interior Stern layer.

    Protein and Stern: as the multi-surface workload (star of ``shape_seed``
    at ico ``nu``, Stern moved out by 2 A).  Solvent cavity: radius 3 A at
    (-7, 0, 0).  Ion cavity at (7, 0, 0): an outer sphere of radius
    ion_radius + cav_stern bounds its Stern shell (solvent eps, no ions),
    an inner sphere of radius ion_radius bounds the ionic interior (solvent
    eps and kappa).  Charges in the protein region, >= 2 A from every
    surface.
    """
    shape = StarShape(r0, shape_seed)
    vp, fp = star_surface(shape, nu, "ico")
    vs = radial_offset(vp, stern)
    regions = [
        Region(4.0, 0.0, "protein"),
        Region(eps_out, 0.0, "stern"),
        Region(eps_out, kappa, "solvent"),
        Region(eps_out, 0.0, "cavity"),
        Region(eps_out, 0.0, "cavity_stern"),
        Region(eps_out, kappa, "cavity_ions"),
    ]
    c_sol, c_ion = (-7.0, 0.0, 0.0), (7.0, 0.0, 0.0)
    surfaces = [Surface(vp, fp, 0, 1, "SES"), Surface(vs, fp.copy(), 1, 2, "stern")]
    v, f = geodesic_sphere("oct", cav_nu, 3.0, c_sol)
    surfaces.append(Surface(v, f, 3, 0, "cavity"))
    v, f = geodesic_sphere("oct", cav_nu, ion_radius + cav_stern, c_ion)
    surfaces.append(Surface(v, f, 4, 0, "cavity_stern"))
    v, f = geodesic_sphere("oct", cav_nu, ion_radius, c_ion)
    surfaces.append(Surface(v, f, 5, 4, "cavity_ions"))
    excl = [(c_sol, 3.0), (c_ion, ion_radius + cav_stern)]
    x, q = star_interior_charges(shape, n_charges, seed, clearance=2.0, exclude=excl)
    return Problem(regions, surfaces, {0: (x, q)}, name=f"ion-cavity-ico{nu}")
