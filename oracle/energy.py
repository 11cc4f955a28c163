"""Coulomb and binding energies (test infrastructure only).

Eq. total_energy: the total electrostatic energy of a species is its
solvation energy (Eq. solv) plus the Coulomb energy of its point charges.
Eq. bind_energy: the binding energy of a complex is its total energy minus
those of the receptor and the ligand, with rigid geometries.

Reading (the paper does not write the Coulomb term out): the potential in
region r is the Coulomb potential of the charges of r in a uniform medium of
permittivity eps_r plus the reaction potential (the identity behind the rows
of the system); so the Coulomb energy is
    E_C = k_e * sum_r sum_{i<j in r} q_i q_j / (eps_r |x_i - x_j|),
and charges of different regions interact only through the reaction
potential.
"""

from __future__ import annotations

import numpy as np

from .bem import KE, Oracle


def coulomb_energy(problem):
    """E_C in kJ/mol (pairs within each region, that region's eps)."""
    total = 0.0
    for r, (x, q) in problem.charges.items():
        x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
        q = np.asarray(q, dtype=np.float64)
        eps = problem.regions[r].eps
        for i in range(len(q)):
            d = np.linalg.norm(x[i + 1:] - x[i], axis=1)
            total += KE * q[i] * float(np.sum(q[i + 1:] / d)) / eps
    return total


def total_energy(problem, tol=1e-10):
    """Eq. total_energy: solvation (dense oracle solve) + Coulomb."""
    solv = Oracle(problem).solve(tol=tol).energy
    coul = coulomb_energy(problem)
    return solv + coul, solv, coul


def binding_energy(complex_, receptor, ligand, tol=1e-10):
    """Eq. bind_energy; returns (ddG, {species: (total, solvation, coulomb)})."""
    parts = {k: total_energy(p, tol) for k, p in
             (("complex", complex_), ("receptor", receptor), ("ligand", ligand))}
    ddg = parts["complex"][0] - parts["receptor"][0] - parts["ligand"][0]
    return ddg, parts
