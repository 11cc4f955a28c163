"""Binding energies and mesh-refinement estimates on top of libpbtc.

Eq. total_energy: the total electrostatic energy of a species is its
solvation energy (Eq. solv, from the GPU solve) plus the Coulomb energy of
its charges (pbtc_coulomb_energy: pairs within each region, that region's
permittivity).  Eq. bind_energy: the binding energy is the total energy of
the complex minus those of the receptor and the ligand, all with the same
rigid geometry.  Sec. 2.4: Richardson extrapolation (Eq. rich_extr) and the
observed order of convergence (Eq. observed_order) from three meshes refined
at a constant ratio of panel counts.  Every energy comes from the HIP
library; this module only combines the numbers.
"""

from __future__ import annotations

import math

from . import lib


def total_energy(problem, device="cuda:0", **params):
    """Solve one species; returns its total, solvation and Coulomb energies
    (kJ/mol) and the solver's counters.  ``problem``: a ``synth`` problem or
    a ``lib.Problem``."""
    if isinstance(problem, lib.Problem):
        plan = lib.Plan(problem, lib.default_params(**params), device)
    else:
        plan = lib.plan_for(problem, device, **params)
    res = plan.solve()
    coul, _ = plan.coulomb_energy()
    return {"total": res["energy_kJmol"] + coul, "solvation": res["energy_kJmol"],
            "coulomb": coul, "iterations": res["n_iter"], "rel_res": res["final_rel_res"]}


def binding_energy(complex_, receptor, ligand, device="cuda:0", **params):
    """Eq. bind_energy: returns (ddG in kJ/mol, per-species energies)."""
    parts = {name: total_energy(p, device, **params)
             for name, p in (("complex", complex_), ("receptor", receptor), ("ligand", ligand))}
    ddg = parts["complex"]["total"] - parts["receptor"]["total"] - parts["ligand"]["total"]
    return ddg, parts


def observed_order(f_fine, f_mid, f_coarse, ratio):
    """Eq. observed_order: p = log((f3 - f2) / (f2 - f1)) / log(r), f1 finest."""
    return math.log((f_coarse - f_mid) / (f_mid - f_fine)) / math.log(ratio)


def richardson(f_fine, f_mid, ratio, order):
    """Eq. rich_extr: f ~ f1 + (f1 - f2) / (r^p - 1)."""
    return f_fine + (f_fine - f_mid) / (ratio ** order - 1.0)


def refinement_study(problems, device="cuda:0", **params):
    """Solves a species on three meshes (coarse to fine, panel counts in a
    constant ratio) and returns the energies, the observed order and the
    Richardson-extrapolated energy."""
    if len(problems) != 3:
        raise ValueError("three meshes are needed")
    e = [total_energy(p, device, **params)["solvation"] for p in problems]
    n = [p.n_panels for p in problems]
    r = n[1] / n[0]
    if abs(n[2] / n[1] - r) > 1e-9 * r:
        raise ValueError("panel counts must grow by a constant ratio")
    p = observed_order(e[2], e[1], e[0], r)
    return {"energies": e, "panels": n, "ratio": r, "order": p,
            "extrapolated": richardson(e[2], e[1], r, p)}
