"""GPU parity of the Coulomb energy, binding energies and the refinement
study (Eqs. total_energy, bind_energy, rich_extr, observed_order).

* pbtc_coulomb_energy against the oracle's pair sum (FP64 both sides, 1e-12),
  per independent system of a batch too.
* Binding energy of two Born ions (kappa = 0.125, d = 20 A): the GPU direct
  FP64 path against the oracle (1e-7 relative on each species' energy,
  1e-5 on the small difference) and against the screened closed form (3e-3).
* A star-shaped receptor / ligand pair with the FP32-refined treecode against
  the oracle: species energies to 1e-4, the difference to 2e-3 of the
  largest species energy.
* Born sphere at oct nu = 4, 8, 16: observed order near 1 (the paper reports
  1.013) and the extrapolated energy within 1e-3 of the closed form.
"""

import math

import numpy as np
import pytest

import synth
from oracle import KE
from oracle.energy import binding_energy as oracle_binding
from oracle.energy import coulomb_energy

pytestmark = pytest.mark.gpu


def test_coulomb_energy(gpu_lib):
    from paper_1309_4018_amd import lib

    for prob in (synth.config2_star(nu=10, n_charges=500),
                 synth.star_pair(nu_rec=8, nu_lig=6, n_rec=300, n_lig=100)[0]):
        pl = lib.plan_for(prob, op="direct", precision="fp64")
        tot, per = pl.coulomb_energy()
        ref = coulomb_energy(prob)
        assert abs(tot - ref) < 1e-12 * abs(ref)
        assert len(per) == 1 and per[0] == tot
    probs = [synth.config1_kirkwood_sphere(nu=4, seed=s) for s in (1, 2, 3)]
    pl = lib.Plan(lib.batch_problem(probs), lib.default_params(), "cuda:0")
    tot, per = pl.coulomb_energy()
    for k, p in enumerate(probs):
        assert abs(per[k] - coulomb_energy(p)) < 1e-12 * abs(coulomb_energy(p))


def test_born_pair_binding(gpu_lib):
    from paper_1309_4018_amd.binding import binding_energy

    a, d, kappa = 2.0, 20.0, 0.125
    c, r, l = synth.born_pair(d, radius=a, nu=8, kappa=kappa)
    ddg, parts = binding_energy(c, r, l, op="direct", precision="fp64", tol=1e-11)
    ref, rparts = oracle_binding(c, r, l, tol=1e-11)
    for k in ("complex", "receptor", "ligand"):
        assert abs(parts[k]["total"] - rparts[k][0]) < 1e-7 * abs(rparts[k][0])
    assert abs(ddg - ref) < 1e-5 * abs(ref) + 1e-9
    expect = -KE * math.exp(-kappa * (d - 2 * a)) / (80.0 * d * (1 + kappa * a) ** 2)
    assert abs(ddg / expect - 1.0) < 3e-3


def test_star_pair_binding_treecode(gpu_lib):
    from paper_1309_4018_amd.binding import binding_energy

    c, r, l = synth.star_pair(gap=3.0, nu_rec=8, nu_lig=6, n_rec=200, n_lig=60)
    ddg, parts = binding_energy(c, r, l, precision="fp32_refined", tol=1e-7, theta=0.5, P=8)
    ref, rparts = oracle_binding(c, r, l, tol=1e-10)
    scale = max(abs(rparts[k][0]) for k in rparts)
    for k in ("complex", "receptor", "ligand"):
        assert abs(parts[k]["total"] - rparts[k][0]) < 1e-4 * abs(rparts[k][0])
        assert abs(parts[k]["coulomb"] - rparts[k][2]) < 1e-12 * abs(rparts[k][2])
    assert abs(ddg - ref) < 2e-3 * scale


def test_refinement_study_born(gpu_lib):
    from paper_1309_4018_amd.binding import refinement_study

    probs = [synth.born_sphere(nu=nu) for nu in (4, 8, 16)]
    out = refinement_study(probs, op="direct", precision="fp64", tol=1e-10)
    exact = 0.5 * KE * (1 / 80.0 - 1 / 4.0) / 4.0
    assert 0.8 < out["order"] < 1.2
    assert abs(out["extrapolated"] - exact) < 1e-3 * abs(exact)
    assert abs(out["energies"][2] - exact) > abs(out["extrapolated"] - exact)
