"""A single system of more than a million unknowns on the GPU.

A Born ion in a Debye-Hueckel solvent (radius 4 A, eps 4 / 80, kappa
0.125 / A) meshed with 528,392 panels (1,056,784 unknowns, more than 256
Krylov reduction chunks of 4,096 entries, so GMRES takes its unfused
Gram-Schmidt path).  The FP32-refined treecode solve must converge to the
tolerance and the energy must match the closed form (Born-DH) within the
discretisation and truncation error.
"""

import pytest

import synth
from oracle.closed_forms import born_dh

pytestmark = pytest.mark.gpu


def test_million_unknown_born_sphere(gpu_lib):
    from paper_1309_4018_amd import lib

    prob = synth.born_sphere(257, kappa=0.125)
    pl = lib.plan_for(prob, precision="fp32_refined", tol=1e-6, theta=0.5, P=6)
    assert pl.n_unknowns > 256 * 4096
    res = pl.solve()
    assert res["converged"] == 1
    assert res["final_rel_res"] <= 1e-6
    ref = born_dh(4.0, 4.0, 80.0, 0.125)
    assert abs(res["energy_kJmol"] - ref) < 5e-4 * abs(ref)
