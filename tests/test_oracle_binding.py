"""Pins of the oracle's Coulomb and binding energies (CPU).

Coulomb energy (Eq. total_energy; pairs within a region, that region's
permittivity): a hand-computed three-charge case, homogeneity of degree -1
in length, invariance under rigid motion, and no cross-region pairs.
Binding energy (Eq. bind_energy) of two Born ions whose centres are d apart:
the self energies cancel and what remains is their interaction through the
solvent, which to leading order in a/d is the Coulomb energy in the solvent,
-k_e q1 q2 / (eps_out d) for kappa = 0, and the screened form
k_e q1 q2 exp(-kappa (d - 2a)) / (eps_out d (1 + kappa a)^2) for kappa > 0
(each ion excludes the electrolyte from its sphere of radius a).
"""

import math

import numpy as np
import pytest

import synth
from oracle import KE
from oracle.energy import binding_energy, coulomb_energy


def _one_region(x, q, eps=4.0):
    v, f = synth.geodesic_sphere("oct", 2, 50.0)
    return synth.Problem([synth.Region(eps, 0.0), synth.Region(80.0, 0.0)],
                         [synth.Surface(v, f, 0, 1)], {0: (np.asarray(x), np.asarray(q))})


def test_three_charges_by_hand():
    s = 3.0
    x = np.array([[0.0, 0.0, 0.0], [s, 0.0, 0.0], [0.5 * s, 0.5 * math.sqrt(3.0) * s, 0.0]])
    q = np.array([1.0, -0.5, 0.25])
    # pairs: (1)(-0.5) + (1)(0.25) + (-0.5)(0.25) = -0.375, all at distance s
    expect = KE * (-0.375) / (4.0 * s)
    assert abs(coulomb_energy(_one_region(x, q)) - expect) < 1e-12 * abs(expect)


def test_homogeneity_and_rigid_motion():
    rng = np.random.default_rng(7)
    x = rng.normal(size=(40, 3)) * 5.0
    q = rng.normal(size=40)
    e = coulomb_energy(_one_region(x, q))
    assert abs(coulomb_energy(_one_region(2.5 * x, q)) - e / 2.5) < 1e-10 * abs(e)
    a = rng.normal(size=(3, 3))
    rot, _ = np.linalg.qr(a)
    moved = x @ rot.T + np.array([3.0, -7.0, 11.0])
    assert abs(coulomb_energy(_one_region(moved, q)) - e) < 1e-10 * abs(e)
    assert abs(coulomb_energy(_one_region(x, 2.0 * q)) - 4.0 * e) < 1e-10 * abs(e)


def test_regions_do_not_mix():
    c, r, l = synth.star_pair(nu_rec=6, nu_lig=4, n_rec=30, n_lig=10)
    ec, er, el = coulomb_energy(c), coulomb_energy(r), coulomb_energy(l)
    assert abs(ec - (er + el)) < 1e-10 * abs(ec)


@pytest.mark.parametrize("kappa,d", [(0.0, 20.0), (0.125, 20.0), (0.125, 30.0)])
def test_born_pair_binding(kappa, d):
    a, q1, q2 = 2.0, 1.0, -1.0
    c, r, l = synth.born_pair(d, radius=a, q=(q1, q2), nu=8, kappa=kappa)
    ddg, parts = binding_energy(c, r, l)
    if kappa == 0.0:
        expect = KE * q1 * q2 / (80.0 * d)
    else:
        expect = KE * q1 * q2 * math.exp(-kappa * (d - 2 * a)) / (80.0 * d * (1 + kappa * a) ** 2)
    assert abs(ddg / expect - 1.0) < 3e-3
    # one charge per region: no Coulomb term anywhere
    assert all(v[2] == 0.0 for v in parts.values())
