"""Pins of the gradient oracle.

* Central finite differences (h = 1e-4) of the oracle's own energy with
  respect to charges, kappa and every eps.
* Born-DH closed-form derivatives dG/dkappa and dG/deps_out.
* Reciprocity: dG/dq_k tends to 4 pi k_e phi_reac(x_k) as the mesh refines.
"""

import copy
import math

import numpy as np

import synth
from oracle import Oracle
from oracle import closed_forms as cf
from oracle.adjoint import C_ENERGY, gradients


def _energy(p):
    o = Oracle(p)
    x = np.linalg.solve(o.matrix(), o.rhs())
    return 0.5 * C_ENERGY * float(o.q @ (o.reaction_matrix() @ x))


def _stern_problem(nu=4):
    xq = np.array([[0.0, 0.0, 2.5], [1.0, 1.5, -1.0], [-2.0, 1.0, 1.0]])
    qq = np.array([1.0, -0.5, 0.7])
    return synth.concentric_spheres([4.0, 5.0], [4, 80, 80], [0, 0, 0.125], (xq, qq), 0, nu=nu)


def test_gradients_vs_central_fd():
    p = _stern_problem()
    g = gradients(Oracle(p))
    h = 1e-4
    for k in range(3):
        pp, pm = copy.deepcopy(p), copy.deepcopy(p)
        for pr, sg in ((pp, 1), (pm, -1)):
            x, q = pr.charges[0]
            q = q.copy()
            q[k] += sg * h
            pr.charges[0] = (x, q)
        fd = (_energy(pp) - _energy(pm)) / (2 * h)
        assert abs(g["dE_dq"][k] - fd) < 1e-7 * abs(fd)
    pp, pm = copy.deepcopy(p), copy.deepcopy(p)
    pp.regions[2].kappa += h
    pm.regions[2].kappa -= h
    fd = (_energy(pp) - _energy(pm)) / (2 * h)
    assert abs(g["dE_dkappa"][2] - fd) < 1e-6 * abs(fd)
    for r in range(3):
        pp, pm = copy.deepcopy(p), copy.deepcopy(p)
        pp.regions[r].eps += h
        pm.regions[r].eps -= h
        fd = (_energy(pp) - _energy(pm)) / (2 * h)
        assert abs(g["dE_deps"][r] - fd) < 1e-6 * abs(fd) + 1e-10


def test_gradients_born_dh_closed_form():
    a, kappa = 4.0, 0.125
    p = synth.born_sphere(8, kappa=kappa)
    g = gradients(Oracle(p))
    dk = cf.born_dh_dkappa(a, 4, 80, kappa)
    de = cf.born_dh_deps_out(a, 4, 80, kappa)
    assert abs(g["dE_dkappa"][1] - dk) < 2e-2 * abs(dk)
    assert abs(g["dE_deps"][1] - de) < 2e-2 * abs(de)
    # energy is quadratic in q: dG/dq = 2 G / q for a single charge
    assert abs(g["dE_dq"][0] - 2.0 * g["energy"]) < 1e-9 * abs(g["energy"])


def test_reciprocity_improves_with_refinement():
    gaps = []
    for nu in (4, 8):
        p = synth.config1_kirkwood_sphere(nu=nu)
        o = Oracle(p)
        g = gradients(o)
        phi = o.reaction_matrix() @ g["x"]
        gaps.append(np.max(np.abs(g["dE_dq"] - C_ENERGY * phi)) / np.max(np.abs(g["dE_dq"])))
    assert gaps[1] < gaps[0]
    assert gaps[1] < 0.05
