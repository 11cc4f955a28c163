"""Pins of the oracle's assembled system, solve and energy.

* Closed forms among themselves: Kirkwood at one interface equals the
  concentric-sphere solve; the Kirkwood n = 0 term is Born / Born-DH; the
  k_n log derivative matches the Bessel recurrence.
* Born sphere: the paper's printed analytic energy, first-order convergence
  in panel area (Eq. observed_order) and the Richardson estimate.
* Born-DH: constant surface potential and normal derivative.
* Kirkwood sphere with kappa: energy and per-charge reaction potential.
* Multi-surface: concentric Stern layer and a concentric solvent-filled
  cavity converge to the layered closed form.
* GMRES: same solution as LU.
"""

import json
import math
import os

import numpy as np
import pytest
from scipy.special import spherical_kn

import synth
from oracle import Oracle, Params
from oracle import closed_forms as cf
from oracle.gmres import gmres
from oracle.refinement import observed_order, richardson

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_sphere.json")


def test_closed_forms_agree():
    xyz, q = synth.ball_charges(8, 3.0, 1, center_charge=1.0)
    for kappa in (0.0, 0.125):
        k1 = cf.kirkwood(4, 4, 80, kappa, xyz, q)
        k2 = cf.concentric([4.0], [4, 80], [0, kappa], 0, xyz, q)
        assert abs(k1 - k2) < 1e-11 * abs(k1)
    c = np.zeros((1, 3)), np.ones(1)
    assert abs(cf.kirkwood(4, 4, 80, 0.0, *c) - cf.born(4, 4, 80)) < 1e-12
    assert abs(cf.kirkwood(4, 4, 80, 0.125, *c) - cf.born_dh(4, 4, 80, 0.125)) < 1e-12
    assert abs(cf.concentric([4.0, 6.0], [4, 80, 80], [0, 0, 0.125], 0, *c)
               - cf.stern_central(4, 6, 4, 80, 0.125)) < 1e-11
    # log derivative of k_n against the recurrence k_n' = -k_{n-1} - (n+1)/x k_n
    x = 0.5
    for n in range(1, 8):
        g = -(n + 1) - x * spherical_kn(n - 1, x) / spherical_kn(n, x)
        assert abs(cf._log_deriv_k(n, x) - g) < 1e-12 * abs(g)
    # reaction potential of one charge reproduces the energy
    phi = cf.kirkwood_phi_reac(4, 4, 80, 0.125, xyz, q, xyz)
    e = 0.5 * 4 * math.pi * 1389.35458 * float(q @ phi)
    assert abs(e - cf.kirkwood(4, 4, 80, 0.125, xyz, q)) < 1e-10 * abs(e)


def test_paper_printed_born_value():
    g = json.load(open(GOLDEN))
    e = cf.born(g["radius"], g["eps_in"], g["eps_out"])
    assert abs(e - g["analytic_energy_kJmol"]) < 5e-5


@pytest.fixture(scope="module")
def born_series():
    out = {}
    for nu in (4, 8, 16):
        o = Oracle(synth.born_sphere(nu), Params(k=4))
        out[nu] = o.solve(tol=1e-10)
    return out


def test_born_convergence_order(born_series):
    g = json.load(open(GOLDEN))
    f3, f2, f1 = (born_series[nu].energy for nu in (4, 8, 16))
    exact = cf.born(4, 4, 80)
    errs = [abs(f - exact) for f in (f3, f2, f1)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] / abs(exact) < 5e-3
    # panel counts grow 4x per level: ratio r = 4 in mean panel area
    p = observed_order(f1, f2, f3, 4.0)
    assert abs(p - g["observed_order_vs_area_pygbe"]) < 0.05
    ext = richardson(f1, f2, 4.0, p)
    assert abs(ext - g["analytic_energy_kJmol"]) < 0.1 * errs[2]


def test_born_dh_surface_values():
    a, kappa = 4.0, 0.125
    o = Oracle(synth.born_sphere(16, kappa=kappa))
    s = o.solve(tol=1e-11)
    phi, psi = o.split(s.x)[0]
    phi_exact = 1.0 / (4 * math.pi * 80 * (1 + kappa * a) * a)
    psi_exact = -1.0 / (4 * math.pi * 4 * a * a)
    assert abs(phi.mean() - phi_exact) < 5e-3 * phi_exact
    assert abs(psi.mean() - psi_exact) < 5e-3 * abs(psi_exact)
    assert phi.std() < 5e-3 * phi_exact and psi.std() < 1e-2 * abs(psi_exact)
    exact = cf.born_dh(a, 4, 80, kappa)
    assert abs(s.energy - exact) < 5e-3 * abs(exact)


def test_kirkwood_config1():
    p = synth.config1_kirkwood_sphere()
    o = Oracle(p)
    s = o.solve(tol=1e-10)
    x, q, _ = p.all_charges()
    exact = cf.kirkwood(4, 4, 80, 0.125, x, q)
    assert abs(s.energy - exact) < 1e-2 * abs(exact)
    phi_k = cf.kirkwood_phi_reac(4, 4, 80, 0.125, x, q, x)
    assert np.max(np.abs(s.phi_reac - phi_k)) < 2e-2 * np.max(np.abs(phi_k))


def test_gmres_matches_lu():
    o = Oracle(synth.config1_kirkwood_sphere(nu=8))
    A, b = o.matrix(), o.rhs()
    x_lu = np.linalg.solve(A, b)
    for restart in (100, 7):
        x, hist = gmres(lambda v: A @ v, b, tol=1e-12, restart=restart, max_iter=2000)
        assert hist[-1] <= 1e-12
        assert np.linalg.norm(x - x_lu) < 1e-9 * np.linalg.norm(x_lu)
        # the implicit residual history tracks the true residual at the end
        assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) < 1e-11
    # a zero right-hand side is solved by x = 0 without iterations
    x0, h0 = gmres(lambda v: A @ v, np.zeros_like(b))
    assert not np.any(x0) and h0 == []


@pytest.mark.parametrize("case", ["stern", "cavity"])
def test_multisurface_concentric(case):
    xq = np.array([[0.0, 0.0, 2.8], [0.8, 2.0, -1.6], [-2.4, 0.8, 0.8]])
    qq = np.array([1.0, -0.5, 0.7])
    if case == "stern":
        radii, eps, kap, creg, xc = [4.0, 6.0], [4, 80, 80], [0, 0, 0.125], 0, xq
    else:
        radii, eps, kap, creg, xc = [2.0, 6.0], [80, 4, 80], [0, 0, 0.125], 1, xq * 1.25
    exact = cf.concentric(radii, eps, kap, creg, xc, qq)
    errs = []
    for nu in (4, 8):
        p = synth.concentric_spheres(radii, eps, kap, (xc, qq), creg, nu=nu)
        errs.append(abs(Oracle(p).solve(tol=1e-10).energy - exact))
    assert errs[1] < errs[0] / 3.0
    assert errs[1] < 0.025 * abs(exact)


def test_ion_holding_cavity_concentric():
    """A cavity holding ions inside its own Stern layer (linearized PB in the
    cavity): ionic ball r < 2.5, Stern shell to 4, protein shell to 9 with
    the charges, Stern to 11, solvent.  The Richardson estimate from oct
    nu = 4 and 8 (first order in panel area, panel ratio 4) matches the
    layered closed form, and is much closer to it than to the same system
    without ions in the cavity."""
    xq = np.array([[0.0, 0.0, 2.8], [0.8, 2.0, -1.6], [-2.4, 0.8, 0.8]]) * 2.3
    qq = np.array([1.0, -0.5, 0.7])
    radii, eps, kap = [2.5, 4.0, 9.0, 11.0], [80, 80, 4, 80, 80], [0.125, 0, 0, 0, 0.125]
    exact = cf.concentric(radii, eps, kap, 2, xq, qq)
    no_ions = cf.concentric(radii, eps, [0, 0, 0, 0, 0.125], 2, xq, qq)
    e = {nu: Oracle(synth.concentric_spheres(radii, eps, kap, (xq, qq), 2, nu=nu))
         .solve(tol=1e-10).energy for nu in (4, 8)}
    ext = richardson(e[8], e[4], 4.0, 1.0)
    assert abs(e[8] - exact) < abs(e[4] - exact) / 3.0
    assert abs(ext - exact) < 3e-3 * abs(exact)
    assert abs(ext - no_ions) > 3.0 * abs(ext - exact)


@pytest.mark.parametrize("which", ["sphere", "three_region"])
def test_apply_rows_equals_assembled_rows(which):
    """Oracle.apply_rows (the matrix-free rows used at sizes too large to
    assemble) against the same rows of the assembled matrix (Eq. matrix and
    its multi-surface form): every surface, both row halves, random rows."""
    if which == "sphere":
        prob = synth.config1_kirkwood_sphere(nu=8)
    else:
        prob = synth.config3_multisurface(nu=4, cav_nu=2, n_charges=40)
    o = Oracle(prob)
    A = o.matrix()
    rng = np.random.default_rng(11)
    x = rng.normal(size=o.n)
    y = A @ x
    for t, nt in enumerate(o.ns):
        rows = rng.choice(nt, size=min(nt, 17), replace=False)
        halves = o.apply_rows(x, t, rows)
        assert len(halves) == 2
        for half, yr in enumerate(halves):
            ref = y[o.uoff[t] + half * nt + rows]
            assert np.max(np.abs(yr - ref)) < 1e-13 * np.max(np.abs(y)), (t, half)
